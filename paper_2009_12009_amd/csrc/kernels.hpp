// Launchers of the gfx950 kernels.  Every launcher enqueues on the given
// stream and returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime_api.h>

#include "tables.hpp"

namespace amrmg {

// The operator's data on one level: box table and coefficients.  The face
// coefficient of the operator is c_f = (beta * b_f) * inv_h2[d].
template <typename T>
struct StencilArgs {
  const BoxInfo* boxes;
  const T* a;   // cell coefficient (ghost-free layout) or null for a = 1
  const T* b0;  // face coefficients, ghost-free face layouts
  const T* b1;
  const T* b2;
  T alpha, beta;
  T ih0, ih1, ih2;  // 1 / h_d^2
  // every array of every box of the level spans < 4 GiB (buffer
  // descriptors with 32-bit offsets work) and a half-sweep's arrays exceed
  // the last-level cache (read-once loads may carry the non-temporal hint)
  int buf = 0;
};

// A max-norm slot: kNormWays words kNormStride apart (one per 128-byte line);
// work-group b folds its maximum into way b % kNormWays, and the slot's norm
// is the largest of its ways.  Clearing a slot clears all kNormSlot words.
constexpr int kNormWays = 64;
constexpr int kNormStride = 16;
constexpr int kNormSlot = kNormWays * kNormStride;

// Launch shape of a tiled kernel: block (lx, ly), each block marching tz
// planes, u planes gathered per step (smoother and residual only).
struct Shape {
  int lx, ly, tz;
  int u = 1;
  // smoother lane mapping: 0 = one x-pair per lane, 1 = the same storing
  // whole x-pairs (see k_gsrb), 2 = one x-quad per lane, two cells of the
  // colour (FP32 streaming levels, see k_gsrb_quad)
  int wp = 0;
};

// x cells a smoother tile row covers (2 or 4 per lane)
inline int gsrb_tx(Shape sh) { return (sh.wp == 2 ? 4 : 2) * sh.lx; }

// Red/black Gauss-Seidel half-sweep over every box: lane (x, y) of a block
// updates the cell of colour `colour` among tile cells x0+2x, x0+2x+1 on row
// y0+y, marching z over tz planes.  zero_guess: phi is taken as 0 (nothing
// but rhs is read).  rhs_ng: 0 or 1.  With wtb/wte (non-null) every update
// is also written into the face ghosts that mirror the cell, so face ghosts
// stay current across half-sweeps without an exchange.  With ec (non-null;
// needs wtb, no zero guess) the half-sweep also performs the interpolation
// phi += P ec of the coarse correction ec (cell data with 1 ghost of the
// boxes cinfo, every phi box's parent): each other-colour value read gets
// its parent's correction added; only cells of `colour` are stored, so the
// other colour is left without the correction and must be overwritten (the
// next half-sweep) before anything reads it.  phi's face ghosts must be
// current without the correction, ec's face ghosts current.
// With rf (zero_guess only, rhs_ng 0): the level's right-hand side is first
// restricted here, rout = R rf, from the finer level's residual rf (no
// ghosts) on boxes finfo, box b of this level being the coarsening of finer
// box b; each lane stores both cells of its x-pair and smooths with the
// active one.  rhs is then not read.
template <typename T>
hipError_t launch_gsrb(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                       const StencilArgs<T>& op, T* phi, const T* rhs, int rhs_ng, int colour,
                       int zero_guess, const WtBox* wtb = nullptr, const WtEntry* wte = nullptr,
                       const BoxInfo* cinfo = nullptr, const T* ec = nullptr,
                       const BoxInfo* finfo = nullptr, const T* rf = nullptr, T* rout = nullptr);

// One full red/black sweep, both colours in one pass, out of place: pout
// receives the result of a red half-sweep followed by a black half-sweep of
// pin, except the black cells on each box's boundary layer (which need the
// neighbouring boxes' new red values); those get their old value and are
// finished by launch_rim after a ghost exchange of pout.  pin's ghosts must
// hold the neighbours' values (not read when zero_guess: pin taken as 0).
// A block of (lx/2)*ly lanes takes an lx x ly x tz tile of one box and
// marches along z, staging pin planes and new red values in LDS and
// recomputing the red cells of a one-cell ring around the tile.  When
// normbits is non-null, max |rhs - A pin| over the tile's cells is folded
// into *normbits (the residual of the state before the sweep).
template <typename T>
hipError_t launch_sweep(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const StencilArgs<T>& op, const T* pin, T* pout, const T* rhs,
                        int rhs_ng, int zero_guess, unsigned long long* normbits);
// LDS bytes of one launch_sweep block (0 when the shape is not supported).
size_t sweep_lds_bytes(Shape sh, size_t elem);

// Black half-sweep restricted to the cells of the rim tiles (in place).
template <typename T>
hipError_t launch_rim(hipStream_t st, const RimTile* tiles, int ntiles, const StencilArgs<T>& op,
                      T* phi, const T* rhs, int rhs_ng);

// With dot_partials, partials[tile] = sum over the tile of phi * out (the
// product computed before out is rounded to TO), for launch_sum_final.
// out = rhs - A phi (mode 0) or out = A phi (mode 1) on every valid cell, one
// lane per cell; out may be null (norm only).  When normbits is non-null the
// max |out| is folded into *normbits as IEEE-754 bits (NaN-propagating).
// out uses the ghost-free layout; TO may be narrower than T (the value is
// computed in T and rounded once).  With pnext (mode 0, TO = T, pnext !=
// phi) the launch also writes phi after a red half-sweep into pnext's valid
// cells (red cells updated with the half-sweep's expression, black cells
// copied), so that a stop test's residual and the next cycle's first
// half-sweep share one pass over the level.  pnext's ghosts are written only
// with the level's write-through tables (wtb, wte; both or neither): then
// each new red value reaches the face ghosts that mirror it (black ghosts
// are left, the next half-sweep being black).
template <typename T, typename TO>
hipError_t launch_residual(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                           const StencilArgs<T>& op, const T* phi, const T* rhs, int rhs_ng,
                           TO* out, unsigned long long* normbits, int mode,
                           double* dot_partials = nullptr, T* pnext = nullptr,
                           const WtBox* wtb = nullptr, const WtEntry* wte = nullptr);

// max |v| over valid cells folded into *normbits (v: ng 0 or 1 layout).
template <typename T>
hipError_t launch_maxabs(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                         const BoxInfo* boxes, const T* v, int ng, unsigned long long* normbits);

// Coarse value = mean of the 8 children (pairwise sum).  Tiles cover the
// coarse cells of each fine box; fine r is ghost-free, coarse rhs ghost-free.
template <typename T>
hipError_t launch_restrict(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                           const BoxInfo* fine, const BoxInfo* coarse, const T* rf, T* rc);

// rc = R (rhs - A phi): the residual pass and the restriction in one pass
// (the fine residual is not stored; same bits in rc).  Tiles of lx x ly
// lanes (lx, ly even, lx*ly <= 256) and tz planes (even), starting at even
// cells of boxes with even extents; cinfo: the coarse boxes (each fine box's
// parent), rc without ghosts.
template <typename T>
hipError_t launch_resid_restrict(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                                 const StencilArgs<T>& op, const T* phi, const T* rhs, int rhs_ng,
                                 const BoxInfo* cinfo, T* rc);

// Fine valid cell += parent coarse value; both with one ghost layer.
template <typename T>
hipError_t launch_prolong_add(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                              const BoxInfo* fine, const BoxInfo* coarse, T* ef, const T* ec);

// phi (double, ng 1) += e (float, ng 1) on valid cells.
hipError_t launch_update(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                         const BoxInfo* boxes, double* phi, const float* e);

// dst = src on valid cells (layouts with ng 0 or 1).
hipError_t launch_copy_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, const double* src, int src_ng, double* dst,
                             int dst_ng);

// v = 0 on valid cells (layout ng).
template <typename T>
hipError_t launch_zero_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, T* v, int ng);

// Deterministic sum of v (layout ng 0 or 1) over valid cells: one partial per
// tile into partials[ntiles], then one work-group adds them in order into
// *sum.  Then v -= *sum / ncell on valid cells.
hipError_t launch_sum_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                            const BoxInfo* boxes, const double* v, int ng, double* partials,
                            double* sum);
hipError_t launch_shift_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                              const BoxInfo* boxes, double* v, int ng, const double* sum,
                              long long ncell);

// Deterministic *out = sum over valid cells of a*b (layouts ang, bng in {0, 1}),
// partials as in launch_sum_valid.
hipError_t launch_dot(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                      const BoxInfo* boxes, const double* a, int ang, const double* b, int bng,
                      double* partials, double* out);
// Conjugate-gradient steps with device scalars: x (ng 1) += alpha p (ng 1),
// r (ng 0) -= alpha q (ng 0), alpha = *num / *den, max |r| into *normbits;
// and p (ng 1) = z (first) or z + (*num / *den) p.
// With r32 (non-null) the new r is also stored rounded to FP32 (ng 0).
hipError_t launch_cg_xr(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const BoxInfo* boxes, double* x, const double* p, double* r,
                        const double* q, const double* num, const double* den,
                        unsigned long long* normbits, float* r32 = nullptr);
// Krylov basis on one level (ghost-free vectors; vector q at V + q*vstride):
// partials[q*pstride + poff + tile] = tile part of w.V_q for q < n;
// out[q] = ordered sum of row q (n partials per row);
// out = sign*w - sum_q (sign*dots[q]) V_q with partials[poff + tile] of out.out;
// v = w / sqrt(*ss); phi (ng 1) += sum_q y[q] Z_q (ng 1, stride zstride).
hipError_t launch_mdot(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                       const BoxInfo* boxes, const double* w, const double* V, long long vstride,
                       int n, double* partials, int pstride, int poff);
hipError_t launch_sum_rows(hipStream_t st, const double* partials, int rows, int n, double* out);
hipError_t launch_maxpy(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const BoxInfo* boxes, const double* w, const double* V, long long vstride,
                        int n, const double* dots, double sign, double* out, double* partials,
                        int poff);
hipError_t launch_vnormalise(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, const double* w, double* v, const double* ss);
hipError_t launch_zaxpy(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const BoxInfo* boxes, double* phi, const double* Z, long long zstride,
                        int n, const double* y);
// *out = partials[0] + ... + partials[n-1] in a fixed order (one work-group).
hipError_t launch_sum_final(hipStream_t st, const double* partials, int n, double* out);
// z (FP64, ng 1) = e (FP32, ng 1) on valid cells and *out = sum r*z (r ng 0).
hipError_t launch_widen_dot(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                            const BoxInfo* boxes, const float* e, double* z, const double* r,
                            double* partials, double* out);
hipError_t launch_cg_p(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                       const BoxInfo* boxes, double* p, const double* z, const double* num,
                       const double* den, int first);

// Ghost exchange: every chunk copies FB_CHUNK cells of one tag, ncomp comps.
template <typename T>
hipError_t launch_fill_boundary(hipStream_t st, const FbTag* tags, const FbChunk* chunks,
                                int nchunks, T* data, int ncomp);

// Plain element-wise helpers over n elements.
hipError_t launch_fill_u64(hipStream_t st, unsigned long long* p, int n, unsigned long long v);

// Size of the static device scratch of the allocation-free ghost exchange,
// and its address on the current device (looked up once per device).
constexpr size_t kFbScratchBytes = size_t(4) << 20;
hipError_t fb_scratch_address(void** ptr);
template <typename TI, typename TO>
hipError_t launch_convert(hipStream_t st, const TI* in, TO* out, long long n);
// out = in over n16 16-byte elements (both 16-byte aligned), one per lane.
hipError_t launch_stream_copy(hipStream_t st, const void* in, void* out, long long n16);
hipError_t launch_scale_faces(hipStream_t st, const double* in, double* out, long long n,
                              double v_if_null);

// Level coefficients from a coarser copy of the next finer level.
template <typename T>
hipError_t launch_coarsen_cell(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                               const BoxInfo* fine, const BoxInfo* coarse, const T* af, T* ac);
hipError_t launch_coarsen_face(hipStream_t st, const BoxInfo* fine, int nbox_fine,
                               const BoxInfo* coarse, int d, const double* bf, double* bc,
                               int max_faces_per_box);

// Global face / cell arrays (x fastest over the domain) -> per-box arrays.
hipError_t launch_scatter_faces(hipStream_t st, const BoxInfo* boxes, int nbox, int d,
                                const int dom_lo[3], const int dom_n[3], const double* g,
                                double* out, int is_log, int max_faces_per_box);
hipError_t launch_scatter_cells(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                                const BoxInfo* boxes, const int dom_lo[3], const int dom_n[3],
                                const double* g, double* out);

// Adjoint face gradient: per box face array (mode 0) or global face array
// (mode 1, each physical face once).
hipError_t launch_face_grad(hipStream_t st, int nbox, const StencilArgs<double>& op,
                            const double* phi, const double* lam, double* const out[3], int mode,
                            const int dom_lo[3], const int dom_n[3], int perbits,
                            const int max_n[3]);

// Two-level composite pieces.
// Covered coarse cells (ghost layer cng) = mean of their 8 fine children (fine
// ghost layer fng), or 0 when zero_only; tiles = coarse cells of each fine box.
template <typename T>
hipError_t launch_avgdown(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                          const BoxInfo* fine, const BoxInfo* coarse, const T* f, int fng, T* c,
                          int cng, int zero_only);
// Fine ghosts from coarse values (one lane per CfGhost).
template <typename T>
hipError_t launch_cf_ghost(hipStream_t st, const CfGhost* g, int n, const T* coarse, T* fine);
// Coarse residual at coarse/fine faces: r += c (phi_I - phi_J) - mean fine flux / h_c,
// ihc[d] = 1/h_c^2, ihf[d] = 1/(h_f h_c).
template <typename T>
hipError_t launch_cf_reflux(hipStream_t st, const CfCell* cells, int ncell, const CfFace* faces,
                            const T* phic, const T* phif, const T* bc0, const T* bc1,
                            const T* bc2, const T* bf0, const T* bf1, const T* bf2, double beta,
                            const double ihc[3], const double ihf[3], T* r);
// v += w on valid cells (both ghost layer 1).
hipError_t launch_axpy_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, double* v, const double* w);

// Bottom solve: CG on a gathered copy of the bottom level (one work-group).
struct BottomTables {
  int n;                 // cells
  const int* nbr;        // [6*n] neighbour cell or -1 (wall), face-major
  const int* fidx;       // [6*n] element index of the face in the level's b_d
  const int* aidx;       // [n] element index of the cell in the level's a (ng 0)
  const int* map_rhs;    // [n] element index in the rhs MultiFab (ng 0)
  const int* map_out;    // [n] element index in the output MultiFab (ng 1)
};
template <typename T>
hipError_t launch_bottom_setup(hipStream_t st, const BottomTables& bt, const StencilArgs<T>& op,
                               T* diag, T* coef);
template <typename T>
hipError_t launch_bottom_cg(hipStream_t st, const BottomTables& bt, const T* diag, const T* coef,
                            const T* rhs, T* out, int accumulate, T* work, double tol,
                            int maxiter, int singular, int* iters_out);
// BiCGStab instead of CG (same arguments; work holds 7 n values).
template <typename T>
hipError_t launch_bottom_bicgstab(hipStream_t st, const BottomTables& bt, const T* diag,
                                  const T* coef, const T* rhs, T* out, int accumulate, T* work,
                                  double tol, int maxiter, int singular, int* iters_out);

// The coarsest levels of a V-cycle in one launch of one work-group
// (launch_tail): the levels from some level down to a CG bottom, every pass
// a loop of the work-group's lanes over the level's cells with a barrier
// after it, the arrays staying in the L2 cache between passes.  Each cell
// gets the arithmetic of the per-level kernels (the same operator, update,
// restriction and interpolation expressions, and the bottom's CG with the
// same lane layout and summation order), so the result is the one of the
// launches it replaces.
// A cell entry packs box-local coordinates and the box:
// kl | jl << 6 | il << 12 | box << 18 (box extents <= 64, < 2^14 boxes).
// A restriction entry packs a coarse cell's offset from coarsen(fine box)'s
// low corner the same way, with the fine box in the top bits.
constexpr int kTailMaxLevels = 6;
constexpr int kTailLanes = 1024;
constexpr int kTailMaxBottom = 1024;  // bottom cells (one per lane)
constexpr int kTailMaxExtent = 64;
constexpr int kTailMaxBoxes = 1 << 14;
// LDS of the tail kernel: the bottom CG's p, every box table it stages
constexpr size_t kTailMaxLds = 60 * 1024;

template <typename T>
struct TailLevel {
  StencilArgs<T> op;
  T* e;    // correction, one ghost layer (face ghosts kept by write-through)
  T* rhs;  // no ghosts
  T* r;    // residual, no ghosts
  const WtBox* wtb;
  const WtEntry* wte;
  const unsigned* cells;  // red cells [0, nred), black cells [nred, ncell)
  int nred, ncell;
  int nbox;
  const unsigned* rcells;  // restriction of r into the next coarser level
  int nrc;
  const BoxInfo* cinfo;  // the next coarser level's boxes (parents)
};

template <typename T>
struct TailPlan {
  int nlev;  // smoothed levels; the bottom level follows the last of them
  int nu1, nu2;
  int reverse;  // post-smoothing black before red
  // restriction of the residual of the level above the tail into the first
  // tail level's right-hand side
  const T* rf;
  const BoxInfo* finfo;
  int fnbox;
  const unsigned* rcells;
  int nrc;
  TailLevel<T> lev[kTailMaxLevels];
  const BoxInfo* binfo;  // the bottom level's boxes
  int bnbox;
  // LDS byte offsets of the staged box tables (the CG's p at 0): BoxInfo of
  // the level above, of tail level l (l = nlev: the bottom), WtBox of tail
  // level l; lds_bytes in all
  int lds_fi;
  int lds_bi[kTailMaxLevels + 1];
  int lds_wb[kTailMaxLevels];
  int lds_bytes;
  // bottom: CG from zero on bt (bt.n <= kTailMaxBottom) into be (ng 1)
  BottomTables bt;
  const T* bdiag;
  const T* bcoef;
  T* be;
  T* brhs;
  double tol;
  int maxiter, singular;
  int* iters;
};

// One launch of kTailLanes lanes: restrict rf, then per level nu1 sweeps
// (the first from zero), residual, restriction; the bottom CG; then per
// level upward the interpolation of the coarser correction and nu2 sweeps.
// plan: device copy (read only); nbottom = plan->bt.n; lds = plan->lds_bytes
// (<= kTailMaxLds).
template <typename T>
hipError_t launch_tail(hipStream_t st, const TailPlan<T>* plan, int nbottom, size_t lds);

}  // namespace amrmg
