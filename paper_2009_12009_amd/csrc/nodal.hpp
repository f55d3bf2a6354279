// Node-centred finite-element solve: device layouts and kernel launchers.
//
// One level = one array per quantity over the level's unknown nodes, padded
// by one ghost node on every side (x fastest).  Along a Dirichlet direction
// the unknowns are the interior nodes 1 .. n-1 and the ghosts are the wall
// nodes (always 0); along a periodic direction the unknowns are nodes
// 0 .. n-1 and the ghosts hold wrapped copies.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace amrmg {

struct NdGeo {
  int mx, my, mz;  // unknowns per direction
  int px, py;      // padded pitches: mx + 2, my + 2
  int per;         // bit d: periodic along d
  int tz;          // planes a work-group marches (level-wise launch depth)
};

// The 14 stored couplings of a coarse node (offsets >= 0 in (z, y, x)
// lexicographic order, the centre first); the other 13 are read mirrored
// from the neighbour: coupling (u, u - o) = stored (u - o, o).
constexpr int kNdStored = 14;
struct NdStencil {
  double* w[kNdStored];
};
struct NdStencilC {
  const double* w[kNdStored];
};

// Cell stiffness of the finest level divided by the cell volume, indexed by
// the pattern of differing coordinates of the two corners (bit d set = the
// corners differ along d).
struct NdKappa {
  double k[8];
};

// Per box of the caller's nodal MultiFab: cell box lo..hi, nodes lo - ng ..
// hi + 1 + ng, element offset of the box's array.
struct NdBox {
  int lo[3], hi[3];
  long long off;
};

enum { ND_JACOBI = 0, ND_ZERO = 1, ND_RESID = 2, ND_APPLY = 3 };

// Finest level (operator from the cell coefficient): mode ND_JACOBI out =
// phi + omega (f - A phi) / diag; ND_ZERO out = omega f / diag (phi not read);
// ND_RESID out = f - A phi.  norm (nullable): max |f - A phi| folded in as
// IEEE bits (NaN-propagating), one of kNdNormWays words per work-group;
// ND_APPLY out = A phi.
hipError_t nd_launch_sweep0(hipStream_t st, const NdGeo& g, const NdKappa& k, const double* sig,
                            const double* phi, const double* f, double* out, double omega,
                            int mode, unsigned long long* norm);
// Coarse levels (stored couplings).
hipError_t nd_launch_sweep_st(hipStream_t st, const NdGeo& g, const NdStencilC& s,
                              const double* phi, const double* f, double* out, double omega,
                              int mode, unsigned long long* norm);
// Full-weighting restriction rc = P^T rf / 8 (fine residual ghosts not read).
hipError_t nd_launch_restrict(hipStream_t st, const NdGeo& gf, const NdGeo& gc, const double* rf,
                              double* rc);
// phi_f += P e_c (trilinear; e_c ghosts not read).
hipError_t nd_launch_interp_add(hipStream_t st, const NdGeo& gf, const NdGeo& gc,
                                const double* ec, double* phif);
// Wrapped copies into the ghosts of the periodic directions (walls untouched).
hipError_t nd_launch_fill_ghosts(hipStream_t st, const NdGeo& g, double* a);
// Galerkin coarse operator R A P of the finest level (from sigma) or of a
// stored-coupling level; writes the coarse level's 14 arrays (valid nodes).
hipError_t nd_launch_rap0(hipStream_t st, const NdGeo& gf, const NdGeo& gc, const NdKappa& k,
                          const double* sig, const NdStencil& out);
hipError_t nd_launch_rap(hipStream_t st, const NdGeo& gf, const NdGeo& gc, const NdStencilC& in,
                         const NdStencil& out);
// CG from zero on the bottom level, one work-group; work: 4 arrays of the
// level's padded size.  iters (device int) receives the iteration count.
hipError_t nd_launch_bottom_cg(hipStream_t st, const NdGeo& g, const NdStencilC& s,
                               const double* rhs, double* x, double* work, double tol, int maxit,
                               int singular, int* iters);
// max |v| over the valid nodes.
hipError_t nd_launch_maxabs(hipStream_t st, const NdGeo& g, const double* v,
                            unsigned long long* norm);
// Caller's nodal MultiFab <-> level-0 array.  gather: every unknown node from
// the box that holds the cell with the same index; scatter: every node of
// every box array (ghosts included) inside the domain's node range, walls 0.
hipError_t nd_launch_gather(hipStream_t st, const NdGeo& g, const NdBox* boxes, int nbox,
                            int maxnodes, int ng, const int dom_lo[3], const double* src,
                            double* dst);
hipError_t nd_launch_scatter(hipStream_t st, const NdGeo& g, const NdBox* boxes, int nbox,
                             int maxnodes, int ng, const int dom_lo[3], const int dom_n[3],
                             const double* src, double* dst);
// Cell MultiFab (ng 0) -> sigma array of the finest level ((mx+1)(my+1)(mz+1):
// node u reads cells u + s, s in {0,1}^3; along a periodic direction entry c
// holds cell c - 1, wrapped).
hipError_t nd_launch_sigma(hipStream_t st, const NdGeo& g, const NdBox* boxes, int nbox,
                           int maxcells, const int dom_lo[3], const int dom_n[3],
                           const double* cells, double* sig);
// The mean of the valid nodes taken out of v (part: nd_sum_partials_count
// doubles of scratch).
int nd_sum_partials_count(const NdGeo& g);
hipError_t nd_launch_remove_mean(hipStream_t st, const NdGeo& g, double* v, double* part);
// Krylov vector work on the valid nodes (scalars stay on the device):
// out = a.b (part: nd_sum_partials_count doubles of scratch); p = z or
// z + (rho / rho_old) p; x += alpha p, r -= alpha q with alpha = rho / pq and
// max |r| folded into norm.
hipError_t nd_launch_dot(hipStream_t st, const NdGeo& g, const double* a, const double* b,
                         double* part, double* out);
hipError_t nd_launch_cg_p(hipStream_t st, const NdGeo& g, double* p, const double* z,
                          const double* rho, const double* rho_old, int restart);
hipError_t nd_launch_cg_xr(hipStream_t st, const NdGeo& g, double* x, const double* p, double* r,
                           const double* q, const double* rho, const double* pq,
                           unsigned long long* norm);
hipError_t nd_launch_fill(hipStream_t st, double* a, long long n, double v);
hipError_t nd_launch_fill_u64(hipStream_t st, unsigned long long* a, int n,
                              unsigned long long v);

constexpr int kNdNormWays = 64;
constexpr int kNdNormStride = 16;
constexpr int kNdNormSlot = kNdNormWays * kNdNormStride;

}  // namespace amrmg
