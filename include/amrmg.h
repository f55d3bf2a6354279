/*
 * amrmg.h - C ABI of the MI355X (gfx950) multigrid library.
 *
 * The library solves the cell-centred variable-coefficient equation of the
 * AMReX paper's "Linear Solvers" section,
 *
 *     alpha * a * phi - beta * div(b grad phi) = f,
 *
 * with scalars alpha, beta, a cell coefficient a and a face coefficient b,
 * on one level held as a MultiFab: a list of non-intersecting boxes, each
 * with its own array grown by ngrow ghost cells ("Basic data structures",
 * "Containers for mesh data").  The solver is a geometric multigrid V-cycle
 * with a CG bottom solve ("Linear Solvers"); ghost cells between boxes are
 * filled by a fused copy ("Operations on a level", "Communication").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: 0 on success, a negative mg_status_t on failure.  No entry
 *   point aborts or exits.  mg_last_error() returns a message for the last
 *   failure on the calling thread.
 * - Boxes hold inclusive cell indices.  Domain = the geometry's box; the
 *   physical domain is [prob_lo, prob_hi] and h_d = (prob_hi_d - prob_lo_d) / n_d.
 * - MultiFab layout: box b's array covers grow(box_b, ngrow) (grown by one
 *   more cell along d when ixtype[d] = 1, face data) and starts at element
 *   offsets[b] of `data`; inside it cell (i, j, k) is at
 *   (i - glo_x) + nx * ((j - glo_y) + ny * (k - glo_z)) over the grown box
 *   (x fastest, "Fortran" order); components follow one another (struct of
 *   arrays).  The solver requires the canonical packing: offsets[0] = 0 and
 *   each box directly after the previous one.
 * - Device pointers: `data` of an mg_multifab_t, the workspace and the
 *   global face arrays are device memory on the current HIP device.  Boxes,
 *   offsets, geometries, options and info structs are host memory.
 * - Ownership: the caller owns every buffer it passes.  The solver copies
 *   coefficients into its workspace, keeps host-side metadata (plans, tile
 *   tables, graphs) until mg_destroy, and never allocates device memory: all
 *   its device storage lives in the caller's workspace, which must outlive
 *   the handle.  fill_boundary keeps a process-wide cache of exchange plans;
 *   each cached plan holds one small device table (released by
 *   mg_release_caches).
 * - Streams: work is enqueued on the stream given (NULL = the default
 *   stream).  mg_solve returns after its result is complete; fill_boundary,
 *   mg_apply and mg_face_grad_logb are asynchronous with respect to the host.
 * - Threading: one handle per thread; handles may be used from different
 *   threads concurrently.
 */
#ifndef AMRMG_H
#define AMRMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MG_OK = 0,
  MG_ERR_ARG = -1,               /* bad argument (null pointer, bad enum, size)          */
  MG_ERR_INVALID_BOXARRAY = -2,  /* overlap, outside the domain, incomplete cover,
                                    not coarsenable                                     */
  MG_ERR_MISMATCH = -3,          /* a MultiFab does not match the solver's boxes/layout */
  MG_ERR_WORKSPACE = -4,         /* workspace missing or smaller than required           */
  MG_ERR_HIP = -5,               /* a HIP runtime call failed                            */
  MG_ERR_NAN = -6,               /* a non-finite value reached a norm                    */
  MG_ERR_DIVERGED = -7,          /* residual grew for 3 cycles and exceeds its start     */
  MG_ERR_NOT_CONVERGED = -8,     /* max_iter reached; phi and info still written         */
  MG_ERR_SINGULAR = -9           /* all-periodic, alpha*a == 0 and rhs of nonzero mean   */
} mg_status_t;

enum { MG_BC_PERIODIC = 0, MG_BC_DIRICHLET0 = 1 };   /* "BCRec" subset: periodic, phi = 0 wall */
enum { MG_F64 = 0, MG_F32 = 1 };                      /* element type of a MultiFab          */
enum { MG_PREC_F64 = 0, MG_PREC_F32_REFINE = 1 };     /* solve precision                     */

/* A rectangular range of cells, inclusive ("Box"). */
typedef struct { int32_t lo[3], hi[3]; } mg_box_t;

/* Index <-> physical mapping and periodicity ("Geometry"). */
typedef struct {
  mg_box_t domain;
  double prob_lo[3], prob_hi[3];
  int32_t is_periodic[3];
} mg_geom_t;

/* Borrowed view of one level's data ("FabArray"/"MultiFab" + "Array4"). */
typedef struct {
  int32_t nbox;
  const mg_box_t* boxes;       /* host: valid boxes, cell index space          */
  int32_t ngrow;               /* ghost layers on every side                    */
  int32_t ncomp;               /* components (the solver uses 1)                */
  int32_t ixtype[3];           /* 0 = cell centred, 1 = face (nodal) along d    */
  int32_t dtype;               /* MG_F64 | MG_F32                               */
  void* data;                  /* device                                        */
  const int64_t* offsets;      /* host [nbox]: element offset of each box       */
} mg_multifab_t;

/* Solver options.  mg_default_opts fills the defaults given in brackets. */
typedef struct {
  int32_t nu1;                 /* [2] pre-smoothing red/black sweeps            */
  int32_t nu2;                 /* [2] post-smoothing sweeps                     */
  int32_t max_iter;            /* [100] V-cycles (refinement steps)             */
  int32_t bottom_max_iter;     /* [0 = number of bottom cells] CG iterations    */
  int32_t min_bottom_edge;     /* [4] coarsen while every edge/2 >= this        */
  int32_t precision;           /* [MG_PREC_F64] or MG_PREC_F32_REFINE           */
  int32_t use_graph;           /* [1] replay the coarse levels as a HIP graph   */
  int32_t tune;                /* [1] 0 default tiles, 1 use tune cache,
                                      2 time the candidates now (and store);
                                      tiles of the level-0 and level-1 smoother
                                      and residual, cached by arch, kernel,
                                      precision, box shape and box count       */
  int32_t verbose;             /* [0] per-cycle log on stderr                   */
  int32_t aggregate;           /* [0] merge boxes once they stop coarsening and
                                      keep coarsening the merged box            */
  double bottom_rel_tol;       /* [1e-4] CG stops at ||r||2 <= tol*||rhs||2     */
  int32_t fused_min_edge;      /* [0] levels (above the bottom) whose box
                                      edges are all >= this run each red/black
                                      sweep as one pass into a second buffer
                                      plus a pass over the box boundary layers
                                      (same result as two half-sweeps);
                                      0 = half-sweeps everywhere               */
  int32_t krylov;              /* [0] 0: V-cycles until the tolerance (the
                                      paper's multigrid solve); 1: conjugate
                                      gradients preconditioned by one symmetric
                                      V-cycle per iteration (post-smoothing black
                                      then red on every level; the paper's
                                      Krylov CG, "Linear Solvers"); with
                                      MG_PREC_F32_REFINE the V-cycle runs in
                                      FP32 on r rounded to FP32 and CG stays in
                                      FP64; iters then counts CG iterations.
                                      The composite solve uses flexible GMRES
                                      instead (see mg_create_amr)              */
  int32_t ghost_write;         /* [1] on levels using half-sweeps (even extents
                                      in periodic directions), each update of a
                                      cell on a box's boundary layer is also
                                      stored into the face ghosts that mirror it,
                                      so only the first half-sweep after an
                                      interpolation needs an exchange (same
                                      result); 0 = exchange before every
                                      half-sweep                               */
  int32_t interp_fold;         /* [1] where a level and the next coarser one
                                      both write through (and the coarser one
                                      is smoothed, not the bottom), the
                                      interpolation of the correction is done
                                      by the first post-smoothing half-sweep,
                                      which adds the correction to each value
                                      it reads, instead of a pass of its own
                                      and an exchange (same result); 0 = a
                                      separate interpolation pass             */
  int32_t bottom_solver;       /* [0] bottom solve on its residual equation,
                                      from zero, to bottom_rel_tol in the
                                      2-norm: 0 = CG, 1 = BiCGStab (the two
                                      Krylov bottom solvers of the paper's
                                      section on linear solvers)              */
  int32_t restrict_fold;       /* [1] where a coarse level is smoothed from
                                      zero and its boxes are the finer boxes
                                      coarsened one to one, the restriction of
                                      the finer residual is done by that
                                      level's first half-sweep (which reads
                                      only its own cell's right-hand side),
                                      not by a pass of its own (same result):
                                      1 = on levels >= 2, and on level 1 where
                                      tune measured it faster; 2 = on every
                                      such level; 0 = separate passes         */
  int32_t stop_fold;           /* [1] FP64 V-cycle solves (krylov 0, more than
                                      one level, nu1 >= 1, level 0 not fused):
                                      the stop test's residual pass also does
                                      the next cycle's first red half-sweep,
                                      into a second level-0 array, and the
                                      cycle goes on there (the stop decision
                                      is read while it runs); same iterates,
                                      norms and result; 0 = a residual pass of
                                      its own before each cycle               */
  int32_t coarse_tail;         /* [1024] the coarsest levels, from the first
                                      level (>= 1) with at most this many cells
                                      down to a CG bottom of at most 1024
                                      cells, run as one launch of one 1024-lane
                                      work-group per V-cycle (every level
                                      between them half-swept with
                                      write-through, nu1 >= 1): each pass of
                                      those levels is a loop of its lanes with
                                      a barrier after it, instead of a launch;
                                      same arithmetic per cell, same result
                                      (the paper's V-cycle, "Linear Solvers");
                                      one compute unit then carries the
                                      level, so this pays only where launches
                                      cost more than its cells' loads;
                                      0 = a launch per pass                   */
} mg_opts_t;

typedef struct {
  int32_t iters;               /* V-cycles done                                 */
  int32_t nlevels;             /* multigrid levels                              */
  int32_t bottom_iters;        /* CG iterations of the last bottom solve        */
  int32_t converged;           /* 1 when the tolerance was met                  */
  double rel_resid;            /* max|f - A phi| / max|f| at return            */
  double abs_resid;            /* max|f - A phi| at return                      */
  double setup_ms;             /* mg_create wall time                           */
  double solve_ms;             /* mg_solve wall time                            */
  int32_t tail_level;          /* first level of the one-launch coarse tail
                                      (opts coarse_tail), counted as nlevels
                                      counts; 0 = none                         */
} mg_info_t;

/* One ghost-copy item: dst cells in dst_region take src cells at p - shift. */
typedef struct { int32_t dst, src; mg_box_t dst_region; int32_t shift[3]; } mg_copy_tag_t;

typedef struct mg_solver mg_solver_t;

/* Defaults listed in mg_opts_t. */
void mg_default_opts(mg_opts_t* opts);

/* Two-level composite solve (coarse level + one level refined by 2; the
 * paper's multi-level multigrid, coarse-to-fine interpolation, averaging and
 * refluxing of "Linear Solvers" and "Operations between levels").
 *
 * Coarse boxes cover the (Dirichlet-walled) domain; fine boxes, in the coarse
 * index space refined by 2, are disjoint unions of whole coarse cells, each
 * inside one coarse box.  Unknowns are the fine cells and the coarse cells no
 * fine box covers; covered coarse cells hold the mean of their children.
 * Fine ghost cells no fine box supplies are interpolated from the coarse
 * level (central slopes, unlimited); an uncovered coarse cell's flux across
 * a coarse/fine face is the mean of the 4 fine fluxes.  a = 1.
 * Each outer step: 2*nu1 fine sweeps, one coarse V-cycle, 2*nu2 fine sweeps.
 * The outer composite residual and the update are FP64; with precision
 * MG_PREC_F32_REFINE the correction (sweeps, V-cycle, interpolation,
 * refluxing) runs in FP32 on that residual rounded once.  With krylov = 1
 * the correction instead preconditions flexible GMRES (restart 20) on the
 * composite system: each cycle starts from the true composite residual and
 * ends when the Krylov estimate of its 2-norm reaches tol scaled by the
 * cycle's starting 2-norm / max-norm ratio; iters counts corrections, the
 * residual history has one entry per cycle.  The workspace then also holds
 * 21 + 20 composite vectors.
 * bcoef_c / bcoef_f: three face MultiFabs per level, or NULL for b = 1.
 * mg_solve_amr stops when the max-norm composite residual (fine cells and
 * uncovered coarse cells) is <= max(rel_tol * max|rhs| over the same cells,
 * abs_tol); phi_c, phi_f: ngrow 1 (in: guess, out: solution, covered coarse
 * cells averaged); rhs_c, rhs_f: ngrow 0 or 1 (covered coarse rhs unused).
 * Destroy with mg_destroy. */
int mg_query_workspace_amr(const mg_box_t* cboxes, int32_t ncb, const mg_box_t* fboxes,
                           int32_t nfb, const mg_geom_t* geom, const mg_opts_t* opts,
                           size_t* bytes);
int mg_create_amr(const mg_box_t* cboxes, int32_t ncb, const mg_box_t* fboxes, int32_t nfb,
                  const mg_geom_t* geom, double alpha, double beta,
                  const mg_multifab_t* const* bcoef_c, const mg_multifab_t* const* bcoef_f,
                  const mg_opts_t* opts, void* workspace, size_t ws_bytes, void* hip_stream,
                  mg_solver_t** out);
int mg_solve_amr(mg_solver_t* s, mg_multifab_t* phi_c, mg_multifab_t* phi_f,
                 const mg_multifab_t* rhs_c, const mg_multifab_t* rhs_f, double rel_tol,
                 double abs_tol, mg_info_t* info, double* resid_history);

/* Bytes of device workspace mg_create needs for these boxes and options
 * (has_acoef: whether a cell coefficient a will be given).  Host only; may be
 * called without a GPU.  Validates the box array like mg_create (nbox < 1 or
 * a null boxes or bytes pointer: MG_ERR_ARG). */
int mg_query_workspace(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                       const mg_opts_t* opts, int32_t has_acoef, size_t* bytes);

/* Build a solver for one level ("Linear Solvers"; box array and geometry of
 * "Basic data structures").  Validates the boxes (disjoint, inside, covering
 * the domain), builds the multigrid hierarchy, the ghost-exchange plans (hash
 * intersection, "Communication") and the tile tables, copies the coefficients
 * into the workspace and coarsens them there (averaging restriction,
 * "Operations between levels").  acoef: cell MultiFab or NULL (a = 1);
 * bcoef: three face MultiFabs (ixtype e_d, ngrow 0) or NULL (b = 1); both
 * MG_F64 over the same boxes.  bc_lo/bc_hi: MG_BC_PERIODIC exactly in the
 * periodic directions of geom, MG_BC_DIRICHLET0 elsewhere.  opts NULL =
 * defaults.  workspace: device memory of at least mg_query_workspace bytes,
 * 256-byte aligned.  hip_stream: hipStream_t or NULL. */
int mg_create(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
              const int32_t bc_lo[3], const int32_t bc_hi[3], double alpha, double beta,
              const mg_multifab_t* acoef, const mg_multifab_t* const* bcoef,
              const mg_opts_t* opts, void* workspace, size_t ws_bytes, void* hip_stream,
              mg_solver_t** out);

/* Replace the coefficients (same conventions as mg_create) and re-coarsen;
 * plans, tables and graphs are kept. */
int mg_set_coefficients(mg_solver_t* s, const mg_multifab_t* acoef,
                        const mg_multifab_t* const* bcoef);

/* Replace the face coefficients from three global face arrays (device,
 * MG_F64): array d has n_d + 1 faces along d and n elsewhere, element (i,j,k)
 * at i + nx_d * (j + ny_d * k) (x fastest), face i on the low side of cell i.
 * is_log = 1: the arrays hold log b.  acoef_global: NULL (a = 1) or a global
 * cell array.  Re-coarsens like mg_set_coefficients. */
int mg_set_coefficients_global(mg_solver_t* s, const void* acoef_global,
                               const void* const* bface_global, int32_t is_log);

/* Solve A phi = rhs by V-cycles until max|rhs - A phi| <= max(rel_tol *
 * max|rhs|, abs_tol) ("Linear Solvers"; the stop norm is the max norm of
 * "Parallel Reductions").  phi: MG_F64 cell MultiFab with ngrow 1, in:
 * initial guess, out: solution (its ghost cells are overwritten).  rhs:
 * MG_F64 cell MultiFab, ngrow 0 or 1.  Both over the solver's boxes.  For an
 * all-periodic singular problem the returned phi has zero mean.
 * resid_history: host array of max_iter + 1 doubles or NULL; entry k is the
 * max-norm residual after k cycles.  Returns MG_ERR_NOT_CONVERGED (phi and
 * info written) when max_iter is reached, MG_ERR_NAN on a non-finite norm. */
int mg_solve(mg_solver_t* s, mg_multifab_t* phi, const mg_multifab_t* rhs, double rel_tol,
             double abs_tol, mg_info_t* info, double* resid_history);

/* out = A phi on every valid cell (phi's ghosts are filled first).  phi as in
 * mg_solve; out: MG_F64 cell MultiFab over the same boxes. */
int mg_apply(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* out);

/* Adjoint face gradient dL/dlog b_f = -b_f * lambda^T (dA/db_f) phi for every
 * face of every box: -c_f (phi_j - phi_i)(lam_j - lam_i) on an interior or
 * periodic face, -2 c_f phi_i lam_i on a Dirichlet wall, c_f = beta b_f / h^2
 * (operator of "Linear Solvers").  phi and lam: as mg_solve's phi (ghosts are
 * filled).  grad: three MG_F64 face MultiFabs (ngrow 0). */
int mg_face_grad_logb(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* lam,
                      mg_multifab_t* const* grad);

/* Same gradient written to three global face arrays (layout of
 * mg_set_coefficients_global); each physical face once; in a periodic
 * direction faces 0 and n both carry the wrap face's value. */
int mg_face_grad_logb_global(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* lam,
                             void* const* grad_global);

/* dst = src on every valid cell (a MultiFab copy between ghost layouts, as
 * "Containers for mesh data" allows any nGrow).  Both MG_F64 cell MultiFabs
 * over the solver's boxes with ngrow 0 or 1; ghost cells of dst untouched.
 * Asynchronous. */
int mg_copy_valid(mg_solver_t* s, const mg_multifab_t* src, mg_multifab_t* dst);

/* Release the solver's host metadata and graphs (not the caller's memory). */
void mg_destroy(mg_solver_t* s);

/* Fill every ghost cell of mf whose periodically wrapped index lies in
 * another box's valid region (or in the same box's periodic image) with that
 * cell's value ("Operations on a level"): one fused copy kernel over all copy
 * tags ("Communication").  Ghost cells outside a non-periodic domain face are
 * left untouched.  mf: cell centred (ixtype 0), any ngrow, ncomp, dtype.
 * Asynchronous on hip_stream. */
int fill_boundary(mg_multifab_t* mf, const mg_geom_t* geom, void* hip_stream);
int mg_fill_boundary(mg_multifab_t* mf, const mg_geom_t* geom, void* hip_stream);

/* fill_boundary for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as fill_boundary, bit for bit, and it
 * calls no hipMalloc/hipFree: the exchange plan (64 bytes per copy tag plus
 * 8 bytes per 256 ghost cells of a tag) is copied on hip_stream into a
 * static device array of 4 MiB that the library holds on each device it
 * runs on until the process ends.  A plan larger than that returns
 * MG_ERR_WORKSPACE without launching anything (fill_boundary then serves the
 * layout).  Every call on one device shares that array: calls that overlap
 * on one device (other streams or threads) race and must be ordered by the
 * caller.  The host side of the plan is built with ordinary host memory
 * and cached like fill_boundary's.  Asynchronous on hip_stream. */
int mg_fill_boundary_noalloc(mg_multifab_t* mf, const mg_geom_t* geom, void* hip_stream);

/* The copy tags fill_boundary applies, in canonical order (dst, src, shift,
 * region lo), built by hash intersection ("Communication").  Host only.
 * Writes up to cap tags to out (out may be NULL when cap = 0) and the total
 * count to *n; returns MG_ERR_ARG if cap < *n and out != NULL. */
int mg_copy_tags(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom, int32_t ngrow,
                 mg_copy_tag_t* out, int32_t cap, int32_t* n);

/* Number of multigrid levels the solver would build (host only). */
int mg_num_levels(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                  const mg_opts_t* opts, int32_t* nlevels);

/* Kernel timing.  When enabled, mg_solve records HIP events around each
 * launch of the level-0 kernels of the given family, on the solver's stream;
 * mg_kernel_stats returns the summed duration and launch count since the last
 * reset.  family: 0 smoother (a half-sweep, or the fused pass of a whole
 * sweep when the level uses fused sweeps), 1 residual, 2 ghost exchange,
 * 3 restriction (kept for numbering; the restriction into level 1 now
 * opens the coarse levels), 4 interpolation (a separate pass, or the first
 * post-smoothing half-sweep that carries it when interp_fold applies),
 * 5 coarse levels (one graph or launch sequence per cycle, from the
 * restriction of the level-0 residual to level 1's corrections), 6 refinement
 * update and Krylov vector work, 7 the rim pass that ends a fused sweep,
 * 8 the face-gradient kernel of mg_face_grad_logb and
 * mg_face_grad_logb_global (the pass alone, without the ghost exchange of
 * phi and lambda before it). */
int mg_profile(mg_solver_t* s, int32_t enable);
int mg_kernel_stats(mg_solver_t* s, int32_t family, double* total_ms, int64_t* launches);

/* dst = src over `bytes` bytes with the library's own streaming kernel (one
 * 16-byte load and store per lane, no solver state): the achievable HBM rate
 * beside the kernels' rooflines, and the reference copy of known size for
 * the HBM traffic counters.  Device pointers, 16-byte aligned, bytes a
 * multiple of 16 (else MG_ERR_ARG).  Asynchronous on hip_stream. */
int mg_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Time one level-0 smoother half-sweep launched alone `reps` times on the
 * solver's stream (colour alternating) and return the mean duration; uses
 * phi/rhs as the data.  For roofline measurements. */
int mg_time_smoother(mg_solver_t* s, mg_multifab_t* phi, const mg_multifab_t* rhs,
                     int32_t reps, double* mean_ms);

/* Override the tile shape of the level-0 smoother (kernel 0: block lx x ly
 * lanes covering 2*lx x ly cells, tz planes per work-group) or of the
 * level-0 one-lane-per-cell kernels (kernel 1: lx x ly cells); kernel 2 = the
 * smoother variant that also stores each lane's unchanged pair cell, so cache
 * lines are written whole; unroll = the
 * number of planes whose loads a lane issues together (1, 2 or 4, <= tz).
 * lx*ly must be 64, 128 or 256 and the shape one of the tuner's candidates
 * (lx in {16,32,64} for kernel 0, {32,64,128} for kernel 1; ly a power of two
 * up to 16 (kernel 0) or 8 (kernel 1); tz in {2,...,64}).  kernel 3: the
 * fused sweep of level 0 (lx x ly x tz cells per work-group of lx/2*ly lanes;
 * (lx, ly) in {(64,4), (64,8), (32,8), (32,16)}, tz in {4,8,16,32}; unroll
 * ignored; MG_ERR_ARG when level 0 does not use fused sweeps).  kernel 4:
 * the level-0 residual pass that writes its restriction into level 1
 * (lx x ly cells, lx, ly and tz even, a kernel 1 candidate with unroll 2;
 * unroll ignored).  kernel 5: the FP32 smoother with one x-quad per lane
 * (block lx x ly lanes covering 4*lx x ly cells, lx in {8,16,32}, tz in
 * {1,2,4,8}, unroll 1 or 2; only for MG_PREC_F32_REFINE solvers whose
 * level 0 streams through buffer loads with write-through and whose level-0
 * boxes all have x extents that are multiples of 4, else MG_ERR_ARG);
 * mg_get_tile_shape reports it as kernel 0 with whole_pairs = 2.  tz in
 * {1,...,64} (kernels 0, 1, 2).  Every
 * shape gives bitwise-identical V-cycle solves; with krylov = 1 the dot
 * p.q is summed per tile of kernel 1, whose shape then changes the last
 * bits of the result. */
int mg_set_tile_shape(mg_solver_t* s, int32_t kernel, int32_t lx, int32_t ly, int32_t tz,
                      int32_t unroll);

/* The level-0 tile shapes in use (after tuning), for reports: kernel 0 the
 * half-sweep smoother -> {lx, ly, tz, unroll, whole_pairs}; kernel 1 the
 * one-lane-per-cell kernels -> {lx, ly, tz, unroll, 0}; kernel 3 the fused
 * sweep -> {lx, ly, tz, in_use, 0} (in_use 0 when level 0 runs half-sweeps;
 * lx = 0 when it has no fused sweep at all); kernel 4 the residual pass
 * that restricts into level 1 -> {lx, ly, tz, in_use, 0}.  shape: host
 * int32_t[5]. */
int mg_get_tile_shape(mg_solver_t* s, int32_t kernel, int32_t* shape);

/* Level-0 smoother tiles per box class ("tile size adjustable at run time",
 * chosen per box class): the boxes whose x extent is x_extent get lx x ly
 * lanes (lx in {16, 32, 64}) over tz planes per work-group, inside the one
 * launch of the level's half-sweep; lx * ly must equal the launch's thread
 * count and tz >= its unroll (the tuner with tune = 2 picks these shapes by
 * timing each class and keeps them only when the whole table is faster).
 * Other classes keep their shapes; mg_set_tile_shape (kernel 0 or 2) returns
 * to one shape for all boxes.  Every choice gives bitwise-identical solves.
 * MG_ERR_ARG when no box has that x extent, the shape is not such a
 * candidate, or level 0 uses fused sweeps. */
int mg_set_class_tile_shape(mg_solver_t* s, int32_t x_extent, int32_t lx, int32_t ly, int32_t tz);
/* The level-0 smoother's per-class shapes in use: *n classes (0 = one shape
 * for every box); out (host, nullable when cap = 0) receives cap >= *n
 * quadruples (x extent, lx, ly, tz), else MG_ERR_ARG. */
int mg_get_class_tile_shapes(mg_solver_t* s, int32_t* out, int32_t cap, int32_t* n);

/* ---------------------------------------------------------------------------
 * Nodal solver ("Linear Solvers": the nodal solver is built on finite
 * elements, its stencil from moment integrals over the cells, its coarse
 * operators from an algebraic coarsening).
 *
 * Solves -div(sigma grad phi) = f for phi at the nodes of the cell grid:
 * phi is the continuous piecewise-trilinear function of its nodal values, the
 * equation is tested with every nodal hat function, f is lumped to the nodes
 * and every row divided by the cell volume:
 *   (A phi)_p = (1/V) sum_{cells c at p} sigma_c sum_{corners q of c} K_pq phi_q,
 * K the trilinear cell stiffness assembled from the 1D moment integrals
 * int l_a l_b = h/3 or h/6 and int l_a' l_b' = +-1/h.  Walls are homogeneous
 * Dirichlet (phi = 0 on every wall node: bc MG_BC_DIRICHLET0 on both sides
 * of a non-periodic direction), periodic directions wrap (MG_BC_PERIODIC on
 * both sides).  All periodic: the problem is singular; the bottom removes
 * the mean of its right-hand side and the returned phi has zero mean.
 *
 * Multigrid: levels halve the cell count while every count stays even and
 * half of it is >= opts.min_bottom_edge (at least two levels are required);
 * interpolation trilinear, restriction its transpose / 8; coarse operators
 * R A P (Galerkin, 27 couplings per node, exactly symmetric); Jacobi
 * smoothing with weight 1 (nu1 >= 1 and nu2 sweeps); unpreconditioned CG at
 * the bottom to opts.bottom_rel_tol; stop at max|f - A phi| over the unknown
 * nodes <= max(rel_tol * max|f|, abs_tol).  FP64 only (precision 0, krylov
 * 0); opts.use_graph replays the coarse levels as a HIP graph.
 *
 * Data: boxes must cover the domain.  sigma is a cell MultiFab (ixtype 0,
 * ngrow 0) over the boxes, or NULL for sigma = 1; phi and rhs are nodal
 * MultiFabs (ixtype 1,1,1: box lo..hi holds nodes lo..hi+1 grown by ngrow,
 * ngrow 0 or 1), FP64, one component, canonical packing (boxes one after
 * another, x fastest), else MG_ERR_MISMATCH.  A node that several boxes hold
 * is read from the box whose cell range contains the node's index; on
 * return every node of every box array inside the domain (ghosts included,
 * walls 0, periodic images wrapped) holds the solution.  Ghost nodes beyond a
 * wall are not written.
 *
 * Workspace: caller-owned device memory of mg_nodal_query_workspace bytes
 * (per level: iterate, rhs and residual arrays over the unknown nodes plus
 * one ghost layer; coarse levels 14 coupling arrays), which must outlive
 * the handle.  The solver copies sigma; sigma may be freed after create.
 * Streams and errors as for mg_create / mg_solve.  mg_nodal_solve returns
 * after its result is complete; mg_nodal_apply is asynchronous. */
typedef struct mg_nodal mg_nodal_t;

int mg_nodal_query_workspace(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                             const mg_opts_t* opts, size_t* bytes);
int mg_nodal_create(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                    const int32_t bc_lo[3], const int32_t bc_hi[3], const mg_multifab_t* sigma,
                    const mg_opts_t* opts, void* workspace, size_t ws_bytes, void* hip_stream,
                    mg_nodal_t** out);
/* phi: in the initial guess, out the solution; info and resid_history (host,
 * max_iter + 1 entries, max-norm residual before each cycle) nullable. */
int mg_nodal_solve(mg_nodal_t* s, mg_multifab_t* phi, const mg_multifab_t* rhs, double rel_tol,
                   double abs_tol, mg_info_t* info, double* resid_history);
/* out = A phi on every node of out's arrays inside the domain (walls 0). */
int mg_nodal_apply(mg_nodal_t* s, const mg_multifab_t* phi, mg_multifab_t* out);
int mg_nodal_num_levels(const mg_nodal_t* s, int32_t* nlevels);
/* Mean duration of one finest-level Jacobi sweep launched alone reps times
 * (between two of the solver's level-0 buffers, on the values the last solve
 * left there), timed with HIP events on the solver's stream.  For roofline
 * measurements; the solver's iterate buffers are overwritten. */
int mg_nodal_time_smoother(mg_nodal_t* s, int32_t reps, double* mean_ms);
void mg_nodal_destroy(mg_nodal_t* s);

/* Free the device tables of fill_boundary's plan cache. */
void mg_release_caches(void);

/* Message for the last failure on this thread ("" if none). */
const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AMRMG_H */
