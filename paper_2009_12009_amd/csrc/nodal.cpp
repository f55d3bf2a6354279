// Node-centred finite-element solve (the nodal solver of the paper's "Linear
// Solvers" section): level hierarchy, workspace layout, Galerkin set-up, the
// V-cycle driver and the C entry points.
//
// The caller's data are nodal MultiFabs over a box array that covers the
// domain; the solve itself works on one array per level over the level's
// unknown nodes (see nodal.hpp), gathered from and scattered back to the
// boxes, so that nodes shared by several boxes are solved for once.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/amrmg.h"
#include "host.hpp"
#include "nodal.hpp"

using namespace amrmg;

namespace {

struct Bump {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct NdLevel {
  int n[3];  // cells
  NdGeo g;
  long long size = 0;  // padded elements
  double* x[3] = {nullptr, nullptr, nullptr};  // iterates (level 0: 3, coarse: 2)
  double *f = nullptr, *r = nullptr;
  NdStencil st{};  // levels >= 1
};

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

#define HIPTRY(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess)                                                      \
      return fail(MG_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

IBox to_ibox(const mg_box_t& b) {
  IBox r;
  for (int d = 0; d < 3; ++d) {
    r.lo[d] = b.lo[d];
    r.hi[d] = b.hi[d];
  }
  return r;
}

NdStencilC cst(const NdStencil& s) {
  NdStencilC c;
  for (int q = 0; q < kNdStored; ++q) c.w[q] = s.w[q];
  return c;
}

}  // namespace

struct mg_nodal {
  IBox domain;
  int n[3];
  int periodic[3];
  mg_opts_t opts;
  double omega = 1.0;
  bool singular = false;
  std::vector<IBox> boxes;
  std::vector<NdLevel> L;
  NdKappa kap;
  double* sig = nullptr;
  // box tables: nodal arrays with ngrow 0 and 1, cell arrays with ngrow 0
  std::vector<NdBox> h_box[3];
  NdBox* d_box[3] = {nullptr, nullptr, nullptr};
  int max_elems[3] = {0, 0, 0};
  double* bwork = nullptr;
  double* partials = nullptr;
  // Krylov outer solve (opts.krylov = 1): finest-level x, r, p, q and the
  // CG scalars rho (two, alternating), p.q
  double *kx = nullptr, *kr = nullptr, *kp = nullptr, *kq = nullptr;
  double* d_cg = nullptr;
  int* d_iters = nullptr;
  unsigned long long* d_norm = nullptr;  // 3 slots
  size_t ws_need = 0;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_norm[2] = {nullptr, nullptr};
  // the coarse part of a cycle captured once per level-0 buffer it
  // interpolates into (opts.use_graph)
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  unsigned long long* h_norm = nullptr;  // pinned: 3 slots, then the iteration count
  double setup_ms = 0;
};

namespace {

unsigned long long* nslot(mg_nodal* s, int k) { return s->d_norm + (size_t)k * kNdNormSlot; }

// Caller stream -> solver stream at entry; solver stream -> caller stream on
// every exit.
class NdCall {
 public:
  explicit NdCall(mg_nodal* s) : s_(s) {
    rc_ = MG_OK;
    if (hipEventRecord(s->ev_in, s->user) != hipSuccess ||
        hipStreamWaitEvent(s->st, s->ev_in, 0) != hipSuccess) {
      rc_ = fail(MG_ERR_HIP, "stream ordering failed");
      s_ = nullptr;
    }
  }
  ~NdCall() {
    if (s_ && hipEventRecord(s_->ev_out, s_->st) == hipSuccess)
      (void)hipStreamWaitEvent(s_->user, s_->ev_out, 0);
  }
  int rc() const { return rc_; }
  int finish() {
    mg_nodal* s = s_;
    s_ = nullptr;
    if (!s) return MG_OK;
    if (hipEventRecord(s->ev_out, s->st) != hipSuccess ||
        hipStreamWaitEvent(s->user, s->ev_out, 0) != hipSuccess)
      return fail(MG_ERR_HIP, "stream ordering failed");
    return MG_OK;
  }

 private:
  mg_nodal* s_;
  int rc_;
};

NdGeo geo_of(const int n[3], const int per[3]) {
  NdGeo g;
  g.mx = per[0] ? n[0] : n[0] - 1;
  g.my = per[1] ? n[1] : n[1] - 1;
  g.mz = per[2] ? n[2] : n[2] - 1;
  g.px = g.mx + 2;
  g.py = g.my + 2;
  g.per = (per[0] ? 1 : 0) | (per[1] ? 2 : 0) | (per[2] ? 4 : 0);
  g.tz = 1;
  return g;
}

long long padded(const NdGeo& g) { return (long long)g.px * g.py * (g.mz + 2); }

// Planes per work-group: as deep as 8 while the level still gets >= 2048
// work-groups of 64 x 4 lanes (coarse levels: shallow, so that their
// launches are not a few long serial marches).
int default_tz(const NdGeo& g) {
  const long long cols = (long long)((g.mx + 63) / 64) * ((g.my + 3) / 4);
  int tz = 8;
  while (tz > 1 && cols * ((g.mz + tz - 1) / tz) < 2048) tz /= 2;
  return tz;
}

// K_ab / V of one cell for corners differing in the coordinates of `pat`,
// from the 1D moment integrals (int l_a l_b = h/3 or h/6, int l_a' l_b' =
// +-1/h).
NdKappa kappa_of(const double h[3]) {
  NdKappa k;
  const double V = h[0] * h[1] * h[2];
  for (int pat = 0; pat < 8; ++pat) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
      const bool dd = (pat >> d) & 1;
      double t = dd ? -1.0 / h[d] : 1.0 / h[d];
      for (int e = 0; e < 3; ++e) {
        if (e == d) continue;
        const bool de = (pat >> e) & 1;
        t *= de ? h[e] / 6.0 : h[e] / 3.0;
      }
      s += t;
    }
    k.k[pat] = s / V;
  }
  return k;
}

int plan(mg_nodal* s, Bump& bump) {
  s->L.clear();
  int n[3] = {s->n[0], s->n[1], s->n[2]};
  const int mb = std::max(1, s->opts.min_bottom_edge);
  while (true) {
    NdLevel lv;
    for (int d = 0; d < 3; ++d) lv.n[d] = n[d];
    lv.g = geo_of(n, s->periodic);
    lv.g.tz = default_tz(lv.g);
    if (lv.g.mx < 1 || lv.g.my < 1 || lv.g.mz < 1)
      return fail(MG_ERR_INVALID_BOXARRAY, "a level has no unknown nodes");
    lv.size = padded(lv.g);
    if (lv.size >= (1ll << 31)) return fail(MG_ERR_INVALID_BOXARRAY, "level too large");
    s->L.push_back(lv);
    bool more = true;
    for (int d = 0; d < 3; ++d) more = more && n[d] % 2 == 0 && n[d] / 2 >= mb;
    if (!more) break;
    for (int d = 0; d < 3; ++d) n[d] /= 2;
  }
  if (s->L.size() < 2)
    return fail(MG_ERR_INVALID_BOXARRAY,
                "the domain cannot be coarsened once under min_bottom_edge (nodal solve)");
  for (size_t l = 0; l < s->L.size(); ++l) {
    NdLevel& lv = s->L[l];
    const int nx = l == 0 ? 3 : 2;
    for (int i = 0; i < nx; ++i) lv.x[i] = bump.take<double>(lv.size);
    lv.f = bump.take<double>(lv.size);
    lv.r = bump.take<double>(lv.size);
    if (l > 0)
      for (int q = 0; q < kNdStored; ++q) lv.st.w[q] = bump.take<double>(lv.size);
  }
  const NdGeo& g0 = s->L[0].g;
  s->sig = bump.take<double>((size_t)(g0.mx + 1) * (g0.my + 1) * (g0.mz + 1));
  s->bwork = bump.take<double>(3 * (size_t)s->L.back().size);
  {
    // room for the partial sums of the shallowest launch depth
    NdGeo g1 = g0;
    g1.tz = 1;
    s->partials = bump.take<double>((size_t)nd_sum_partials_count(g1));
  }
  s->d_norm = bump.take<unsigned long long>(3 * (size_t)kNdNormSlot);
  s->d_iters = bump.take<int>(4);
  if (s->opts.krylov) {
    s->kx = bump.take<double>(s->L[0].size);
    s->kr = bump.take<double>(s->L[0].size);
    s->kp = bump.take<double>(s->L[0].size);
    s->kq = bump.take<double>(s->L[0].size);
    s->d_cg = bump.take<double>(4);
  }
  // box tables: nodal ngrow 0 and 1, cells ngrow 0
  for (int t = 0; t < 3; ++t) {
    s->h_box[t].clear();
    long long off = 0;
    int mx = 0;
    for (const IBox& b : s->boxes) {
      NdBox nb;
      for (int d = 0; d < 3; ++d) {
        nb.lo[d] = b.lo[d];
        nb.hi[d] = b.hi[d];
      }
      nb.off = off;
      s->h_box[t].push_back(nb);
      const int e = t == 2 ? 0 : 1, ng = t == 1 ? 1 : 0;
      const long long v = (long long)(ext(b, 0) + e + 2 * ng) * (ext(b, 1) + e + 2 * ng) *
                          (ext(b, 2) + e + 2 * ng);
      off += v;
      mx = (int)std::min<long long>(std::max<long long>(mx, v), 1ll << 30);
    }
    s->max_elems[t] = mx;
    s->d_box[t] = bump.take<NdBox>(s->boxes.size());
  }
  s->ws_need = bump.off + 256;
  return MG_OK;
}

// MultiFab check: the solver's boxes, canonical packing, FP64, ncomp 1.
int check_mf(const mg_nodal* s, const mg_multifab_t* mf, bool nodal, int ng_max, const char* what) {
  if (!mf) return fail(MG_ERR_ARG, std::string(what) + " is null");
  if (mf->nbox != (int)s->boxes.size() || !mf->boxes || !mf->offsets || !mf->data)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": box count or pointers differ");
  if (mf->dtype != MG_F64 || mf->ncomp != 1)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": FP64, one component expected");
  if (mf->ngrow < 0 || mf->ngrow > ng_max)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": unsupported ngrow");
  for (int d = 0; d < 3; ++d)
    if (mf->ixtype[d] != (nodal ? 1 : 0))
      return fail(MG_ERR_MISMATCH, std::string(what) + (nodal ? ": nodal data expected"
                                                             : ": cell data expected"));
  const int e = nodal ? 1 : 0;
  int64_t off = 0;
  for (size_t b = 0; b < s->boxes.size(); ++b) {
    if (!same(to_ibox(mf->boxes[b]), s->boxes[b]))
      return fail(MG_ERR_MISMATCH, std::string(what) + ": box " + std::to_string(b) + " differs");
    if (mf->offsets[b] != off)
      return fail(MG_ERR_MISMATCH, std::string(what) + ": non-canonical offsets");
    const IBox& B = s->boxes[b];
    off += (int64_t)(ext(B, 0) + e + 2 * mf->ngrow) * (ext(B, 1) + e + 2 * mf->ngrow) *
           (ext(B, 2) + e + 2 * mf->ngrow);
  }
  return MG_OK;
}

int fill_ghosts(mg_nodal* s, const NdLevel& lv, double* a) {
  if (lv.g.per) HIPTRY(nd_launch_fill_ghosts(s->st, lv.g, a));
  return MG_OK;
}

// Sweep, residual or apply on level l.
int sweep(mg_nodal* s, size_t l, const double* phi, const double* f, double* out, int mode,
          unsigned long long* norm) {
  NdLevel& lv = s->L[l];
  if (l == 0)
    HIPTRY(nd_launch_sweep0(s->st, lv.g, s->kap, s->sig, phi, f, out, s->omega, mode, norm));
  else
    HIPTRY(nd_launch_sweep_st(s->st, lv.g, cst(lv.st), phi, f, out, s->omega, mode, norm));
  if (mode != ND_RESID && mode != ND_APPLY) return fill_ghosts(s, lv, out);
  return MG_OK;
}

// Levels l >= 1 from a zero guess on their f; returns in *res the index of
// the level's iterate buffer that holds the correction.
int coarse(mg_nodal* s, size_t l, int* res) {
  NdLevel& lv = s->L[l];
  int rc;
  if (l + 1 == s->L.size()) {
    const int maxit = s->opts.bottom_max_iter > 0 ? s->opts.bottom_max_iter
                                                  : lv.g.mx * lv.g.my * lv.g.mz;
    HIPTRY(nd_launch_bottom_cg(s->st, lv.g, cst(lv.st), lv.f, lv.x[0], s->bwork,
                               s->opts.bottom_rel_tol, maxit, s->singular ? 1 : 0, s->d_iters));
    *res = 0;
    return MG_OK;
  }
  int cur = 0;
  if ((rc = sweep(s, l, nullptr, lv.f, lv.x[0], ND_ZERO, nullptr))) return rc;
  for (int k = 1; k < s->opts.nu1; ++k) {
    if ((rc = sweep(s, l, lv.x[cur], lv.f, lv.x[1 - cur], ND_JACOBI, nullptr))) return rc;
    cur = 1 - cur;
  }
  if ((rc = sweep(s, l, lv.x[cur], lv.f, lv.r, ND_RESID, nullptr))) return rc;
  NdLevel& cl = s->L[l + 1];
  HIPTRY(nd_launch_restrict(s->st, lv.g, cl.g, lv.r, cl.f));
  int cres = 0;
  if ((rc = coarse(s, l + 1, &cres))) return rc;
  HIPTRY(nd_launch_interp_add(s->st, lv.g, cl.g, cl.x[cres], lv.x[cur]));
  if ((rc = fill_ghosts(s, lv, lv.x[cur]))) return rc;
  for (int k = 0; k < s->opts.nu2; ++k) {
    if ((rc = sweep(s, l, lv.x[cur], lv.f, lv.x[1 - cur], ND_JACOBI, nullptr))) return rc;
    cur = 1 - cur;
  }
  *res = cur;
  return MG_OK;
}

// From the finest residual L0.r: restriction into level 1, levels >= 1, and
// the interpolation of level 1's correction into out.  Captured once as a
// HIP graph when opts.use_graph.
int coarse_part(mg_nodal* s, double* out) {
  NdLevel& l0 = s->L[0];
  NdLevel& l1 = s->L[1];
  HIPTRY(nd_launch_restrict(s->st, l0.g, l1.g, l0.r, l1.f));
  int cres = 0;
  int rc;
  if ((rc = coarse(s, 1, &cres))) return rc;
  HIPTRY(nd_launch_interp_add(s->st, l0.g, l1.g, l1.x[cres], out));
  return fill_ghosts(s, l0, out);
}

int read_slot(mg_nodal* s, int slot, double* out) {
  HIPTRY(hipMemcpyAsync(s->h_norm + (size_t)slot * kNdNormSlot, nslot(s, slot),
                        sizeof(unsigned long long) * kNdNormSlot, hipMemcpyDeviceToHost, s->st));
  HIPTRY(hipStreamSynchronize(s->st));
  unsigned long long m = 0;
  for (int w = 0; w < kNdNormWays; ++w)
    m = std::max(m, s->h_norm[(size_t)slot * kNdNormSlot + (size_t)w * kNdNormStride]);
  std::memcpy(out, &m, sizeof(double));
  return MG_OK;
}

// z = M r: one finest-level V-cycle from zero on right-hand side r (the
// Krylov preconditioner).  Returns the level-0 buffer holding z.
int precond(mg_nodal* s, const double* r, int* zi) {
  NdLevel& l0 = s->L[0];
  int rc;
  int cur = 0;
  if ((rc = sweep(s, 0, nullptr, r, l0.x[0], ND_ZERO, nullptr))) return rc;
  for (int k = 1; k < s->opts.nu1; ++k) {
    if ((rc = sweep(s, 0, l0.x[cur], r, l0.x[1 - cur], ND_JACOBI, nullptr))) return rc;
    cur = 1 - cur;
  }
  if ((rc = sweep(s, 0, l0.x[cur], r, l0.r, ND_RESID, nullptr))) return rc;
  if (s->graph[cur]) {
    HIPTRY(hipGraphLaunch(s->graph[cur], s->st));
  } else if ((rc = coarse_part(s, l0.x[cur]))) {
    return rc;
  }
  for (int k = 0; k < s->opts.nu2; ++k) {
    if ((rc = sweep(s, 0, l0.x[cur], r, l0.x[1 - cur], ND_JACOBI, nullptr))) return rc;
    cur = 1 - cur;
  }
  *zi = cur;
  return MG_OK;
}

// Conjugate gradients on the finest level preconditioned by one V-cycle per
// iteration, from the gathered initial guess in kx: standard recurrences
// with the scalars on the device; stop on the max norm of the recurrence
// residual, confirmed on the true residual (if that is still above tol, r is
// replaced by it and the recurrence restarts from p = M r).  All periodic:
// the mean is taken out of r at the start and after a restart and out of
// every z.
int solve_pcg(mg_nodal* s, double tol, mg_info_t* inf, double* hist, int* status) {
  NdLevel& l0 = s->L[0];
  const NdGeo& g = l0.g;
  double *x = s->kx, *r = s->kr, *p = s->kp, *q = s->kq;
  int rc;
  auto true_residual = [&](double* buf, double* norm) -> int {
    int rc2;
    if ((rc2 = fill_ghosts(s, l0, x))) return rc2;
    HIPTRY(nd_launch_fill_u64(s->st, nslot(s, 2), kNdNormSlot, 0ull));
    if ((rc2 = sweep(s, 0, x, l0.f, buf, ND_RESID, s->singular ? nullptr : nslot(s, 2))))
      return rc2;
    if (s->singular) {
      HIPTRY(nd_launch_remove_mean(s->st, g, buf, s->partials));
      HIPTRY(nd_launch_maxabs(s->st, g, buf, nslot(s, 2)));
    }
    return read_slot(s, 2, norm);
  };
  double rn;
  if ((rc = true_residual(r, &rn))) return rc;
  int it = 0;
  bool restart = true;
  *status = MG_OK;
  while (true) {
    if (hist) hist[it] = rn;
    if (s->opts.verbose) fprintf(stderr, "amrmg nodal pcg %d  max|r| = %.6e\n", it, rn);
    if (!std::isfinite(rn)) {
      *status = fail(MG_ERR_NAN, "residual norm is not finite");
      break;
    }
    if (rn <= tol) {
      double rt;
      if ((rc = true_residual(q, &rt))) return rc;
      if (rt <= tol) {
        inf->converged = 1;
        break;
      }
      HIPTRY(hipMemcpyAsync(r, q, sizeof(double) * l0.size, hipMemcpyDeviceToDevice, s->st));
      restart = true;
    }
    if (it == s->opts.max_iter) {
      *status = fail(MG_ERR_NOT_CONVERGED, "max_iter reached");
      break;
    }
    int zi = 0;
    if ((rc = precond(s, r, &zi))) return rc;
    double* z = l0.x[zi];
    if (s->singular) HIPTRY(nd_launch_remove_mean(s->st, g, z, s->partials));
    double* rho_new = s->d_cg + (it & 1);
    double* rho_old = s->d_cg + ((it + 1) & 1);
    HIPTRY(nd_launch_dot(s->st, g, r, z, s->partials, rho_new));
    HIPTRY(nd_launch_cg_p(s->st, g, p, z, rho_new, rho_old, restart ? 1 : 0));
    if ((rc = fill_ghosts(s, l0, p))) return rc;
    restart = false;
    if ((rc = sweep(s, 0, p, l0.f, q, ND_APPLY, nullptr))) return rc;
    HIPTRY(nd_launch_dot(s->st, g, p, q, s->partials, s->d_cg + 2));
    HIPTRY(nd_launch_fill_u64(s->st, nslot(s, 2), kNdNormSlot, 0ull));
    HIPTRY(nd_launch_cg_xr(s->st, g, x, p, r, q, rho_new, s->d_cg + 2, nslot(s, 2)));
    ++it;
    if ((rc = read_slot(s, 2, &rn))) return rc;
  }
  inf->iters = it;
  inf->abs_resid = rn;
  return MG_OK;
}

// The rest of a finest-level V-cycle after its first sweep (from a to b):
// the iterate never returns to buffer a.  Returns the buffer index holding
// the new iterate.
int cycle_rest(mg_nodal* s, int a, int b, const double* F, int* out_idx) {
  NdLevel& l0 = s->L[0];
  const int c = 3 - a - b;
  int cur = b, other = c;
  int rc;
  for (int k = 1; k < s->opts.nu1; ++k) {
    if ((rc = sweep(s, 0, l0.x[cur], F, l0.x[other], ND_JACOBI, nullptr))) return rc;
    std::swap(cur, other);
  }
  if ((rc = sweep(s, 0, l0.x[cur], F, l0.r, ND_RESID, nullptr))) return rc;
  if (s->graph[cur]) {
    HIPTRY(hipGraphLaunch(s->graph[cur], s->st));
  } else if ((rc = coarse_part(s, l0.x[cur]))) {
    return rc;
  }
  for (int k = 0; k < s->opts.nu2; ++k) {
    if ((rc = sweep(s, 0, l0.x[cur], F, l0.x[other], ND_JACOBI, nullptr))) return rc;
    std::swap(cur, other);
  }
  *out_idx = cur;
  return MG_OK;
}


}  // namespace

extern "C" {

int mg_nodal_query_workspace(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                             const mg_opts_t* opts, size_t* bytes) {
  if (!boxes || nbox <= 0 || !geom || !bytes) return fail(MG_ERR_ARG, "bad argument");
  mg_nodal s;
  s.domain = to_ibox(geom->domain);
  for (int d = 0; d < 3; ++d) {
    s.n[d] = ext(s.domain, d);
    s.periodic[d] = geom->is_periodic[d] != 0;
  }
  if (opts)
    s.opts = *opts;
  else
    mg_default_opts(&s.opts);
  for (int i = 0; i < nbox; ++i) s.boxes.push_back(to_ibox(boxes[i]));
  Bump dry{nullptr};
  int rc = plan(&s, dry);
  if (rc) return rc;
  *bytes = s.ws_need;
  return MG_OK;
}

int mg_nodal_create(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                    const int32_t bc_lo[3], const int32_t bc_hi[3], const mg_multifab_t* sigma,
                    const mg_opts_t* opts, void* workspace, size_t ws_bytes, void* hip_stream,
                    mg_nodal_t** out) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!boxes || nbox <= 0 || !geom || !bc_lo || !bc_hi || !out)
    return fail(MG_ERR_ARG, "bad argument");
  *out = nullptr;
  std::unique_ptr<mg_nodal> s(new mg_nodal());
  s->domain = to_ibox(geom->domain);
  if (!ok(s->domain)) return fail(MG_ERR_ARG, "empty domain");
  for (int d = 0; d < 3; ++d) {
    s->n[d] = ext(s->domain, d);
    const bool per = geom->is_periodic[d] != 0;
    const int want = per ? MG_BC_PERIODIC : MG_BC_DIRICHLET0;
    if (bc_lo[d] != want || bc_hi[d] != want)
      return fail(MG_ERR_ARG, "boundary conditions must be periodic where the geometry is "
                              "periodic and homogeneous Dirichlet elsewhere");
    s->periodic[d] = per;
  }
  if (opts)
    s->opts = *opts;
  else
    mg_default_opts(&s->opts);
  if (s->opts.precision != MG_PREC_F64 || (s->opts.krylov != 0 && s->opts.krylov != 1))
    return fail(MG_ERR_ARG, "the nodal solve runs in FP64 (precision 0, krylov 0 or 1)");
  if (s->opts.krylov && s->opts.nu1 != s->opts.nu2)
    return fail(MG_ERR_ARG, "the nodal Krylov solve needs a symmetric V-cycle (nu1 == nu2)");
  if (s->opts.nu1 < 1 || s->opts.nu2 < 0 || s->opts.max_iter < 0 ||
      !(s->opts.bottom_rel_tol >= 0))
    return fail(MG_ERR_ARG, "the nodal solve needs nu1 >= 1, nu2 >= 0, max_iter >= 0");
  for (int i = 0; i < nbox; ++i) s->boxes.push_back(to_ibox(boxes[i]));
  std::string err;
  if (!validate_boxes(s->boxes, s->domain, true, &err)) return fail(MG_ERR_INVALID_BOXARRAY, err);
  s->singular = s->periodic[0] && s->periodic[1] && s->periodic[2];
  int rc;
  {
    Bump dry{nullptr};
    if ((rc = plan(s.get(), dry))) return rc;
  }
  if (!workspace || ws_bytes < s->ws_need)
    return fail(MG_ERR_WORKSPACE, "workspace needs " + std::to_string(s->ws_need) + " bytes");
  {
    Bump real{static_cast<char*>(workspace)};
    if ((rc = plan(s.get(), real))) return rc;
  }
  double h[3];
  for (int d = 0; d < 3; ++d) h[d] = (geom->prob_hi[d] - geom->prob_lo[d]) / s->n[d];
  if (!(h[0] > 0 && h[1] > 0 && h[2] > 0)) return fail(MG_ERR_ARG, "bad geometry extent");
  s->kap = kappa_of(h);
  if (sigma && (rc = check_mf(s.get(), sigma, false, 0, "sigma"))) return rc;
  s->user = static_cast<hipStream_t>(hip_stream);
  HIPTRY(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
  HIPTRY(hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
  HIPTRY(hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
  for (hipEvent_t& e : s->ev_norm) HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPTRY(hipHostMalloc((void**)&s->h_norm, sizeof(unsigned long long) * (3 * kNdNormSlot + 8),
                       hipHostMallocDefault));
  {
    NdCall call(s.get());
    if ((rc = call.rc())) return rc;
    // every array starts at 0 (wall ghosts stay 0 for good)
    HIPTRY(nd_launch_fill(s->st, static_cast<double*>(workspace), (long long)(s->ws_need / 8), 0.0));
    for (int t = 0; t < 3; ++t)
      HIPTRY(hipMemcpyAsync(s->d_box[t], s->h_box[t].data(), sizeof(NdBox) * s->h_box[t].size(),
                            hipMemcpyHostToDevice, s->st));
    const NdGeo& g0 = s->L[0].g;
    const int dlo[3] = {s->domain.lo[0], s->domain.lo[1], s->domain.lo[2]};
    if (sigma) {
      HIPTRY(nd_launch_sigma(s->st, g0, s->d_box[2], nbox, s->max_elems[2], dlo, s->n,
                             static_cast<const double*>(sigma->data), s->sig));
    } else {
      HIPTRY(nd_launch_fill(s->st, s->sig, (long long)(g0.mx + 1) * (g0.my + 1) * (g0.mz + 1), 1.0));
    }
    // Galerkin coarse operators
    for (size_t l = 1; l < s->L.size(); ++l) {
      NdLevel& f = s->L[l - 1];
      NdLevel& c = s->L[l];
      if (l == 1)
        HIPTRY(nd_launch_rap0(s->st, f.g, c.g, s->kap, s->sig, c.st));
      else
        HIPTRY(nd_launch_rap(s->st, f.g, c.g, cst(f.st), c.st));
      for (int q = 0; q < kNdStored; ++q)
        if ((rc = fill_ghosts(s.get(), c, c.st.w[q]))) return rc;
    }
    // tune = 2: the finest level's launch depth by timing its Jacobi sweep
    // (on the zeroed buffers: the speed does not depend on the values)
    if (s->opts.tune == 2) {
      NdLevel& l0 = s->L[0];
      hipEvent_t a = nullptr, b = nullptr;
      HIPTRY(hipEventCreate(&a));
      HIPTRY(hipEventCreate(&b));
      float best = 1e30f;
      int btz = l0.g.tz;
      for (int tz : {2, 4, 8, 16}) {
        l0.g.tz = tz;
        for (int k = 0; k < 8 && !rc; ++k) {
          if (k == 2 && hipEventRecord(a, s->st) != hipSuccess) rc = fail(MG_ERR_HIP, "event");
          if (!rc) rc = sweep(s.get(), 0, l0.x[k & 1], l0.f, l0.x[1 - (k & 1)], ND_JACOBI, nullptr);
        }
        float ms = 0.f;
        if (!rc && (hipEventRecord(b, s->st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&ms, a, b) != hipSuccess))
          rc = fail(MG_ERR_HIP, "event timing");
        if (rc) break;
        if (ms < best) {
          best = ms;
          btz = tz;
        }
      }
      hipEventDestroy(a);
      hipEventDestroy(b);
      if (rc) return rc;
      l0.g.tz = btz;
      if (s->opts.verbose)
        fprintf(stderr, "amrmg nodal tune: finest sweep %d planes, %.4f ms\n", btz, best / 6);
    }
    // the coarse part of the cycle as a graph, one per level-0 buffer it
    // interpolates into
    for (int i = 0; i < 3 && s->opts.use_graph; ++i) {
      HIPTRY(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
      rc = coarse_part(s.get(), s->L[0].x[i]);
      hipGraph_t gr = nullptr;
      const hipError_t e = hipStreamEndCapture(s->st, &gr);
      if (rc) {
        if (gr) hipGraphDestroy(gr);
        return rc;
      }
      if (e != hipSuccess) return fail(MG_ERR_HIP, "graph capture failed");
      hipGraphExec_t ex;
      const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      hipGraphDestroy(gr);
      if (ei != hipSuccess) return fail(MG_ERR_HIP, "graph instantiate failed");
      s->graph[i] = ex;
    }
    HIPTRY(hipStreamSynchronize(s->st));
    if ((rc = call.finish())) return rc;
  }
  s->setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = s.release();
  return MG_OK;
}

int mg_nodal_solve(mg_nodal_t* s, mg_multifab_t* phi, const mg_multifab_t* rhs, double rel_tol,
                   double abs_tol, mg_info_t* info, double* resid_history) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!s) return fail(MG_ERR_ARG, "null solver");
  int rc;
  if ((rc = check_mf(s, phi, true, 1, "phi"))) return rc;
  if ((rc = check_mf(s, rhs, true, 1, "rhs"))) return rc;
  if (!(rel_tol >= 0) || !(abs_tol >= 0)) return fail(MG_ERR_ARG, "negative tolerance");
  NdCall call(s);
  if ((rc = call.rc())) return rc;
  NdLevel& l0 = s->L[0];
  const int nbox = (int)s->boxes.size();
  const int dlo[3] = {s->domain.lo[0], s->domain.lo[1], s->domain.lo[2]};
  const int tp = phi->ngrow, tr = rhs->ngrow;
  mg_info_t inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.nlevels = (int)s->L.size();
  inf.setup_ms = s->setup_ms;
  // f and the initial guess into level-0 arrays; the iterate then rotates
  // over the three level-0 buffers
  HIPTRY(nd_launch_gather(s->st, l0.g, s->d_box[tr], nbox, s->max_elems[tr], tr, dlo,
                          static_cast<const double*>(rhs->data), l0.f));
  double* x0 = s->opts.krylov ? s->kx : l0.x[0];
  HIPTRY(nd_launch_gather(s->st, l0.g, s->d_box[tp], nbox, s->max_elems[tp], tp, dlo,
                          static_cast<const double*>(phi->data), x0));
  if ((rc = fill_ghosts(s, l0, x0))) return rc;
  HIPTRY(nd_launch_fill_u64(s->st, s->d_norm, 3 * kNdNormSlot, 0ull));
  HIPTRY(nd_launch_maxabs(s->st, l0.g, l0.f, nslot(s, 0)));
  double normf;
  if ((rc = read_slot(s, 0, &normf))) return rc;
  if (!std::isfinite(normf)) return fail(MG_ERR_NAN, "rhs holds a non-finite value");
  int status = MG_OK;
  int cur = 0;
  double* result = nullptr;
  if (normf == 0.0) {
    HIPTRY(nd_launch_fill(s->st, x0, l0.size, 0.0));
    result = x0;
    inf.converged = 1;
    if (resid_history) resid_history[0] = 0.0;
  } else if (s->opts.krylov) {
    if ((rc = solve_pcg(s, std::max(rel_tol * normf, abs_tol), &inf, resid_history, &status)))
      return rc;
    inf.rel_resid = inf.abs_resid / normf;
    result = s->kx;
  } else {
    const double tol = std::max(rel_tol * normf, abs_tol);
    int it = 0, rising = 0;
    double rn = 0, first = 0, prev = 0, prev2 = 0;
    // The first sweep of a cycle reads the iterate (buffer a), writes buffer
    // a + 1 and gives the stop test's residual; the rest of the cycle never
    // writes buffer a, which is the result if that residual meets the
    // tolerance (the norm is read while the rest of the cycle runs, unless
    // the norms' trend puts it within reach of the tolerance).
    auto decide = [&]() -> int {
      if (hipEventSynchronize(s->ev_norm[it & 1]) != hipSuccess) return -1;
      const unsigned long long* h = s->h_norm + (size_t)(1 + (it & 1)) * kNdNormSlot;
      unsigned long long m = 0;
      for (int w = 0; w < kNdNormWays; ++w) m = std::max(m, h[(size_t)w * kNdNormStride]);
      std::memcpy(&rn, &m, sizeof(double));
      if (resid_history) resid_history[it] = rn;
      if (s->opts.verbose) fprintf(stderr, "amrmg nodal cycle %d  max|r| = %.6e\n", it, rn);
      if (!std::isfinite(rn)) {
        status = fail(MG_ERR_NAN, "residual norm is not finite");
        return 1;
      }
      if (it == 0) first = rn;
      if (rn <= tol) {
        inf.converged = 1;
        return 1;
      }
      if (it == s->opts.max_iter) {
        status = fail(MG_ERR_NOT_CONVERGED, "max_iter reached");
        return 1;
      }
      if (it > 0) rising = rn > prev ? rising + 1 : 0;
      if (rising >= 3 && rn > first) {
        status = fail(MG_ERR_DIVERGED, "residual grew for 3 cycles");
        return 1;
      }
      prev2 = prev;
      prev = rn;
      return 0;
    };
    while (true) {
      const int a = cur, b = (cur + 1) % 3;
      const int slot = 1 + (it & 1);
      HIPTRY(nd_launch_fill_u64(s->st, nslot(s, slot), kNdNormSlot, 0ull));
      if ((rc = sweep(s, 0, l0.x[a], l0.f, l0.x[b], ND_JACOBI, nslot(s, slot)))) return rc;
      HIPTRY(hipMemcpyAsync(s->h_norm + (size_t)slot * kNdNormSlot, nslot(s, slot),
                            sizeof(unsigned long long) * kNdNormSlot, hipMemcpyDeviceToHost,
                            s->st));
      HIPTRY(hipEventRecord(s->ev_norm[it & 1], s->st));
      bool wait = it < 2 || it >= s->opts.max_iter;
      if (!wait) {
        const double pred = prev * (prev / prev2);
        wait = !(pred > 8.0 * tol);
      }
      if (wait) {
        const int d = decide();
        if (d < 0) return fail(MG_ERR_HIP, "norm read-back failed");
        if (d) break;
      }
      {
        int nx = 0;
        if ((rc = cycle_rest(s, a, b, l0.f, &nx))) return rc;
        cur = nx;
      }
      if (!wait) {
        const int d = decide();
        if (d < 0) return fail(MG_ERR_HIP, "norm read-back failed");
        if (d) {
          cur = a;
          break;
        }
      }
      ++it;
    }
    inf.iters = it;
    inf.abs_resid = rn;
    inf.rel_resid = rn / normf;
    result = l0.x[cur];
  }
  if (s->singular) HIPTRY(nd_launch_remove_mean(s->st, l0.g, result, s->partials));
  HIPTRY(nd_launch_scatter(s->st, l0.g, s->d_box[tp], nbox, s->max_elems[tp], tp, dlo, s->n,
                           result, static_cast<double*>(phi->data)));
  HIPTRY(hipMemcpyAsync(s->h_norm + 3 * kNdNormSlot, s->d_iters, sizeof(int),
                        hipMemcpyDeviceToHost, s->st));
  HIPTRY(hipStreamSynchronize(s->st));
  std::memcpy(&inf.bottom_iters, s->h_norm + 3 * kNdNormSlot, sizeof(int));
  if ((rc = call.finish())) return rc;
  inf.solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

int mg_nodal_apply(mg_nodal_t* s, const mg_multifab_t* phi, mg_multifab_t* out) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  int rc;
  if ((rc = check_mf(s, phi, true, 1, "phi"))) return rc;
  if ((rc = check_mf(s, out, true, 1, "out"))) return rc;
  NdCall call(s);
  if ((rc = call.rc())) return rc;
  NdLevel& l0 = s->L[0];
  const int nbox = (int)s->boxes.size();
  const int dlo[3] = {s->domain.lo[0], s->domain.lo[1], s->domain.lo[2]};
  HIPTRY(nd_launch_gather(s->st, l0.g, s->d_box[phi->ngrow], nbox, s->max_elems[phi->ngrow],
                          phi->ngrow, dlo, static_cast<const double*>(phi->data), l0.x[0]));
  if ((rc = fill_ghosts(s, l0, l0.x[0]))) return rc;
  if ((rc = sweep(s, 0, l0.x[0], l0.f, l0.r, ND_APPLY, nullptr))) return rc;
  HIPTRY(nd_launch_scatter(s->st, l0.g, s->d_box[out->ngrow], nbox, s->max_elems[out->ngrow],
                           out->ngrow, dlo, s->n, l0.r, static_cast<double*>(out->data)));
  return call.finish();
}

int mg_nodal_time_smoother(mg_nodal_t* s, int32_t reps, double* mean_ms) {
  if (!s || reps < 1 || !mean_ms) return fail(MG_ERR_ARG, "bad argument");
  NdCall call(s);
  int rc;
  if ((rc = call.rc())) return rc;
  NdLevel& l0 = s->L[0];
  hipEvent_t a = nullptr, b = nullptr;
  HIPTRY(hipEventCreate(&a));
  HIPTRY(hipEventCreate(&b));
  auto one = [&](int k) {
    return sweep(s, 0, l0.x[k & 1], l0.f, l0.x[1 - (k & 1)], ND_JACOBI, nullptr);
  };
  for (int k = 0; k < 2 && !rc; ++k) rc = one(k);
  if (!rc && hipEventRecord(a, s->st) != hipSuccess) rc = fail(MG_ERR_HIP, "event record");
  for (int k = 0; k < reps && !rc; ++k) rc = one(k);
  if (!rc && hipEventRecord(b, s->st) != hipSuccess) rc = fail(MG_ERR_HIP, "event record");
  float ms = 0.f;
  if (!rc && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
    rc = fail(MG_ERR_HIP, "event timing");
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (rc) return rc;
  *mean_ms = ms / reps;
  return call.finish();
}

int mg_nodal_num_levels(const mg_nodal_t* s, int32_t* nlevels) {
  if (!s || !nlevels) return fail(MG_ERR_ARG, "bad argument");
  *nlevels = (int32_t)s->L.size();
  return MG_OK;
}

void mg_nodal_destroy(mg_nodal_t* s) {
  if (!s) return;
  if (s->st) hipStreamSynchronize(s->st);
  for (hipGraphExec_t g : s->graph)
    if (g) hipGraphExecDestroy(g);
  for (hipEvent_t e : s->ev_norm)
    if (e) hipEventDestroy(e);
  if (s->ev_in) hipEventDestroy(s->ev_in);
  if (s->ev_out) hipEventDestroy(s->ev_out);
  if (s->h_norm) hipHostFree(s->h_norm);
  if (s->st) hipStreamDestroy(s->st);
  delete s;
}

}  // extern "C"
