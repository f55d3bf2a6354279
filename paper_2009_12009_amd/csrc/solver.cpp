// Multigrid driver behind the C ABI: hierarchy and table construction,
// workspace layout, the V-cycle schedule and the solve loop.
//
// Schedule of one V-cycle ("Linear Solvers": geometric multigrid with a CG
// bottom solve).  Level 0 works on the caller's phi in place:
//   nu1 x [exchange, red, exchange, black]; exchange; r = f - A phi;
//   rhs_1 = R r; coarse levels; phi += P e_1; nu2 x [exchange, red, ...]
// A coarse level l solves for a correction e_l from a zero guess (so its
// first red half-sweep reads nothing but rhs_l); the bottom level runs CG.
// The coarse part uses only workspace pointers, so it is captured once into
// a HIP graph and replayed every cycle.  The stop test reads one max-norm
// per cycle back to the host.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/amrmg.h"
#include "host.hpp"
#include "kernels.hpp"
#include "tables.hpp"

using namespace amrmg;

namespace {

#define HIPTRY(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return MG_ERR_HIP;                                                              \
    }                                                                                 \
  } while (0)

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

IBox to_ibox(const mg_box_t& b) {
  IBox r;
  for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d]; r.hi[d] = b.hi[d]; }
  return r;
}

int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

int64_t grown_volume(const IBox& b, int ng, int face_d) {
  int64_t v = 1;
  for (int d = 0; d < 3; ++d) v *= ext(b, d) + 2 * ng + (d == face_d ? 1 : 0);
  return v;
}

// ---------------------------------------------------------------------------
// Workspace: a bump allocator with 256-byte alignment.  The same code runs in
// "measure" mode (base = null) for mg_query_workspace.
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

struct Level {
  std::vector<IBox> boxes;
  IBox domain;
  bool merged = false;
  bool buf = false;  // every box array < 4 GiB (32-bit buffer offsets)
  // box b is the coarsening of box b of the next finer level (level >= 1)
  bool coarsened_1to1 = false;
  // the restriction into this level may fold into its first half-sweep
  // (level 1: only where the tuner measured the folded kernel faster)
  bool fold_rs = true;
  int nbox = 0;
  double h[3];
  int64_t ncell = 0, n_g1 = 0, n_g0 = 0, n_f[3] = {0, 0, 0};
  int max_faces = 0;
  std::vector<BoxInfo> info;
  // tile tables (host) and shapes
  std::vector<Tile> t_gsrb, t_cell, t_rst;
  Shape s_gsrb{32, 8, 16}, s_cell{64, 4, 16}, s_rst{64, 4, 16};
  // level 0: deep tiles for streaming vector kernels (CG updates, dots): the
  // residual's tuned tiles can be a few hundred cells, and a block reduction
  // per tiny tile costs more than the data it covers
  std::vector<Tile> t_vec;
  Shape s_vec{64, 4, 16};
  Tile* d_vec = nullptr;
  // level 0: tiles of the residual pass that writes the restriction into
  // level 1's right-hand side (lx, ly, tz even)
  std::vector<Tile> t_rr;
  Shape s_rr{64, 4, 2, 2};
  Tile* d_rr = nullptr;
  size_t cap_rr = 0;
  size_t cap_gsrb = 0, cap_cell = 0;  // tile slots reserved in the workspace
  // level 0: smoother tile shapes per box class (a box's x extent); empty =
  // one shape for every box (s_gsrb)
  std::map<int, Shape> cls;
  Shape cls_base{32, 8, 16};  // the shape of boxes of other classes (with cls)
  // fused sweeps (both colours in one pass, out of place, rim pass after)
  bool fused = false;
  Shape s_sweep{64, 8, 16};
  std::vector<Tile> t_sweep;
  std::vector<RimTile> t_rim;
  size_t cap_sweep = 0;
  Tile* d_sweep = nullptr;
  RimTile* d_rim = nullptr;
  double* alt64 = nullptr;  // second buffer of the smoothed array (ng 1)
  float* alt32 = nullptr;
  // half-sweeps write updates straight into the face ghosts of other boxes
  bool wt = false;
  std::vector<WtEntry> h_wt;
  std::vector<WtBox> h_wtbox;
  WtEntry* d_wt = nullptr;
  WtBox* d_wtbox = nullptr;
  std::vector<FbTag> tags;
  std::vector<FbChunk> chunks;
  // device
  BoxInfo* d_info = nullptr;
  Tile *d_gsrb = nullptr, *d_cell = nullptr, *d_rst = nullptr;
  FbTag* d_tags = nullptr;
  FbChunk* d_chunks = nullptr;
  double *b64[3] = {nullptr, nullptr, nullptr}, *a64 = nullptr;
  double *e64 = nullptr, *rhs64 = nullptr, *r64 = nullptr;
  double* p64 = nullptr;  // level 0, preconditioned CG: search direction (ng 1)
  double* next64 = nullptr;  // level 0, folded stop test: the other iterate (ng 1)
  float *b32[3] = {nullptr, nullptr, nullptr}, *a32 = nullptr;
  float *e32 = nullptr, *rhs32 = nullptr, *r32 = nullptr;
  // coarse tail (launch_tail): packed cells of a tail level (red, then
  // black) and the restriction entries of this level's residual into the
  // next coarser one (the level above the tail and the tail levels)
  std::vector<unsigned> h_tcells, h_trc;
  int tail_nred = 0;
  unsigned *d_tcells = nullptr, *d_trc = nullptr;
};

struct ProfRec {
  int fam;
  hipEvent_t a, b;
};

}  // namespace

struct mg_solver {
  mg_opts_t opts;
  IBox domain;
  int periodic[3];
  int bc_lo[3], bc_hi[3];
  double alpha, beta;
  bool has_a = false;
  bool singular = false;
  std::vector<Level> L;
  // bottom
  int nb = 0;
  std::vector<int> h_nbr, h_fidx, h_aidx, h_map_rhs, h_map_out;
  int *d_nbr = nullptr, *d_fidx = nullptr, *d_aidx = nullptr, *d_map_rhs = nullptr,
      *d_map_out = nullptr;
  double *bdiag64 = nullptr, *bcoef64 = nullptr, *bwork64 = nullptr;
  float *bdiag32 = nullptr, *bcoef32 = nullptr, *bwork32 = nullptr;
  // scratch
  unsigned long long* d_norm = nullptr;  // 4 norm slots of kNormSlot words
  double* d_cg = nullptr;                // [4] preconditioned CG scalars
  int* d_iters = nullptr;
  double* d_sum = nullptr;
  double* d_partials = nullptr;
  double* tune_scratch = nullptr;
  // runtime
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  hipStream_t user = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_norm[2] = {nullptr, nullptr};  // folded stop test: norm copies landed
  hipGraphExec_t graph64 = nullptr, graph32 = nullptr;
  // the level-0 residual pass writes its restriction into level 1's rhs
  bool rr_fold = false;
  // first level of the coarse tail (-1: none) and its device plan
  int tail_lev = -1;
  char* d_tail = nullptr;
  // pinned: [0, kNormSlot) read_norm; two more slots for the folded stop
  // test's copies in flight; then h_iters
  unsigned long long* h_norm = nullptr;
  int* h_iters = nullptr;
  bool profile = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double setup_ms = 0;
  // two-level composite (fine level over part of the coarse level 0)
  bool composite = false;
  Level F;
  std::vector<Tile> t_fcov;  // coarse cells under each fine box
  Shape s_fcov{64, 4, 16, 1};
  Tile* d_fcov = nullptr;
  std::vector<CfGhost> h_ghost;
  std::vector<CfCell> h_cfcell;
  std::vector<CfFace> h_cfface;
  CfGhost* d_ghost = nullptr;
  CfCell* d_cfcell = nullptr;
  CfFace* d_cfface = nullptr;
  double *Rc = nullptr, *ef = nullptr, *Rf = nullptr, *rf2 = nullptr;
  // FP32 correction of the composite solve (precision MG_PREC_F32_REFINE)
  float *Rc32 = nullptr, *ef32 = nullptr, *Rf32 = nullptr, *rf2_32 = nullptr;
  // flexible GMRES of the composite solve (krylov = 1): restart length,
  // basis (m+1 ghost-free pairs), preconditioned directions (m pairs, ng 1),
  // W = -A z, zero right-hand sides, partial sums, device and pinned scalars
  int gm_m = 20;
  double *gm_Vf = nullptr, *gm_Vc = nullptr, *gm_Zf = nullptr, *gm_Zc = nullptr;
  double *gm_Wf = nullptr, *gm_Wc = nullptr, *gm_zero_f = nullptr, *gm_zero_c = nullptr;
  double *gm_part = nullptr, *d_gm = nullptr, *h_gm = nullptr;
};

// Norm slot k (kNormSlot words) of the solver's norm scratch.
inline unsigned long long* norm_slot(mg_solver* s, int k) {
  return s->d_norm + (size_t)k * kNormSlot;
}

namespace {

// ---------------------------------------------------------------------------
// Plan construction (host only).

void make_tiles(const std::vector<BoxInfo>& info, Shape sh, int tx, bool coarse_of_box,
                std::vector<Tile>& out) {
  out.clear();
  for (int b = 0; b < (int)info.size(); ++b) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = coarse_of_box ? floordiv(info[b].lo[d], 2) : info[b].lo[d];
      hi[d] = coarse_of_box ? floordiv(info[b].hi[d], 2) : info[b].hi[d];
    }
    for (int z = lo[2]; z <= hi[2]; z += sh.tz)
      for (int y = lo[1]; y <= hi[1]; y += sh.ly)
        for (int x = lo[0]; x <= hi[0]; x += tx) out.push_back({b, x, y, z});
  }
  // Work-groups go to the 8 XCDs round robin (block i -> XCD i % 8); place
  // contiguous runs of tiles on one XCD so neighbouring tiles share its L2.
  const size_t n = out.size(), q = n / 8;
  if (q > 0) {
    std::vector<Tile> perm(out);
    for (size_t p = 0; p < 8 * q; ++p) perm[p] = out[(p % 8) * q + p / 8];
    out.swap(perm);
  }
}

Shape shape_gsrb(int nx, int ny, int nz) {
  int lx = std::min(32, std::max(1, pow2ceil((nx + 1) / 2)));
  int ly = std::min(256 / lx, pow2ceil(ny));
  while (lx * ly < 64) ly *= 2;
  return {lx, ly, std::min(16, pow2ceil(nz)), 2};
}
Shape shape_cell(int nx, int ny, int nz) {
  int lx = std::min(64, pow2ceil(nx));
  int ly = std::min(256 / lx, pow2ceil(ny));
  while (lx * ly < 64) ly *= 2;
  return {lx, ly, std::min(16, pow2ceil(nz)), 2};
}

void build_fb(Level& lv, const int periodic[3], int ng) {
  std::vector<int64_t> offs(lv.nbox);
  for (int b = 0; b < lv.nbox; ++b) offs[b] = lv.info[b].off_g1;
  make_fb_tables(lv.boxes, lv.domain, periodic, ng, offs, 1, lv.tags, lv.chunks);
}

void fill_info(Level& lv, const IBox& domain, const int periodic[3]) {
  lv.nbox = (int)lv.boxes.size();
  lv.info.resize(lv.nbox);
  int64_t o1 = 0, o0 = 0, of[3] = {0, 0, 0};
  lv.max_faces = 0;
  for (int b = 0; b < lv.nbox; ++b) {
    BoxInfo& I = lv.info[b];
    const IBox& B = lv.boxes[b];
    int m = 0;
    for (int d = 0; d < 3; ++d) {
      I.lo[d] = B.lo[d];
      I.hi[d] = B.hi[d];
      if (!periodic[d] && B.lo[d] == domain.lo[d]) m |= 1 << (2 * d);
      if (!periodic[d] && B.hi[d] == domain.hi[d]) m |= 1 << (2 * d + 1);
    }
    I.bcmask = m;
    I.parent = b;
    I.off_g1 = o1;
    I.off_g0 = o0;
    o1 += grown_volume(B, 1, -1);
    o0 += volume(B);
    for (int d = 0; d < 3; ++d) {
      I.off_f[d] = of[d];
      const int64_t nf = grown_volume(B, 0, d);
      of[d] += nf;
      lv.max_faces = std::max<int64_t>(lv.max_faces, nf);
    }
  }
  lv.ncell = o0;
  lv.n_g1 = o1;
  lv.n_g0 = o0;
  for (int d = 0; d < 3; ++d) lv.n_f[d] = of[d];
}

bool shape_ok(Shape sh) {
  const int t = sh.lx * sh.ly;
  return sh.lx >= 1 && sh.ly >= 1 && sh.tz >= 1 && t >= 64 && t <= 256 && t % 64 == 0;
}

// Tile shapes the tuner times for the level-0 smoother and residual.
std::vector<Shape> gsrb_candidates() {
  std::vector<Shape> c;
  for (int lx : {16, 32, 64})
    for (int ly : {1, 2, 4, 8, 16})
      for (int tz : {1, 2, 4, 8, 16, 32, 64})
        for (int u : {1, 2, 4})
          for (int wp : {0, 1})
            if (shape_ok({lx, ly, tz, u}) && u <= tz) c.push_back({lx, ly, tz, u, wp});
  return c;
}
// FP32 smoother tiles with one x-quad per lane (streaming levels only).
std::vector<Shape> quad_candidates() {
  std::vector<Shape> c;
  for (int lx : {8, 16, 32})
    for (int ly : {2, 4, 8, 16, 32})
      for (int tz : {1, 2, 4, 8})
        for (int u : {1, 2})
          if (shape_ok({lx, ly, tz, u}) && u <= tz) c.push_back({lx, ly, tz, u, 2});
  return c;
}
std::vector<Shape> cell_candidates() {
  std::vector<Shape> c;
  for (int lx : {32, 64, 128})
    for (int ly : {1, 2, 4, 8})
      for (int tz : {1, 2, 4, 8, 16, 32, 64})
        for (int u : {1, 2, 4})
          if (shape_ok({lx, ly, tz, u}) && u <= tz) c.push_back({lx, ly, tz, u});
  return c;
}

// tiles of the fused residual-restriction pass: lx, ly, tz even
std::vector<Shape> rr_candidates() {
  std::vector<Shape> c;
  for (Shape sh : cell_candidates())
    if (sh.lx >= 2 && sh.lx % 2 == 0 && sh.ly % 2 == 0 && sh.tz % 2 == 0 && sh.u == 2)
      c.push_back(sh);
  return c;
}

std::vector<Shape> sweep_candidates() {
  std::vector<Shape> c;
  for (int lx : {32, 64})
    for (int ly : {2, 4, 8, 16})
      for (int tz : {4, 8, 16, 32})
        if (sweep_lds_bytes({lx, ly, tz}, sizeof(double))) c.push_back({lx, ly, tz});
  return c;
}

Shape shape_sweep(int nx) { return nx >= 64 ? Shape{64, 8, 16} : Shape{32, 8, 8}; }

// The boundary layer of every box, as blocks of <= 256 cells: the two z
// faces, then the two y faces without their z-edge rows, then the two x faces
// without any edge.  Blocks of a face are x-rows, or y-columns of the x faces.
void make_rim_tiles(const std::vector<BoxInfo>& info, std::vector<RimTile>& out) {
  out.clear();
  auto emit = [&](int b, int i0, int j0, int k0, int ni, int nj, int nk) {
    if (ni <= 0 || nj <= 0 || nk <= 0) return;
    const int px = std::min(ni, 256);
    const int ry = std::min(nj, 256 / px);
    const int rz = ry == nj ? std::max(1, std::min(nk, 256 / (px * nj))) : 1;
    for (int k = 0; k < nk; k += rz)
      for (int j = 0; j < nj; j += ry)
        for (int i = 0; i < ni; i += px)
          out.push_back({b, i0 + i, j0 + j, k0 + k, std::min(px, ni - i), std::min(ry, nj - j),
                         std::min(rz, nk - k), 0});
  };
  for (int b = 0; b < (int)info.size(); ++b) {
    const BoxInfo& B = info[b];
    const int nx = B.hi[0] - B.lo[0] + 1, ny = B.hi[1] - B.lo[1] + 1, nz = B.hi[2] - B.lo[2] + 1;
    emit(b, 0, 0, 0, nx, ny, 1);
    if (nz > 1) emit(b, 0, 0, nz - 1, nx, ny, 1);
    emit(b, 0, 0, 1, nx, 1, nz - 2);
    if (ny > 1) emit(b, 0, ny - 1, 1, nx, 1, nz - 2);
    emit(b, 0, 1, 1, 1, ny - 2, nz - 2);
    if (nx > 1) emit(b, nx - 1, 1, 1, 1, ny - 2, nz - 2);
  }
}

size_t tile_count(const std::vector<BoxInfo>& info, Shape sh, int tx) {
  size_t n = 0;
  for (const BoxInfo& b : info) {
    const size_t nx = (b.hi[0] - b.lo[0] + tx) / tx;
    const size_t ny = (b.hi[1] - b.lo[1] + sh.ly) / sh.ly;
    const size_t nz = (b.hi[2] - b.lo[2] + sh.tz) / sh.tz;
    n += nx * ny * nz;
  }
  return n;
}

size_t tile_count_c(const std::vector<BoxInfo>& info, Shape sh, int tx, bool coarse) {
  size_t n = 0;
  for (const BoxInfo& b : info) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = coarse ? floordiv(b.lo[d], 2) : b.lo[d];
      hi[d] = coarse ? floordiv(b.hi[d], 2) : b.hi[d];
    }
    n += (size_t)((hi[0] - lo[0] + tx) / tx) * ((hi[1] - lo[1] + sh.ly) / sh.ly) *
         ((hi[2] - lo[2] + sh.tz) / sh.tz);
  }
  return n;
}

Shape fit_tz(const std::vector<BoxInfo>& info, Shape sh, int xmul, bool coarse) {
  while (sh.tz > 1 && tile_count_c(info, sh, xmul * sh.lx, coarse) < 2048) sh.tz /= 2;
  return sh;
}

// ---------------------------------------------------------------------------
// Smoother tile shapes per box class.  A class is a box's x extent (the
// direction a wavefront's lanes run along, where a tile wider than the box
// leaves lanes idle); all classes of a launch share its thread count, unroll
// and whole-pair choice, and each tile carries its class's lane layout and
// depth (Tile::shape).

int pack_shape(Shape sh) { return __builtin_ctz((unsigned)sh.lx) | (sh.ly << 4) | (sh.tz << 16); }

// Candidate class shapes for a launch of `threads` threads and unroll u.
std::vector<Shape> class_candidates(int threads, int u, int wp) {
  std::vector<Shape> c;
  for (int lx : {16, 32, 64}) {
    const int ly = threads / lx;
    if (ly < 1 || lx * ly != threads || ly > 255) continue;
    for (int tz : {1, 2, 4, 8, 16})
      if (u <= tz) c.push_back({lx, ly, tz, u, wp});
  }
  return c;
}

// Tiles of the boxes in `only` (all boxes when empty) with each box's class
// shape (dflt for classes not in cls), in the XCD-grouped order of
// make_tiles.
void make_class_tiles(const std::vector<BoxInfo>& info, const std::map<int, Shape>& cls, Shape dflt,
                      const std::vector<int>& only, std::vector<Tile>& out) {
  out.clear();
  std::vector<int> boxes = only;
  if (boxes.empty())
    for (int b = 0; b < (int)info.size(); ++b) boxes.push_back(b);
  for (int b : boxes) {
    const int nx = info[b].hi[0] - info[b].lo[0] + 1;
    auto it = cls.find(nx);
    const Shape sh = it == cls.end() ? dflt : it->second;
    const int code = pack_shape(sh);
    for (int z = info[b].lo[2]; z <= info[b].hi[2]; z += sh.tz)
      for (int y = info[b].lo[1]; y <= info[b].hi[1]; y += sh.ly)
        for (int x = info[b].lo[0]; x <= info[b].hi[0]; x += 2 * sh.lx)
          out.push_back({b, x, y, z, code});
  }
  const size_t n = out.size(), q = n / 8;
  if (q > 0) {
    std::vector<Tile> perm(out);
    for (size_t p = 0; p < 8 * q; ++p) perm[p] = out[(p % 8) * q + p / 8];
    out.swap(perm);
  }
}

// The launch shape of a class table: dflt's lanes, unroll and whole pairs,
// tz raised so that the write-through's LDS (2 ly tz values) fits every class.
Shape class_launch_shape(const std::map<int, Shape>& cls, Shape dflt) {
  int need = dflt.ly * dflt.tz;
  for (const auto& kv : cls) need = std::max(need, kv.second.ly * kv.second.tz);
  Shape l = dflt;
  l.tz = (need + dflt.ly - 1) / dflt.ly;
  return l;
}

// Write-through tables of a level: for every copy tag of the one-layer
// exchange, the part of its destination region on one of the destination
// box's six face-ghost slabs (edges and corners are never read by the
// 7-point kernels) becomes an entry of the source box's opposite face.
bool make_wt_tables(Level& lv, const int periodic[3]) {
  std::vector<CopyTag> tags = copy_tags(lv.boxes, lv.domain, periodic, 1);
  std::vector<std::vector<WtEntry>> per(lv.nbox * 6);
  for (const CopyTag& t : tags) {
    const IBox& D = lv.boxes[t.dst];
    const IBox& S = lv.boxes[t.src];
    const BoxInfo& DI = lv.info[t.dst];
    const long long dsy = ext(D, 0) + 2, dsz = dsy * (ext(D, 1) + 2);
    for (int d = 0; d < 3; ++d)
      for (int side = 0; side < 2; ++side) {
        IBox slab = D;
        slab.lo[d] = slab.hi[d] = side ? D.hi[d] + 1 : D.lo[d] - 1;
        const IBox r = intersect(t.region, slab);
        if (!ok(r)) continue;
        WtEntry e;
        for (int a = 0; a < 3; ++a) {
          e.lo[a] = r.lo[a] - t.shift[a] - S.lo[a];
          e.hi[a] = r.hi[a] - t.shift[a] - S.lo[a];
        }
        // the source cells sit on the source box's face opposite to the slab
        const int sf = 2 * d + (side ? 0 : 1);
        e.base = DI.off_g1 + (S.lo[0] + t.shift[0] - D.lo[0] + 1) +
                 (S.lo[1] + t.shift[1] - D.lo[1] + 1) * dsy +
                 (S.lo[2] + t.shift[2] - D.lo[2] + 1) * dsz;
        e.sy = (int)dsy;
        e.sz = (int)dsz;
        // every target must be a face ghost of the destination's grown array
        const long long first = e.base + e.lo[0] + e.lo[1] * dsy + e.lo[2] * dsz;
        const long long last = e.base + e.hi[0] + e.hi[1] * dsy + e.hi[2] * dsz;
        const long long end = DI.off_g1 + grown_volume(D, 1, -1);
        const bool src_face = side ? (e.lo[d] == 0 && e.hi[d] == 0)
                                   : (e.lo[d] == ext(S, d) - 1 && e.hi[d] == ext(S, d) - 1);
        if (first < DI.off_g1 || last >= end || !src_face) return false;
        per[t.src * 6 + sf].push_back(e);
      }
  }
  lv.h_wt.clear();
  lv.h_wtbox.assign(lv.nbox, WtBox{});
  for (int b = 0; b < lv.nbox; ++b)
    for (int f = 0; f < 6; ++f) {
      lv.h_wtbox[b].first[f] = (int)lv.h_wt.size();
      lv.h_wtbox[b].count[f] = (int)per[b * 6 + f].size();
      for (const WtEntry& e : per[b * 6 + f]) lv.h_wt.push_back(e);
    }
  return true;
}

// Builds every host table; with a Bump in measure mode it also lays out the
// workspace.  Returns 0 or an error code.
// Whether FP64 V-cycle solves fold the stop test's residual into the next
// cycle's first half-sweep (needs the level hierarchy: call after it is set).
bool stop_fold_on(const mg_solver* s) {
  return s->opts.stop_fold && s->opts.precision == MG_PREC_F64 && !s->opts.krylov &&
         !s->composite && s->opts.nu1 >= 1 && s->L.size() > 1 && !s->L[0].fused;
}

// LDS bytes of the tail kernel starting at level t: the bottom CG's p (FP64
// at most), BoxInfo of the level above, of every tail level and of the
// bottom, WtBox of every tail level; offsets into *tp when given.
template <typename T>
size_t tail_lds_layout(const mg_solver* s, int t, TailPlan<T>* tp) {
  const int nl = (int)s->L.size();
  size_t off = (sizeof(double) * (size_t)s->L.back().ncell + 15) & ~size_t(15);
  if (tp) tp->lds_fi = (int)off;
  off += sizeof(BoxInfo) * s->L[t - 1].info.size();
  for (int l = t; l <= nl - 1; ++l) {
    if (tp) tp->lds_bi[l - t] = (int)off;
    off += sizeof(BoxInfo) * s->L[l].info.size();
  }
  for (int l = t; l <= nl - 2; ++l) {
    if (tp) tp->lds_wb[l - t] = (int)off;
    off += sizeof(WtBox) * s->L[l].info.size();
  }
  if (tp) tp->lds_bytes = (int)off;
  return off;
}

size_t tail_lds_need(const mg_solver* s, int t) {
  return tail_lds_layout<double>(s, t, nullptr);
}

// The first level of the coarse tail: the levels from it down to the
// bottom each hold at most opts.coarse_tail cells and are half-swept with
// write-through (so are not the bottom), the bottom is a CG of at most
// kTailMaxBottom cells, and the entries pack (box extents, box counts; the
// level above the tail packs restriction entries, half its extents).
// -1: no tail.
int choose_tail(const mg_solver* s) {
  const int nl = (int)s->L.size();
  if (s->opts.coarse_tail <= 0 || nl < 3 || s->opts.bottom_solver != 0 || s->opts.nu1 < 1 ||
      s->L.back().ncell > kTailMaxBottom)
    return -1;
  auto packs = [](const Level& lv, int max_extent) {
    if (lv.nbox >= kTailMaxBoxes) return false;
    for (const BoxInfo& b : lv.info)
      for (int d = 0; d < 3; ++d)
        if (b.hi[d] - b.lo[d] + 1 > max_extent) return false;
    return true;
  };
  int start = nl - 1;
  for (int l = nl - 2; l >= 1; --l) {
    const Level& lv = s->L[l];
    if (lv.ncell > s->opts.coarse_tail || !lv.wt || lv.fused || !packs(lv, kTailMaxExtent)) break;
    start = l;
  }
  start = std::max(start, nl - 1 - kTailMaxLevels);
  // the staged box tables must fit the kernel's LDS: start lower if not
  while (start <= nl - 2 && tail_lds_need(s, start) > kTailMaxLds) ++start;
  if (start > nl - 2) return -1;
  if (!packs(s->L[start - 1], 2 * kTailMaxExtent)) return -1;
  return start;
}

unsigned tail_pack(int b, int i, int j, int k) {
  return (unsigned)k | ((unsigned)j << 6) | ((unsigned)i << 12) | ((unsigned)b << 18);
}

void build_tail_tables(mg_solver* s) {
  for (Level& lv : s->L) {
    lv.h_tcells.clear();
    lv.h_trc.clear();
    lv.tail_nred = 0;
  }
  const int t = s->tail_lev;
  if (t < 1) return;
  const int nl = (int)s->L.size();
  for (int l = t; l <= nl - 2; ++l) {
    Level& lv = s->L[l];
    std::vector<unsigned> black;
    for (int b = 0; b < lv.nbox; ++b) {
      const BoxInfo& I = lv.info[b];
      for (int k = I.lo[2]; k <= I.hi[2]; ++k)
        for (int j = I.lo[1]; j <= I.hi[1]; ++j)
          for (int i = I.lo[0]; i <= I.hi[0]; ++i) {
            const unsigned e = tail_pack(b, i - I.lo[0], j - I.lo[1], k - I.lo[2]);
            ((i + j + k) & 1 ? black : lv.h_tcells).push_back(e);
          }
    }
    lv.tail_nred = (int)lv.h_tcells.size();
    lv.h_tcells.insert(lv.h_tcells.end(), black.begin(), black.end());
  }
  for (int l = t - 1; l <= nl - 2; ++l) {
    Level& lv = s->L[l];
    for (int b = 0; b < lv.nbox; ++b) {
      const BoxInfo& F = lv.info[b];
      int clo[3], chi[3];
      for (int d = 0; d < 3; ++d) {
        clo[d] = floordiv(F.lo[d], 2);
        chi[d] = floordiv(F.hi[d], 2);
      }
      for (int k = clo[2]; k <= chi[2]; ++k)
        for (int j = clo[1]; j <= chi[1]; ++j)
          for (int i = clo[0]; i <= chi[0]; ++i)
            lv.h_trc.push_back(tail_pack(b, i - clo[0], j - clo[1], k - clo[2]));
    }
  }
}

int build_plan(mg_solver* s, const std::vector<IBox>& boxes, Bump& bump) {
  std::string err;
  if (!validate_boxes(boxes, s->domain, true, &err)) return fail(MG_ERR_INVALID_BOXARRAY, err);
  for (const IBox& b : boxes)
    if (grown_volume(b, 1, 0) >= (int64_t(1) << 31))
      return fail(MG_ERR_INVALID_BOXARRAY, "a box holds 2^31 or more cells; split it");
  std::vector<LevelBoxes> hb =
      hierarchy(boxes, s->domain, s->opts.min_bottom_edge, s->opts.aggregate != 0);
  s->L.clear();
  s->L.resize(hb.size());
  const int n[3] = {ext(s->domain, 0), ext(s->domain, 1), ext(s->domain, 2)};
  for (size_t l = 0; l < hb.size(); ++l) {
    Level& lv = s->L[l];
    lv.boxes = hb[l].boxes;
    lv.domain = hb[l].domain;
    lv.merged = hb[l].merged;
    for (int d = 0; d < 3; ++d) lv.h[d] = 0;  // set by caller from geometry
    fill_info(lv, lv.domain, s->periodic);
    int mx[3] = {1, 1, 1};
    for (const IBox& b : lv.boxes)
      for (int d = 0; d < 3; ++d) mx[d] = std::max(mx[d], ext(b, d));
    // z-depth of a tile: as deep as 16 planes while the level still gets
    // >= 2048 work-groups (8 per CU); coarse levels use shallow tiles so that
    // their launches are not a handful of long serial z-marches
    lv.s_gsrb = fit_tz(lv.info, shape_gsrb(mx[0], mx[1], mx[2]), 2, false);
    lv.s_cell = fit_tz(lv.info, shape_cell(mx[0], mx[1], mx[2]), 1, false);
    lv.s_rst = fit_tz(lv.info,
                      shape_cell(std::max(1, mx[0] / 2), std::max(1, mx[1] / 2), std::max(1, mx[2] / 2)),
                      1, true);
    make_tiles(lv.info, lv.s_gsrb, gsrb_tx(lv.s_gsrb), false, lv.t_gsrb);
    make_tiles(lv.info, lv.s_cell, lv.s_cell.lx, false, lv.t_cell);
    if (l + 1 < hb.size()) make_tiles(lv.info, lv.s_rst, lv.s_rst.lx, true, lv.t_rst);
    if (l == 0) {
      lv.s_vec = fit_tz(lv.info, shape_cell(mx[0], mx[1], mx[2]), 1, false);
      make_tiles(lv.info, lv.s_vec, lv.s_vec.lx, false, lv.t_vec);
      const int rlx = std::max(2, std::min(64, pow2ceil(mx[0])));
      lv.s_rr = Shape{rlx, std::max(2, std::min(256 / rlx, 4)), 2, 2};
      lv.t_rr.clear();
      if (hb.size() >= 2) make_tiles(lv.info, lv.s_rr, lv.s_rr.lx, false, lv.t_rr);
      lv.cap_rr = lv.t_rr.size();
      if (hb.size() >= 2)
        for (Shape c : rr_candidates())
          lv.cap_rr = std::max(lv.cap_rr, tile_count(lv.info, c, c.lx));
    }
    build_fb(lv, s->periodic, 1);
    lv.cap_gsrb = lv.t_gsrb.size();
    lv.cap_cell = lv.t_cell.size();
    if (l <= 1) {
      for (Shape c : gsrb_candidates())
        lv.cap_gsrb = std::max(lv.cap_gsrb, tile_count(lv.info, c, gsrb_tx(c)));
      if (l == 0)
        for (Shape c : quad_candidates())
          lv.cap_gsrb = std::max(lv.cap_gsrb, tile_count(lv.info, c, gsrb_tx(c)));
      if (l == 0) {
        // class tables: every box may take any class candidate of any thread count
        size_t per_box = 0;
        for (const BoxInfo& b : lv.info) {
          size_t m = 0;
          for (int th : {64, 128, 256})
            for (Shape c : class_candidates(th, 1, 0)) {
              std::vector<BoxInfo> one{b};
              m = std::max(m, tile_count(one, c, 2 * c.lx));
            }
          for (Shape c : gsrb_candidates()) {
            std::vector<BoxInfo> one{b};
            m = std::max(m, tile_count(one, c, 2 * c.lx));
          }
          per_box += m;
        }
        lv.cap_gsrb = std::max(lv.cap_gsrb, per_box);
      }
      for (Shape c : cell_candidates())
        lv.cap_cell = std::max(lv.cap_cell, tile_count(lv.info, c, c.lx));
    }
    int mn = 1 << 30;
    for (const IBox& b : lv.boxes)
      for (int d = 0; d < 3; ++d) mn = std::min(mn, ext(b, d));
    // small boxes leave most cells to the rim pass; opts.fused_min_edge says
    // how small is too small
    lv.fused = s->opts.fused_min_edge > 0 && l + 1 < hb.size() && mn >= s->opts.fused_min_edge;
    // write-through keeps the colours apart only if they alternate across
    // every periodic wrap
    bool even = true;
    for (int d = 0; d < 3; ++d)
      if (s->periodic[d] && ext(lv.domain, d) % 2) even = false;
    lv.wt = s->opts.ghost_write && !lv.fused && l + 1 < hb.size() && even;
    // largest array of a box: cells with one ghost layer, FP64
    long long big = 0;
    for (const IBox& b : lv.boxes)
      big = std::max(big, (long long)(ext(b, 0) + 2) * (ext(b, 1) + 2) * (ext(b, 2) + 2));
    lv.buf = big * 8 < (1ll << 32);
    if (lv.wt && !make_wt_tables(lv, s->periodic))
      return fail(MG_ERR_INVALID_BOXARRAY, "write-through table outside a box's ghost layer");
    if (lv.fused) {
      lv.s_sweep = shape_sweep(mx[0]);
      make_tiles(lv.info, lv.s_sweep, lv.s_sweep.lx, false, lv.t_sweep);
      make_rim_tiles(lv.info, lv.t_rim);
      lv.cap_sweep = lv.t_sweep.size();
      if (l == 0)
        for (Shape c : sweep_candidates())
          lv.cap_sweep = std::max(lv.cap_sweep, tile_count(lv.info, c, c.lx));
    }
  }
  (void)n;
  // parent links: box b of level l -> box of level l+1 holding coarsen(b)
  for (size_t l = 0; l + 1 < s->L.size(); ++l)
    for (int b = 0; b < s->L[l].nbox; ++b) s->L[l].info[b].parent = s->L[l + 1].merged ? 0 : b;
  for (size_t l = 1; l < s->L.size(); ++l) {
    const Level& f = s->L[l - 1];
    Level& c = s->L[l];
    bool one = !c.merged && c.nbox == f.nbox;
    for (int b = 0; one && b < c.nbox; ++b)
      for (int d = 0; d < 3; ++d)
        one = one && f.info[b].parent == b && f.info[b].lo[d] % 2 == 0 &&
              f.info[b].hi[d] % 2 != 0 && c.info[b].lo[d] * 2 == f.info[b].lo[d] &&
              c.info[b].hi[d] * 2 + 1 == f.info[b].hi[d];
    c.coarsened_1to1 = one;
    // level 1 restricts the finest residual, read from HBM: there the folded
    // kernel costs about what the two passes cost together (FP64 a few per
    // cent more), so it runs only where the tuner measured it faster
    c.fold_rs = l >= 2;
  }

  // the level-0 residual restricts as it goes: every level-0 box splits
  // into whole 2x2x2 blocks (true whenever there is a level 1)
  s->rr_fold = s->L.size() >= 2 && s->opts.restrict_fold >= 1 && !s->composite;
  for (const BoxInfo& b : s->L[0].info)
    for (int d = 0; d < 3; ++d)
      if (((b.lo[d] % 2) + 2) % 2 != 0 || (b.hi[d] - b.lo[d] + 1) % 2 != 0) s->rr_fold = false;
  s->tail_lev = choose_tail(s);
  build_tail_tables(s);

  // bottom tables: cells of the bottom level enumerated box by box, x fastest
  Level& bl = s->L.back();
  s->nb = (int)bl.ncell;
  const int nb = s->nb;
  s->h_nbr.assign(6 * (size_t)nb, -1);
  s->h_fidx.assign(6 * (size_t)nb, 0);
  s->h_aidx.assign(nb, 0);
  s->h_map_rhs.assign(nb, 0);
  s->h_map_out.assign(nb, 0);
  {
    const IBox& D = bl.domain;
    const int gn[3] = {ext(D, 0), ext(D, 1), ext(D, 2)};
    std::vector<int> gmap((size_t)gn[0] * gn[1] * gn[2], -1);
    int c = 0;
    for (int b = 0; b < bl.nbox; ++b) {
      const IBox& B = bl.boxes[b];
      for (int k = B.lo[2]; k <= B.hi[2]; ++k)
        for (int j = B.lo[1]; j <= B.hi[1]; ++j)
          for (int i = B.lo[0]; i <= B.hi[0]; ++i)
            gmap[(i - D.lo[0]) + (size_t)gn[0] * ((j - D.lo[1]) + (size_t)gn[1] * (k - D.lo[2]))] =
                c++;
    }
    c = 0;
    for (int b = 0; b < bl.nbox; ++b) {
      const IBox& B = bl.boxes[b];
      const BoxInfo& I = bl.info[b];
      const int nx = ext(B, 0), ny = ext(B, 1);
      for (int k = B.lo[2]; k <= B.hi[2]; ++k)
        for (int j = B.lo[1]; j <= B.hi[1]; ++j)
          for (int i = B.lo[0]; i <= B.hi[0]; ++i, ++c) {
            const int il = i - B.lo[0], jl = j - B.lo[1], kl = k - B.lo[2];
            const int64_t g0 = il + (int64_t)nx * (jl + (int64_t)ny * kl);
            s->h_aidx[c] = (int)(I.off_g0 + g0);
            s->h_map_rhs[c] = (int)(I.off_g0 + g0);
            s->h_map_out[c] =
                (int)(I.off_g1 + (il + 1) + (int64_t)(nx + 2) * ((jl + 1) + (int64_t)(ny + 2) * (kl + 1)));
            const int p[3] = {i, j, k};
            const int loc[3] = {il, jl, kl};
            for (int f = 0; f < 6; ++f) {
              const int d = f >> 1, side = f & 1;
              // face element index in b_d of this box
              int fl[3] = {loc[0], loc[1], loc[2]};
              fl[d] += side;
              const int fnx = nx + (d == 0), fny = ny + (d == 1);
              s->h_fidx[(size_t)f * nb + c] =
                  (int)(I.off_f[d] + fl[0] + (int64_t)fnx * (fl[1] + (int64_t)fny * fl[2]));
              int q[3] = {p[0], p[1], p[2]};
              q[d] += side ? 1 : -1;
              if (q[d] < D.lo[d] || q[d] > D.hi[d]) {
                if (!s->periodic[d]) continue;  // wall: -1
                q[d] = q[d] < D.lo[d] ? D.hi[d] : D.lo[d];
              }
              s->h_nbr[(size_t)f * nb + c] =
                  gmap[(q[0] - D.lo[0]) + (size_t)gn[0] * ((q[1] - D.lo[1]) + (size_t)gn[1] * (q[2] - D.lo[2]))];
            }
          }
    }
  }

  // workspace layout
  const bool f32 = s->opts.precision == MG_PREC_F32_REFINE;
  const size_t nlev = s->L.size();
  for (size_t l = 0; l < nlev; ++l) {
    Level& lv = s->L[l];
    lv.d_info = bump.take<BoxInfo>(lv.info.size());
    lv.d_gsrb = bump.take<Tile>(lv.cap_gsrb);
    lv.d_cell = bump.take<Tile>(lv.cap_cell);
    lv.d_rst = bump.take<Tile>(lv.t_rst.size());
    lv.d_tags = bump.take<FbTag>(lv.tags.size());
    lv.d_chunks = bump.take<FbChunk>(lv.chunks.size());
    for (int d = 0; d < 3; ++d) lv.b64[d] = bump.take<double>(lv.n_f[d]);
    if (s->has_a) lv.a64 = bump.take<double>(lv.n_g0);
    const bool bottom = l + 1 == nlev;
    if (l == 0) {
      lv.r64 = bump.take<double>(lv.n_g0);
      if (s->composite || s->opts.krylov) {
        lv.e64 = bump.take<double>(lv.n_g1);
        lv.rhs64 = bump.take<double>(lv.n_g0);
      }
      if (s->opts.krylov) lv.p64 = bump.take<double>(lv.n_g1);
      if (stop_fold_on(s)) lv.next64 = bump.take<double>(lv.n_g1);
    } else if (!f32) {
      lv.e64 = bump.take<double>(lv.n_g1);
      lv.rhs64 = bump.take<double>(lv.n_g0);
      if (!bottom) lv.r64 = bump.take<double>(lv.n_g0);
    }
    if (l == 0) {
      lv.d_vec = bump.take<Tile>(lv.t_vec.size());
      lv.d_rr = lv.t_rr.empty() ? nullptr : bump.take<Tile>(lv.cap_rr);
    }
    if (lv.wt) {
      lv.d_wt = bump.take<WtEntry>(std::max<size_t>(1, lv.h_wt.size()));
      lv.d_wtbox = bump.take<WtBox>(lv.h_wtbox.size());
    }
    lv.d_tcells = lv.h_tcells.empty() ? nullptr : bump.take<unsigned>(lv.h_tcells.size());
    lv.d_trc = lv.h_trc.empty() ? nullptr : bump.take<unsigned>(lv.h_trc.size());
    if (lv.fused) {
      lv.d_sweep = bump.take<Tile>(lv.cap_sweep);
      lv.d_rim = bump.take<RimTile>(lv.t_rim.size());
      // the array each precision smooths on this level gets a twin
      if (!f32 || (l == 0 && s->composite)) lv.alt64 = bump.take<double>(lv.n_g1);
      if (f32) lv.alt32 = bump.take<float>(lv.n_g1);
    }
    if (f32) {
      for (int d = 0; d < 3; ++d) lv.b32[d] = bump.take<float>(lv.n_f[d]);
      if (s->has_a) lv.a32 = bump.take<float>(lv.n_g0);
      lv.e32 = bump.take<float>(lv.n_g1);
      lv.rhs32 = bump.take<float>(lv.n_g0);
      if (!bottom) lv.r32 = bump.take<float>(lv.n_g0);
    }
  }
  s->d_nbr = bump.take<int>(6 * (size_t)nb);
  s->d_fidx = bump.take<int>(6 * (size_t)nb);
  s->d_aidx = bump.take<int>(nb);
  s->d_map_rhs = bump.take<int>(nb);
  s->d_map_out = bump.take<int>(nb);
  if (f32) {
    s->bdiag32 = bump.take<float>(nb);
    s->bcoef32 = bump.take<float>(6 * (size_t)nb);
    s->bwork32 = bump.take<float>(7 * (size_t)nb);  // CG 4 n, BiCGStab 7 n
  } else {
    s->bdiag64 = bump.take<double>(nb);
    s->bcoef64 = bump.take<double>(6 * (size_t)nb);
    s->bwork64 = bump.take<double>(7 * (size_t)nb);  // CG 4 n, BiCGStab 7 n
  }
  s->d_norm = bump.take<unsigned long long>(4 * kNormSlot);
  s->d_cg = bump.take<double>(4);
  s->d_iters = bump.take<int>(4);
  s->d_sum = bump.take<double>(2);
  s->d_partials =
      bump.take<double>(std::max<size_t>({1, s->L[0].cap_cell, s->L[0].t_vec.size()}));
  if (s->opts.tune == 2) s->tune_scratch = bump.take<double>(s->L[0].n_g1);
  s->d_tail = s->tail_lev > 0 ? bump.take<char>(sizeof(TailPlan<double>)) : nullptr;
  s->ws_need = bump.off + 256;
  return MG_OK;
}

int check_geom(const mg_geom_t* geom, const int32_t* bc_lo, const int32_t* bc_hi, mg_solver* s) {
  if (!geom) return fail(MG_ERR_ARG, "geometry is null");
  s->domain = to_ibox(geom->domain);
  if (!ok(s->domain)) return fail(MG_ERR_ARG, "empty domain");
  for (int d = 0; d < 3; ++d) {
    s->periodic[d] = geom->is_periodic[d] ? 1 : 0;
    const int lo = bc_lo ? bc_lo[d] : (s->periodic[d] ? MG_BC_PERIODIC : MG_BC_DIRICHLET0);
    const int hi = bc_hi ? bc_hi[d] : (s->periodic[d] ? MG_BC_PERIODIC : MG_BC_DIRICHLET0);
    if (lo != MG_BC_PERIODIC && lo != MG_BC_DIRICHLET0) return fail(MG_ERR_ARG, "bad bc_lo");
    if (hi != MG_BC_PERIODIC && hi != MG_BC_DIRICHLET0) return fail(MG_ERR_ARG, "bad bc_hi");
    if ((lo == MG_BC_PERIODIC) != (s->periodic[d] != 0) ||
        (hi == MG_BC_PERIODIC) != (s->periodic[d] != 0))
      return fail(MG_ERR_ARG, "bc must be MG_BC_PERIODIC exactly in the periodic directions");
    s->bc_lo[d] = lo;
    s->bc_hi[d] = hi;
    if (!(geom->prob_hi[d] > geom->prob_lo[d])) return fail(MG_ERR_ARG, "prob_hi <= prob_lo");
  }
  return MG_OK;
}

void set_h(mg_solver* s, const mg_geom_t* geom) {
  for (size_t l = 0; l < s->L.size(); ++l)
    for (int d = 0; d < 3; ++d)
      s->L[l].h[d] = (geom->prob_hi[d] - geom->prob_lo[d]) / ext(s->L[l].domain, d);
}

template <typename T>
StencilArgs<T> stencil_of(const mg_solver* s, const Level& lv, bool f32) {
  StencilArgs<T> op;
  op.boxes = lv.d_info;
  if (f32) {
    op.a = (const T*)lv.a32;
    op.b0 = (const T*)lv.b32[0];
    op.b1 = (const T*)lv.b32[1];
    op.b2 = (const T*)lv.b32[2];
  } else {
    op.a = (const T*)lv.a64;
    op.b0 = (const T*)lv.b64[0];
    op.b1 = (const T*)lv.b64[1];
    op.b2 = (const T*)lv.b64[2];
  }
  op.alpha = (T)s->alpha;
  op.beta = (T)s->beta;
  op.ih0 = (T)(1.0 / (lv.h[0] * lv.h[0]));
  op.ih1 = (T)(1.0 / (lv.h[1] * lv.h[1]));
  op.ih2 = (T)(1.0 / (lv.h[2] * lv.h[2]));
  // phi (read and written), f and three face arrays against the 256 MiB
  // last-level cache
  op.buf = lv.buf && 6.0 * sizeof(T) * (double)lv.n_g0 > 256.0 * (1 << 20) ? 1 : 0;
  return op;
}

BottomTables bottom_tables(const mg_solver* s) {
  BottomTables bt;
  bt.n = s->nb;
  bt.nbr = s->d_nbr;
  bt.fidx = s->d_fidx;
  bt.aidx = s->d_aidx;
  bt.map_rhs = s->d_map_rhs;
  bt.map_out = s->d_map_out;
  return bt;
}

// MultiFab check: same boxes, the canonical packing for (ngrow, ixtype).
int check_mf(const mg_solver* s, const mg_multifab_t* mf, int want_dtype, int ng_min, int ng_max,
             int face_d, const char* what) {
  if (!mf) return fail(MG_ERR_ARG, std::string(what) + " is null");
  const Level& lv = s->L[0];
  if (mf->nbox != lv.nbox || !mf->boxes || !mf->offsets || !mf->data)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": box count or pointers differ");
  if (mf->dtype != want_dtype) return fail(MG_ERR_MISMATCH, std::string(what) + ": wrong dtype");
  if (mf->ncomp != 1) return fail(MG_ERR_MISMATCH, std::string(what) + ": ncomp must be 1");
  if (mf->ngrow < ng_min || mf->ngrow > ng_max)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": unsupported ngrow");
  for (int d = 0; d < 3; ++d)
    if (mf->ixtype[d] != (d == face_d ? 1 : 0))
      return fail(MG_ERR_MISMATCH, std::string(what) + ": wrong index type");
  int64_t off = 0;
  for (int b = 0; b < lv.nbox; ++b) {
    if (!same(to_ibox(mf->boxes[b]), lv.boxes[b]))
      return fail(MG_ERR_MISMATCH, std::string(what) + ": box " + std::to_string(b) + " differs");
    if (mf->offsets[b] != off)
      return fail(MG_ERR_MISMATCH, std::string(what) + ": non-canonical offsets");
    off += grown_volume(lv.boxes[b], mf->ngrow, face_d);
  }
  return MG_OK;
}

// ---------------------------------------------------------------------------
// Profiling helpers

hipEvent_t take_event(mg_solver* s) {
  if (s->ev_used == s->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->ev_pool.push_back(e);
  }
  return s->ev_pool[s->ev_used++];
}

struct ProfScope {
  mg_solver* s;
  int fam;
  hipEvent_t b = nullptr;
  ProfScope(mg_solver* s_, int f, bool on) : s(s_), fam(f) {
    if (on && s->profile) {
      hipEvent_t a = take_event(s);
      b = take_event(s);
      if (a && b) {
        hipEventRecord(a, s->st);
        s->prof.push_back({fam, a, b});
      } else {
        b = nullptr;
      }
    }
  }
  ~ProfScope() {
    if (b) hipEventRecord(b, s->st);
  }
};

// ---------------------------------------------------------------------------
// Setup: coefficient copies and coarsening.

int setup_coefficients(mg_solver* s, const mg_multifab_t* acoef, const mg_multifab_t* const* bcoef) {
  Level& l0 = s->L[0];
  for (int d = 0; d < 3; ++d) {
    const double* src = bcoef ? (const double*)bcoef[d]->data : nullptr;
    HIPTRY(launch_scale_faces(s->st, src, l0.b64[d], l0.n_f[d], 1.0));
  }
  if (s->has_a)
    HIPTRY(hipMemcpyAsync(l0.a64, acoef->data, sizeof(double) * l0.n_g0, hipMemcpyDeviceToDevice,
                          s->st));
  return MG_OK;
}

int coarsen_all(mg_solver* s) {
  const bool f32 = s->opts.precision == MG_PREC_F32_REFINE;
  for (size_t l = 0; l + 1 < s->L.size(); ++l) {
    Level& f = s->L[l];
    Level& c = s->L[l + 1];
    for (int d = 0; d < 3; ++d)
      HIPTRY(launch_coarsen_face(s->st, f.d_info, f.nbox, c.d_info, d, f.b64[d], c.b64[d],
                                 f.max_faces));
    if (s->has_a)
      HIPTRY(launch_coarsen_cell<double>(s->st, f.d_rst, (int)f.t_rst.size(), f.s_rst, f.d_info,
                                         c.d_info, f.a64, c.a64));
  }
  if (f32) {
    for (Level& lv : s->L) {
      for (int d = 0; d < 3; ++d)
        HIPTRY((launch_convert<double, float>(s->st, lv.b64[d], lv.b32[d], lv.n_f[d])));
      if (s->has_a) HIPTRY((launch_convert<double, float>(s->st, lv.a64, lv.a32, lv.n_g0)));
    }
  }
  const Level& bl = s->L.back();
  BottomTables bt = bottom_tables(s);
  if (f32)
    HIPTRY(launch_bottom_setup<float>(s->st, bt, stencil_of<float>(s, bl, true), s->bdiag32,
                                      s->bcoef32));
  else
    HIPTRY(launch_bottom_setup<double>(s->st, bt, stencil_of<double>(s, bl, false), s->bdiag64,
                                       s->bcoef64));
  return MG_OK;
}

// ---------------------------------------------------------------------------
// The V-cycle.

template <typename T>
struct LevelData {
  T *e, *rhs, *r;
};

template <typename T>
LevelData<T> ldata(Level& lv, bool f32) {
  if (f32) return {(T*)lv.e32, (T*)lv.rhs32, (T*)lv.r32};
  return {(T*)lv.e64, (T*)lv.rhs64, (T*)lv.r64};
}

template <typename T>
int exchange(mg_solver* s, Level& lv, T* v, bool prof) {
  ProfScope ps(s, 2, prof);
  HIPTRY(launch_fill_boundary<T>(s->st, lv.d_tags, lv.d_chunks, (int)lv.chunks.size(), v, 1));
  return MG_OK;
}

template <typename T>
T* alt_of(Level& lv);
template <>
double* alt_of<double>(Level& lv) { return lv.alt64; }
template <>
float* alt_of<float>(Level& lv) { return lv.alt32; }

// Fused sweeps: phi -> alt -> phi ...; each sweep is the fused pass, an
// exchange of its output and the rim pass.  An odd count ends with a copy
// back into phi.
template <typename T>
int smooth_fused(mg_solver* s, Level& lv, const StencilArgs<T>& op, T* phi, const T* rhs,
                 int rhs_ng, int sweeps, bool zero_first, bool prof) {
  T* cur = phi;
  T* nxt = alt_of<T>(lv);
  if (!nxt) return fail(MG_ERR_ARG, "fused sweep without its second buffer");
  int rc;
  for (int k = 0; k < sweeps; ++k) {
    const bool zg = zero_first && k == 0;
    if (!zg && (rc = exchange<T>(s, lv, cur, prof))) return rc;
    {
      ProfScope ps(s, 0, prof);
      HIPTRY(launch_sweep<T>(s->st, lv.d_sweep, (int)lv.t_sweep.size(), lv.s_sweep, op, cur, nxt,
                             rhs, rhs_ng, zg ? 1 : 0, nullptr));
    }
    if ((rc = exchange<T>(s, lv, nxt, prof))) return rc;
    {
      ProfScope ps(s, 7, prof);
      HIPTRY(launch_rim<T>(s->st, lv.d_rim, (int)lv.t_rim.size(), op, nxt, rhs, rhs_ng));
    }
    std::swap(cur, nxt);
  }
  if (cur != phi)
    HIPTRY(hipMemcpyAsync(phi, cur, sizeof(T) * lv.n_g1, hipMemcpyDeviceToDevice, s->st));
  return MG_OK;
}

// reverse: black before red in every sweep (the post-smoothing of the
// symmetric V-cycle; always as half-sweeps).  On a write-through level the
// face ghosts stay current from half-sweep to half-sweep, so only the first
// one needs them exchanged, and only when the caller's data may have stale
// ghosts (ghosts_current false; a zero-guess start reads none).  On return
// a write-through level's face ghosts are current.
//
// With a coarse correction ec (cinfo: the coarse level's box table) the
// first half-sweep also adds P ec to phi (interpolation folded in; see
// launch_gsrb): phi's face ghosts must be current without the correction
// and ec's face ghosts current (fold_interp says when the V-cycle has that).
template <typename T>
int smooth(mg_solver* s, Level& lv, const StencilArgs<T>& op, T* phi, const T* rhs, int rhs_ng,
           int sweeps, bool zero_first, bool prof, bool reverse = false,
           bool ghosts_current = false, const BoxInfo* cinfo = nullptr, const T* ec = nullptr,
           const BoxInfo* finfo = nullptr, const T* rf = nullptr, T* rout = nullptr) {
  if (ec && (!lv.wt || lv.fused || zero_first || sweeps < 1))
    return fail(MG_ERR_ARG, "folded interpolation on a level without write-through");
  if (rf && (!zero_first || lv.fused || reverse || sweeps < 1 || rhs_ng != 0 || rout != rhs))
    return fail(MG_ERR_ARG, "folded restriction outside a zero-guess smoothing");
  if (lv.fused && !reverse)
    return smooth_fused<T>(s, lv, op, phi, rhs, rhs_ng, sweeps, zero_first, prof);
  const int c0 = reverse ? 1 : 0;
  const WtBox* wtb = lv.wt ? lv.d_wtbox : nullptr;
  const WtEntry* wte = lv.wt ? lv.d_wt : nullptr;
  if (ec) ghosts_current = true;
  int rc;
  for (int k = 0; k < sweeps; ++k) {
    const bool zg = zero_first && k == 0;
    const bool need = lv.wt ? (k == 0 && !zg && !ghosts_current) : !zg;
    if (need && (rc = exchange<T>(s, lv, phi, prof))) return rc;
    if (k == 0 && ec) {
      // counted as interpolation, which it replaces
      ProfScope ps(s, 4, prof);
      HIPTRY(launch_gsrb<T>(s->st, lv.d_gsrb, (int)lv.t_gsrb.size(), lv.s_gsrb, op, phi, rhs,
                            rhs_ng, c0, 0, wtb, wte, cinfo, ec));
    } else {
      ProfScope ps(s, 0, prof);
      HIPTRY(launch_gsrb<T>(s->st, lv.d_gsrb, (int)lv.t_gsrb.size(), lv.s_gsrb, op, phi, rhs,
                            rhs_ng, c0, zg ? 1 : 0, wtb, wte, nullptr, nullptr,
                            zg ? finfo : nullptr, zg ? rf : nullptr, zg ? rout : nullptr));
    }
    if (!lv.wt && (rc = exchange<T>(s, lv, phi, prof))) return rc;
    {
      ProfScope ps(s, 0, prof);
      HIPTRY(launch_gsrb<T>(s->st, lv.d_gsrb, (int)lv.t_gsrb.size(), lv.s_gsrb, op, phi, rhs,
                            rhs_ng, 1 - c0, 0, wtb, wte));
    }
  }
  return MG_OK;
}

// Whether level l's interpolation from level l+1 folds into its first
// post-smoothing half-sweep: both levels write through (so phi's face ghosts
// are current before the interpolation and level l+1's, which is smoothed
// and not the bottom, are current after its post-smoothing), and there is a
// half-sweep to fold into.
bool fold_interp(const mg_solver* s, size_t l) {
  if (!s->opts.interp_fold || s->opts.nu2 < 1 || l + 1 >= s->L.size()) return false;
  const Level& f = s->L[l];
  const Level& c = s->L[l + 1];
  return f.wt && c.wt && !f.fused && !c.fused;
}

// Whether the restriction into level l (>= 1) folds into level l's first
// pre-smoothing half-sweep, which with a zero initial guess reads only the
// right-hand side at its own cell: the level is smoothed (not the bottom)
// by half-sweeps from zero, and its boxes are the finer boxes coarsened one
// to one.
bool fold_restrict(const mg_solver* s, size_t l) {
  if (!s->opts.restrict_fold || l == 0 || l + 1 >= s->L.size() || s->opts.nu1 < 1) return false;
  const Level& c = s->L[l];
  return c.coarsened_1to1 && (c.fold_rs || s->opts.restrict_fold == 2) && !c.fused;
}

// Coarse levels l >= lstart in correction form (zero initial guess).  rf:
// the finer level's residual, restricted here into this level's rhs.
template <typename T>
int coarse_cycle(mg_solver* s, size_t l, bool f32, const T* rf = nullptr) {
  Level& lv = s->L[l];
  LevelData<T> D = ldata<T>(lv, f32);
  const StencilArgs<T> op = stencil_of<T>(s, lv, f32);
  const bool prof = l == 0;
  int rc;
  if ((int)l == s->tail_lev) {
    // the plan was built for the solver's precision (FP32 refinement: float)
    if (f32 != (s->opts.precision == MG_PREC_F32_REFINE))
      return fail(MG_ERR_ARG, "coarse tail in the other precision");
    HIPTRY(launch_tail<T>(s->st, reinterpret_cast<const TailPlan<T>*>(s->d_tail), s->nb,
                          tail_lds_need(s, s->tail_lev)));
    return MG_OK;
  }
  const bool rs = rf && fold_restrict(s, l);
  if (rf && !rs) {
    const Level& fl = s->L[l - 1];
    HIPTRY(launch_restrict<T>(s->st, fl.d_rst, (int)fl.t_rst.size(), fl.s_rst, fl.d_info,
                              lv.d_info, rf, D.rhs));
  }
  if (l + 1 == s->L.size()) {
    const BottomTables bt = bottom_tables(s);
    const T* diag = f32 ? (const T*)s->bdiag32 : (const T*)s->bdiag64;
    const T* coef = f32 ? (const T*)s->bcoef32 : (const T*)s->bcoef64;
    T* work = f32 ? (T*)s->bwork32 : (T*)s->bwork64;
    const int maxit = s->opts.bottom_max_iter > 0 ? s->opts.bottom_max_iter : s->nb;
    if (s->opts.bottom_solver == 1)
      HIPTRY(launch_bottom_bicgstab<T>(s->st, bt, diag, coef, D.rhs, D.e, 0, work,
                                       s->opts.bottom_rel_tol, maxit, s->singular ? 1 : 0,
                                       s->d_iters));
    else
      HIPTRY(launch_bottom_cg<T>(s->st, bt, diag, coef, D.rhs, D.e, 0, work,
                                 s->opts.bottom_rel_tol, maxit, s->singular ? 1 : 0, s->d_iters));
    return MG_OK;
  }
  if (s->opts.nu1 == 0)
    HIPTRY(launch_zero_valid<T>(s->st, lv.d_cell, (int)lv.t_cell.size(), lv.s_cell, lv.d_info, D.e,
                                1));
  if ((rc = smooth<T>(s, lv, op, D.e, D.rhs, 0, s->opts.nu1, s->opts.nu1 > 0, prof, false, false,
                      nullptr, nullptr, rs ? s->L[l - 1].d_info : nullptr, rs ? rf : nullptr,
                      rs ? D.rhs : nullptr)))
    return rc;
  // write-through smoothing leaves the face ghosts current
  if (!(lv.wt && s->opts.nu1 > 0) && (rc = exchange<T>(s, lv, D.e, prof))) return rc;
  Level& cl = s->L[l + 1];
  LevelData<T> C = ldata<T>(cl, f32);
  // level 0 may restrict inside its residual pass (then level 1 gets no rf)
  const bool rr = l == 0 && s->rr_fold;
  {
    ProfScope ps(s, 1, prof);
    if (rr)
      HIPTRY(launch_resid_restrict<T>(s->st, lv.d_rr, (int)lv.t_rr.size(), lv.s_rr, op, D.e,
                                      D.rhs, 0, cl.d_info, C.rhs));
    else
      HIPTRY((launch_residual<T, T>(s->st, lv.d_cell, (int)lv.t_cell.size(), lv.s_cell, op, D.e,
                                    D.rhs, 0, D.r, nullptr, 0)));
  }
  // the coarser levels, starting with the restriction of D.r
  if (l == 0 && s->opts.use_graph) {
    hipGraphExec_t g = f32 ? s->graph32 : s->graph64;
    ProfScope ps(s, 5, true);
    HIPTRY(hipGraphLaunch(g, s->st));
  } else {
    ProfScope ps(s, 5, l == 0);
    if ((rc = coarse_cycle<T>(s, l + 1, f32, rr ? nullptr : D.r))) return rc;
  }
  if (fold_interp(s, l))
    return smooth<T>(s, lv, op, D.e, D.rhs, 0, s->opts.nu2, false, prof, s->opts.krylov != 0,
                     true, cl.d_info, C.e);
  {
    ProfScope ps(s, 4, prof);
    HIPTRY(launch_prolong_add<T>(s->st, lv.d_cell, (int)lv.t_cell.size(), lv.s_cell, lv.d_info,
                                 cl.d_info, D.e, C.e));
  }
  return smooth<T>(s, lv, op, D.e, D.rhs, 0, s->opts.nu2, false, prof, s->opts.krylov != 0);
}

int capture_graphs(mg_solver* s) {
  if (!s->opts.use_graph || s->L.size() < 2) {
    s->opts.use_graph = 0;
    return MG_OK;
  }
  const bool f32 = s->opts.precision == MG_PREC_F32_REFINE;
  hipGraph_t g;
  HIPTRY(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
  const bool saved = s->profile;
  s->profile = false;
  // the level-0 residual pass restricts into level 1 itself with rr_fold
  int rc = f32 ? coarse_cycle<float>(s, 1, true, s->rr_fold ? nullptr : s->L[0].r32)
               : coarse_cycle<double>(s, 1, false, s->rr_fold ? nullptr : s->L[0].r64);
  s->profile = saved;
  hipError_t e = hipStreamEndCapture(s->st, &g);
  if (rc) return rc;
  if (e != hipSuccess) return fail(MG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t ex;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return fail(MG_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  if (f32)
    s->graph32 = ex;
  else
    s->graph64 = ex;
  return MG_OK;
}

// Level-0 V-cycle on the caller's phi (direct form, FP64).  red_done: the
// first pre-smoothing half-sweep (red) has already been applied to phi's
// valid cells (by the stop test's residual pass) and phi's ghosts exchanged.
int vcycle64(mg_solver* s, double* phi, const double* rhs, int rhs_ng, bool red_done = false) {
  Level& l0 = s->L[0];
  const StencilArgs<double> op = stencil_of<double>(s, l0, false);
  int rc;
  if (s->L.size() == 1) {
    if ((rc = exchange<double>(s, l0, phi, true))) return rc;
    HIPTRY((launch_residual<double, double>(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, op,
                                            phi, rhs, rhs_ng, l0.r64, nullptr, 0)));
    const int maxit = s->opts.bottom_max_iter > 0 ? s->opts.bottom_max_iter : s->nb;
    if (s->opts.bottom_solver == 1)
      HIPTRY(launch_bottom_bicgstab<double>(s->st, bottom_tables(s), s->bdiag64, s->bcoef64, l0.r64,
                                            phi, 1, s->bwork64, s->opts.bottom_rel_tol, maxit,
                                            s->singular ? 1 : 0, s->d_iters));
    else
      HIPTRY(launch_bottom_cg<double>(s->st, bottom_tables(s), s->bdiag64, s->bcoef64, l0.r64,
                                      phi, 1, s->bwork64, s->opts.bottom_rel_tol, maxit,
                                      s->singular ? 1 : 0, s->d_iters));
    return MG_OK;
  }
  // the caller's last exchange (or write-through smoothing) left phi's face
  // ghosts current
  if (red_done) {
    if (s->opts.nu1 < 1) return fail(MG_ERR_ARG, "folded red half-sweep without pre-smoothing");
    {
      ProfScope ps(s, 0, true);
      HIPTRY(launch_gsrb<double>(s->st, l0.d_gsrb, (int)l0.t_gsrb.size(), l0.s_gsrb, op, phi, rhs,
                                 rhs_ng, 1, 0, l0.wt ? l0.d_wtbox : nullptr,
                                 l0.wt ? l0.d_wt : nullptr));
    }
    if ((rc = smooth<double>(s, l0, op, phi, rhs, rhs_ng, s->opts.nu1 - 1, false, true, false,
                             true)))
      return rc;
  } else if ((rc = smooth<double>(s, l0, op, phi, rhs, rhs_ng, s->opts.nu1, false, true, false,
                                  true))) {
    return rc;
  }
  if (!(l0.wt && s->opts.nu1 > 0) && (rc = exchange<double>(s, l0, phi, true))) return rc;
  Level& l1 = s->L[1];
  {
    ProfScope ps(s, 1, true);
    if (s->rr_fold)
      HIPTRY(launch_resid_restrict<double>(s->st, l0.d_rr, (int)l0.t_rr.size(), l0.s_rr, op, phi,
                                           rhs, rhs_ng, l1.d_info, l1.rhs64));
    else
      HIPTRY((launch_residual<double, double>(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell,
                                              op, phi, rhs, rhs_ng, l0.r64, nullptr, 0)));
  }
  // the coarser levels, starting with the restriction of the residual
  // (already in level 1's rhs with rr_fold)
  if (s->opts.use_graph) {
    ProfScope ps(s, 5, true);
    HIPTRY(hipGraphLaunch(s->graph64, s->st));
  } else {
    ProfScope ps(s, 5, true);
    if ((rc = coarse_cycle<double>(s, 1, false, s->rr_fold ? nullptr : l0.r64))) return rc;
  }
  if (fold_interp(s, 0))
    return smooth<double>(s, l0, op, phi, rhs, rhs_ng, s->opts.nu2, false, true, false, true,
                          l1.d_info, l1.e64);
  {
    ProfScope ps(s, 4, true);
    HIPTRY(launch_prolong_add<double>(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell,
                                      l0.d_info, l1.d_info, phi, l1.e64));
  }
  return smooth<double>(s, l0, op, phi, rhs, rhs_ng, s->opts.nu2, false, true);
}

// The norm of a slot: the largest of its ways (bit patterns of |x|, so the
// unsigned maximum is the maximum of the values, NaN included).
int read_norm(mg_solver* s, int slot, double* out) {
  HIPTRY(hipMemcpyAsync(s->h_norm, norm_slot(s, slot), sizeof(unsigned long long) * kNormSlot,
                        hipMemcpyDeviceToHost, s->st));
  HIPTRY(hipStreamSynchronize(s->st));
  unsigned long long m = 0;
  for (int w = 0; w < kNormWays; ++w) m = std::max(m, s->h_norm[w * kNormStride]);
  double v;
  std::memcpy(&v, &m, sizeof(double));
  *out = v;
  return MG_OK;
}

int begin_call(mg_solver* s) {
  HIPTRY(hipEventRecord(s->ev_in, s->user));
  HIPTRY(hipStreamWaitEvent(s->st, s->ev_in, 0));
  return MG_OK;
}
int end_call(mg_solver* s) {
  HIPTRY(hipEventRecord(s->ev_out, s->st));
  HIPTRY(hipStreamWaitEvent(s->user, s->ev_out, 0));
  return MG_OK;
}

// One entry-point call: the solver stream waits for the caller's stream on
// entry, and on every exit (error returns included) the caller's stream waits
// for everything the call enqueued, so memory the caller frees or reuses
// after an error is not still being written by the call's kernels.  On an
// error exit the ordering is best effort and keeps the message of the failure
// that caused the exit.
class CallScope {
 public:
  explicit CallScope(mg_solver* s) : s_(s), rc_(begin_call(s)) {
    if (rc_ != MG_OK) s_ = nullptr;
  }
  ~CallScope() {
    if (s_ && hipEventRecord(s_->ev_out, s_->st) == hipSuccess)
      (void)hipStreamWaitEvent(s_->user, s_->ev_out, 0);
  }
  CallScope(const CallScope&) = delete;
  CallScope& operator=(const CallScope&) = delete;
  int rc() const { return rc_; }
  // The normal exit: the ordering's own errors are reported.
  int finish() {
    mg_solver* s = s_;
    s_ = nullptr;
    return s ? end_call(s) : MG_OK;
  }

 private:
  mg_solver* s_;
  int rc_;
};

// ---------------------------------------------------------------------------
// Tile-shape tuning of the level-0 smoother and residual.

std::string tune_key(const mg_solver* s, const char* kern, bool f32, size_t lev = 0) {
  const Level& l0 = s->L[lev];
  int mx[3] = {0, 0, 0};
  for (const IBox& b : l0.boxes)
    for (int d = 0; d < 3; ++d) mx[d] = std::max(mx[d], ext(b, d));
  hipDeviceProp_t p;
  int dev = 0;
  hipGetDevice(&dev);
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) arch = p.gcnArchName;
  std::ostringstream o;
  o << arch << "|" << kern << "|" << (f32 ? "f32" : "f64") << "|" << mx[0] << "x" << mx[1] << "x"
    << mx[2] << "|" << l0.nbox;
  return o.str();
}

const char* tune_path() {
  const char* p = std::getenv("AMRMG_TUNE_CACHE");
  return p && *p ? p : nullptr;
}

std::map<std::string, Shape> read_cache() {
  std::map<std::string, Shape> m;
  const char* p = tune_path();
  if (!p) return m;
  std::ifstream in(p);
  std::string key;
  Shape sh;
  while (in >> key >> sh.lx >> sh.ly >> sh.tz >> sh.u >> sh.wp) m[key] = sh;
  return m;
}

void write_cache(const std::map<std::string, Shape>& m) {
  const char* p = tune_path();
  if (!p) return;
  std::ofstream out(p);
  for (auto& kv : m)
    out << kv.first << " " << kv.second.lx << " " << kv.second.ly << " " << kv.second.tz << " "
        << kv.second.u << " " << kv.second.wp << "\n";
}

int apply_shape(mg_solver* s, Shape sh, bool gsrb, size_t lev = 0) {
  Level& l0 = s->L[lev];
  if (gsrb) {
    std::vector<Tile> t;
    make_tiles(l0.info, sh, gsrb_tx(sh), false, t);
    if (t.size() > l0.cap_gsrb) return fail(MG_ERR_ARG, "tile table larger than its reservation");
    l0.t_gsrb = t;
    l0.s_gsrb = sh;
    l0.cls.clear();
    HIPTRY(hipMemcpyAsync(l0.d_gsrb, l0.t_gsrb.data(), sizeof(Tile) * l0.t_gsrb.size(),
                          hipMemcpyHostToDevice, s->st));
  } else {
    std::vector<Tile> t;
    make_tiles(l0.info, sh, sh.lx, false, t);
    if (t.size() > l0.cap_cell) return fail(MG_ERR_ARG, "tile table larger than its reservation");
    l0.t_cell = t;
    l0.s_cell = sh;
    HIPTRY(hipMemcpyAsync(l0.d_cell, l0.t_cell.data(), sizeof(Tile) * l0.t_cell.size(),
                          hipMemcpyHostToDevice, s->st));
  }
  HIPTRY(hipStreamSynchronize(s->st));
  return MG_OK;
}

// Level-0 tiles of the fused residual-restriction pass.
int apply_rr_shape(mg_solver* s, Shape sh) {
  Level& l0 = s->L[0];
  std::vector<Tile> t;
  make_tiles(l0.info, sh, sh.lx, false, t);
  if (t.size() > l0.cap_rr) return fail(MG_ERR_ARG, "tile table larger than its reservation");
  l0.t_rr = t;
  l0.s_rr = sh;
  HIPTRY(hipMemcpyAsync(l0.d_rr, l0.t_rr.data(), sizeof(Tile) * l0.t_rr.size(),
                        hipMemcpyHostToDevice, s->st));
  HIPTRY(hipStreamSynchronize(s->st));
  return MG_OK;
}

// Level-0 smoother tiles with class shapes cls (dflt for other classes).
int apply_class_tiles(mg_solver* s, const std::map<int, Shape>& cls, Shape dflt) {
  Level& l0 = s->L[0];
  std::vector<Tile> t;
  make_class_tiles(l0.info, cls, dflt, {}, t);
  if (t.size() > l0.cap_gsrb) return fail(MG_ERR_ARG, "tile table larger than its reservation");
  l0.t_gsrb = t;
  l0.s_gsrb = class_launch_shape(cls, dflt);
  l0.cls = cls;
  l0.cls_base = dflt;
  HIPTRY(hipMemcpyAsync(l0.d_gsrb, l0.t_gsrb.data(), sizeof(Tile) * l0.t_gsrb.size(),
                        hipMemcpyHostToDevice, s->st));
  HIPTRY(hipStreamSynchronize(s->st));
  return MG_OK;
}

int apply_sweep_shape(mg_solver* s, Shape sh) {
  Level& l0 = s->L[0];
  if (!l0.fused || !sweep_lds_bytes(sh, sizeof(double))) return fail(MG_ERR_ARG, "no fused sweep shape");
  std::vector<Tile> t;
  make_tiles(l0.info, sh, sh.lx, false, t);
  if (t.size() > l0.cap_sweep) return fail(MG_ERR_ARG, "tile table larger than its reservation");
  l0.t_sweep = t;
  l0.s_sweep = sh;
  HIPTRY(hipMemcpyAsync(l0.d_sweep, l0.t_sweep.data(), sizeof(Tile) * l0.t_sweep.size(),
                        hipMemcpyHostToDevice, s->st));
  return MG_OK;
}

// Mean time of one fused sweep (fused pass + rim pass, no exchanges) with
// shape sh, ping-ponging between phi and the level's second buffer.
template <typename T>
int time_sweep(mg_solver* s, Shape sh, T* phi, const T* rhs, const StencilArgs<T>& op, float* ms) {
  int rc;
  if ((rc = apply_sweep_shape(s, sh))) return rc;
  Level& l0 = s->L[0];
  T* alt = alt_of<T>(l0);
  hipEvent_t a = take_event(s), b = take_event(s);
  auto one = [&](int w) -> hipError_t {
    T* in = (w & 1) ? alt : phi;
    T* out = (w & 1) ? phi : alt;
    hipError_t e = launch_sweep<T>(s->st, l0.d_sweep, (int)l0.t_sweep.size(), sh, op, in, out,
                                   rhs, 0, 0, nullptr);
    if (e != hipSuccess) return e;
    return launch_rim<T>(s->st, l0.d_rim, (int)l0.t_rim.size(), op, out, rhs, 0);
  };
  for (int w = 0; w < 2; ++w) HIPTRY(one(w));
  HIPTRY(hipEventRecord(a, s->st));
  const int reps = 6;
  for (int w = 0; w < reps; ++w) HIPTRY(one(w));
  HIPTRY(hipEventRecord(b, s->st));
  HIPTRY(hipEventSynchronize(b));
  float t;
  HIPTRY(hipEventElapsedTime(&t, a, b));
  *ms = t / reps;
  s->ev_used -= 2;
  return MG_OK;
}

template <typename T>
int time_gsrb(mg_solver* s, Shape sh, T* phi, const T* rhs, const StencilArgs<T>& op, float* ms,
              size_t lev = 0) {
  int rc;
  if ((rc = apply_shape(s, sh, true, lev))) return rc;
  hipEvent_t a = take_event(s), b = take_event(s);
  Level& l0 = s->L[lev];
  // with the level's write-through tables, as the solve launches it
  const WtBox* wtb = l0.wt ? l0.d_wtbox : nullptr;
  const WtEntry* wte = l0.wt ? l0.d_wt : nullptr;
  for (int w = 0; w < 2; ++w)
    HIPTRY(launch_gsrb<T>(s->st, l0.d_gsrb, (int)l0.t_gsrb.size(), sh, op, phi, rhs, 0, w & 1, 0,
                          wtb, wte));
  HIPTRY(hipEventRecord(a, s->st));
  const int reps = lev ? 24 : 6;
  for (int w = 0; w < reps; ++w)
    HIPTRY(launch_gsrb<T>(s->st, l0.d_gsrb, (int)l0.t_gsrb.size(), sh, op, phi, rhs, 0, w & 1, 0,
                          wtb, wte));
  HIPTRY(hipEventRecord(b, s->st));
  HIPTRY(hipEventSynchronize(b));
  float t;
  HIPTRY(hipEventElapsedTime(&t, a, b));
  *ms = t / reps;
  s->ev_used -= 2;
  return MG_OK;
}

// A residual that writes r, and with_norm a norm-only residual (into the
// spare norm slot 3) after it: the two ways an FP64 solve runs the kernel
// (the FP32 V-cycle only writes r; its norms come from FP64 residuals).
// Where the FP64 solve folds its stop test into the next half-sweep, the
// norm launch also writes the next iterate, as the solve runs it.
template <typename T>
int time_resid(mg_solver* s, Shape sh, const T* phi, const T* rhs, const StencilArgs<T>& op,
               T* out, bool with_norm, float* ms, size_t lev = 0) {
  int rc;
  if ((rc = apply_shape(s, sh, false, lev))) return rc;
  hipEvent_t a = take_event(s), b = take_event(s);
  Level& l0 = s->L[lev];
  unsigned long long* nb = norm_slot(s, 3);
  // with rr_fold the level-0 V-cycle residual is the fused pass (tiles of
  // its own): these tiles then serve the stop test alone
  const bool stop_only = with_norm && lev == 0 && s->rr_fold;
  auto pair = [&]() -> hipError_t {
    if (!stop_only) {
      hipError_t e = launch_residual<T, T>(s->st, l0.d_cell, (int)l0.t_cell.size(), sh, op, phi,
                                           rhs, 0, out, nullptr, 0);
      if (e != hipSuccess || !with_norm) return e;
    }
    T* nx = nullptr;
    if constexpr (std::is_same<T, double>::value) nx = lev == 0 ? l0.next64 : nullptr;
    return launch_residual<T, T>(s->st, l0.d_cell, (int)l0.t_cell.size(), sh, op, phi, rhs, 0,
                                 (T*)nullptr, nb, 0, nullptr, nx);
  };
  HIPTRY(launch_fill_u64(s->st, nb, kNormSlot, 0ull));
  for (int w = 0; w < 2; ++w) HIPTRY(pair());
  HIPTRY(hipEventRecord(a, s->st));
  const int reps = lev ? 24 : with_norm ? 3 : 6;
  for (int w = 0; w < reps; ++w) HIPTRY(pair());
  HIPTRY(hipEventRecord(b, s->st));
  HIPTRY(hipEventSynchronize(b));
  float t;
  HIPTRY(hipEventElapsedTime(&t, a, b));
  *ms = t / reps;
  s->ev_used -= 2;
  return MG_OK;
}

// Mean time of the fused residual-restriction pass (level 0 into level 1's
// rhs, which the solve overwrites before use) with tiles sh.
template <typename T>
int time_rr(mg_solver* s, Shape sh, const T* phi, const T* rhs, const StencilArgs<T>& op,
            T* rc, float* ms) {
  int rc_;
  if ((rc_ = apply_rr_shape(s, sh))) return rc_;
  Level& l0 = s->L[0];
  hipEvent_t a = take_event(s), b = take_event(s);
  auto one = [&]() {
    return launch_resid_restrict<T>(s->st, l0.d_rr, (int)l0.t_rr.size(), sh, op, phi, rhs, 0,
                                    s->L[1].d_info, rc);
  };
  for (int w = 0; w < 2; ++w) HIPTRY(one());
  HIPTRY(hipEventRecord(a, s->st));
  const int reps = 6;
  for (int w = 0; w < reps; ++w) HIPTRY(one());
  HIPTRY(hipEventRecord(b, s->st));
  HIPTRY(hipEventSynchronize(b));
  float t;
  HIPTRY(hipEventElapsedTime(&t, a, b));
  *ms = t / reps;
  s->ev_used -= 2;
  return MG_OK;
}

// Second pass of a shape search: the best few shapes of the first pass are
// timed again, several times and interleaved, and the lowest median wins
// (single short timings of shapes within a few per cent pick by noise).
template <typename F>
int pick_finalist(std::vector<std::pair<float, Shape>>& first, F&& time_one, Shape* best,
                  float* best_ms) {
  std::stable_sort(first.begin(), first.end(),
                   [](const std::pair<float, Shape>& x, const std::pair<float, Shape>& y) {
                     return x.first < y.first;
                   });
  const size_t k = std::min<size_t>(4, first.size());
  std::vector<std::vector<float>> t(k);
  for (int round = 0; round < 3; ++round)
    for (size_t c = 0; c < k; ++c) {
      float ms;
      int rc = time_one(first[c].second, &ms);
      if (rc) return rc;
      t[c].push_back(ms);
    }
  float bm = 1e30f;
  for (size_t c = 0; c < k; ++c) {
    std::sort(t[c].begin(), t[c].end());
    if (t[c][1] < bm) {
      bm = t[c][1];
      *best = first[c].second;
    }
  }
  *best_ms = bm;
  return MG_OK;
}

// Level 1, one eighth of the cells, runs from the last-level cache rather
// than from HBM, so its best shapes differ from level 0's: its smoother and
// residual are timed on its own boxes (the residual writes r only; the norm
// is taken on level 0).  Levels below it are a few microseconds per launch.
bool tune_level1_ok(const mg_solver* s) { return s->L.size() >= 3 && !s->L[1].fused; }

template <typename T>
int tune_level1(mg_solver* s, bool f32, T* phi, Shape* best_g, Shape* best_c, float* tg,
                float* tr) {
  Level& l1 = s->L[1];
  const LevelData<T> D = ldata<T>(l1, f32);
  const StencilArgs<T> op = stencil_of<T>(s, l1, f32);
  HIPTRY(hipMemsetAsync(phi, 0, sizeof(T) * l1.n_g1, s->st));
  HIPTRY(hipMemsetAsync(D.rhs, 0, sizeof(T) * l1.n_g0, s->st));
  int rc;
  float t;
  std::vector<std::pair<float, Shape>> fg, fr;
  for (Shape sh : gsrb_candidates()) {
    if ((rc = time_gsrb<T>(s, sh, phi, D.rhs, op, &t, 1))) return rc;
    fg.push_back({t, sh});
  }
  if ((rc = pick_finalist(fg, [&](Shape sh, float* ms) {
         return time_gsrb<T>(s, sh, phi, D.rhs, op, ms, 1);
       }, best_g, tg)))
    return rc;
  for (Shape sh : cell_candidates()) {
    if ((rc = time_resid<T>(s, sh, phi, D.rhs, op, D.r, false, &t, 1))) return rc;
    fr.push_back({t, sh});
  }
  if ((rc = pick_finalist(fr, [&](Shape sh, float* ms) {
         return time_resid<T>(s, sh, phi, D.rhs, op, D.r, false, ms, 1);
       }, best_c, tr)))
    return rc;
  if ((rc = apply_shape(s, *best_g, true, 1))) return rc;
  return apply_shape(s, *best_c, false, 1);
}

// Restriction into level 1 plus its zero-guess half-sweep: two passes, or
// the half-sweep that restricts as it goes (mean time of one pair / one).
template <typename T>
int time_rfold(mg_solver* s, bool f32, bool fold, T* phi, float* ms) {
  Level& fl = s->L[0];
  Level& cl = s->L[1];
  const LevelData<T> F = ldata<T>(fl, f32), C = ldata<T>(cl, f32);
  const StencilArgs<T> op = stencil_of<T>(s, cl, f32);
  const WtBox* wtb = cl.wt ? cl.d_wtbox : nullptr;
  const WtEntry* wte = cl.wt ? cl.d_wt : nullptr;
  const int nt = (int)cl.t_gsrb.size();
  auto one = [&]() -> hipError_t {
    if (fold)
      return launch_gsrb<T>(s->st, cl.d_gsrb, nt, cl.s_gsrb, op, phi, C.rhs, 0, 0, 1, wtb, wte,
                            nullptr, nullptr, fl.d_info, F.r, C.rhs);
    hipError_t e = launch_restrict<T>(s->st, fl.d_rst, (int)fl.t_rst.size(), fl.s_rst, fl.d_info,
                                      cl.d_info, F.r, C.rhs);
    if (e != hipSuccess) return e;
    return launch_gsrb<T>(s->st, cl.d_gsrb, nt, cl.s_gsrb, op, phi, C.rhs, 0, 0, 1, wtb, wte);
  };
  hipEvent_t a = take_event(s), b = take_event(s);
  for (int w = 0; w < 2; ++w) HIPTRY(one());
  HIPTRY(hipEventRecord(a, s->st));
  const int reps = 24;
  for (int w = 0; w < reps; ++w) HIPTRY(one());
  HIPTRY(hipEventRecord(b, s->st));
  HIPTRY(hipEventSynchronize(b));
  float t;
  HIPTRY(hipEventElapsedTime(&t, a, b));
  *ms = t / reps;
  s->ev_used -= 2;
  return MG_OK;
}

// Time a level-0 smoother tile table (as the solve launches it, with the
// level's write-through tables), colours alternating.  Leaves the table on
// the device; the caller re-applies the one it keeps.
template <typename T>
int time_table(mg_solver* s, const std::vector<Tile>& t, Shape launch, T* phi, const T* rhs,
               const StencilArgs<T>& op, float* ms) {
  Level& l0 = s->L[0];
  if (t.size() > l0.cap_gsrb) return fail(MG_ERR_ARG, "tile table larger than its reservation");
  HIPTRY(hipMemcpyAsync(l0.d_gsrb, t.data(), sizeof(Tile) * t.size(), hipMemcpyHostToDevice, s->st));
  const WtBox* wtb = l0.wt ? l0.d_wtbox : nullptr;
  const WtEntry* wte = l0.wt ? l0.d_wt : nullptr;
  hipEvent_t a = take_event(s), b = take_event(s);
  for (int w = 0; w < 2; ++w)
    HIPTRY(launch_gsrb<T>(s->st, l0.d_gsrb, (int)t.size(), launch, op, phi, rhs, 0, w & 1, 0, wtb,
                          wte));
  HIPTRY(hipEventRecord(a, s->st));
  const int reps = 6;
  for (int w = 0; w < reps; ++w)
    HIPTRY(launch_gsrb<T>(s->st, l0.d_gsrb, (int)t.size(), launch, op, phi, rhs, 0, w & 1, 0, wtb,
                          wte));
  HIPTRY(hipEventRecord(b, s->st));
  HIPTRY(hipEventSynchronize(b));
  float tm;
  HIPTRY(hipEventElapsedTime(&tm, a, b));
  *ms = tm / reps;
  s->ev_used -= 2;
  return MG_OK;
}

// Per-class smoother shapes for level 0 (boxes of at least two x extents):
// each class's candidates (best_g's thread count, unroll and whole-pair
// choice) are timed on that class's boxes alone, the best few again; the
// table with every class at its winner is then timed against best_g's
// uniform table, three times each, interleaved, and kept only if faster.
// On return the kept table is applied; *cls is empty when the uniform one
// won.
template <typename T>
int tune_classes(mg_solver* s, Shape best_g, T* phi, const T* rhs, const StencilArgs<T>& op,
                 std::map<int, Shape>* cls, float* t_uni, float* t_cls) {
  Level& l0 = s->L[0];
  cls->clear();
  std::map<int, std::vector<int>> members;
  for (int b = 0; b < (int)l0.info.size(); ++b)
    members[l0.info[b].hi[0] - l0.info[b].lo[0] + 1].push_back(b);
  int rc;
  *t_uni = *t_cls = 0;
  // class tables keep the pair mapping
  if (members.size() < 2 || l0.fused || best_g.wp == 2) return MG_OK;
  const int threads = best_g.lx * best_g.ly;
  std::map<int, Shape> pick;
  for (const auto& kv : members) {
    std::vector<std::pair<float, Shape>> first;
    for (Shape c : class_candidates(threads, best_g.u, best_g.wp)) {
      std::map<int, Shape> one{{kv.first, c}};
      std::vector<Tile> t;
      make_class_tiles(l0.info, one, best_g, kv.second, t);
      float ms;
      if ((rc = time_table<T>(s, t, class_launch_shape(one, best_g), phi, rhs, op, &ms))) return rc;
      first.push_back({ms, c});
    }
    Shape best = best_g;
    float bt;
    if ((rc = pick_finalist(first, [&](Shape c, float* ms) {
           std::map<int, Shape> one{{kv.first, c}};
           std::vector<Tile> t;
           make_class_tiles(l0.info, one, best_g, kv.second, t);
           return time_table<T>(s, t, class_launch_shape(one, best_g), phi, rhs, op, ms);
         }, &best, &bt)))
      return rc;
    pick[kv.first] = best;
  }
  std::vector<Tile> tu, tc;
  make_tiles(l0.info, best_g, gsrb_tx(best_g), false, tu);
  make_class_tiles(l0.info, pick, best_g, {}, tc);
  const Shape lc = class_launch_shape(pick, best_g);
  float bu = 1e30f, bc = 1e30f, ms;
  for (int rep = 0; rep < 3; ++rep) {
    if ((rc = time_table<T>(s, tu, best_g, phi, rhs, op, &ms))) return rc;
    bu = std::min(bu, ms);
    if ((rc = time_table<T>(s, tc, lc, phi, rhs, op, &ms))) return rc;
    bc = std::min(bc, ms);
  }
  *t_uni = bu;
  *t_cls = bc;
  if (bc < bu) {
    *cls = pick;
    return apply_class_tiles(s, pick, best_g);
  }
  return apply_shape(s, best_g, true);
}

std::string class_key(const mg_solver* s, bool f32, int x_extent) {
  return tune_key(s, "gsrbclass", f32) + "|x" + std::to_string(x_extent);
}

// The quad smoother mapping runs on FP32 level-0 half-sweeps that stream
// through buffer loads with write-through, one tile shape for every box.
bool quad_ok(const mg_solver* s) {
  const Level& l0 = s->L[0];
  // with every box's x extent a multiple of 4 no quad load reaches past the
  // end of an array (its cells past a row's end are the next row's); a
  // partly out-of-range load would leave its in-range cells to the
  // hardware's range check
  for (const BoxInfo& b : l0.info)
    if ((b.hi[0] - b.lo[0] + 1) % 4) return false;
  return s->opts.precision == MG_PREC_F32_REFINE && l0.wt && !l0.fused &&
         stencil_of<float>(s, l0, true).buf != 0;
}

int autotune(mg_solver* s) {
  const bool f32 = s->opts.precision == MG_PREC_F32_REFINE;
  Level& l0 = s->L[0];
  auto cache = read_cache();
  const std::string kg = tune_key(s, "gsrb", f32), kr = tune_key(s, "resid", f32);
  const std::string ks = tune_key(s, "sweep", f32);
  const std::string krr = tune_key(s, "rr", f32);
  const bool t1 = tune_level1_ok(s);
  const std::string kg1 = t1 ? tune_key(s, "gsrb", f32, 1) : "", kr1 = t1 ? tune_key(s, "resid", f32, 1) : "";
  // whether the restriction into level 1 folds (entry u = 1)
  const bool tf = t1 && s->L[1].coarsened_1to1 && s->opts.restrict_fold == 1 &&
                  s->opts.nu1 >= 1 && !s->rr_fold;
  const std::string kf = tf ? tune_key(s, "rfold", f32, 1) : "";
  int rc;
  if (s->opts.tune == 1) {
    auto itf = tf ? cache.find(kf) : cache.end();
    if (itf != cache.end()) s->L[1].fold_rs = itf->second.u == 1;
    // level 1 entries (keyed by the level's own box shape and count)
    for (int g = 0; t1 && g < 2; ++g) {
      auto it = cache.find(g ? kg1 : kr1);
      if (it == cache.end() || !shape_ok(it->second)) continue;
      std::vector<Tile> t;
      make_tiles(s->L[1].info, it->second, g ? gsrb_tx(it->second) : it->second.lx, false, t);
      if (t.size() <= (g ? s->L[1].cap_gsrb : s->L[1].cap_cell) &&
          (rc = apply_shape(s, it->second, g == 1, 1)))
        return rc;
    }
    // sweep entry: the fused shape, u = 1 when it beat two half-sweeps
    auto is = cache.find(ks);
    if (l0.fused && is != cache.end()) {
      std::vector<Tile> t;
      make_tiles(l0.info, is->second, is->second.lx, false, t);
      if (sweep_lds_bytes(is->second, sizeof(double)) && t.size() <= l0.cap_sweep &&
          (rc = apply_sweep_shape(s, is->second)))
        return rc;
      if (is->second.u == 0) l0.fused = false;
    }
    auto it = cache.find(kg);
    if (it != cache.end() && shape_ok(it->second) && (it->second.wp != 2 || quad_ok(s))) {
      std::vector<Tile> t;
      make_tiles(l0.info, it->second, gsrb_tx(it->second), false, t);
      if (t.size() <= l0.cap_gsrb && (rc = apply_shape(s, it->second, true))) return rc;
      // class shapes, where the tuner found them faster than the uniform one
      std::map<int, Shape> cls;
      bool all = !l0.fused;
      std::set<int> xs;
      for (const BoxInfo& b : l0.info) xs.insert(b.hi[0] - b.lo[0] + 1);
      for (int x : xs) {
        auto ic = cache.find(class_key(s, f32, x));
        if (ic == cache.end()) {
          all = false;
          break;
        }
        cls[x] = ic->second;
      }
      if (all && xs.size() >= 2) {
        bool fits = true;
        for (const auto& kv : cls)
          fits = fits && kv.second.lx * kv.second.ly == it->second.lx * it->second.ly &&
                 kv.second.u == it->second.u && kv.second.wp == it->second.wp;
        std::vector<Tile> tc;
        make_class_tiles(l0.info, cls, it->second, {}, tc);
        if (fits && tc.size() <= l0.cap_gsrb && (rc = apply_class_tiles(s, cls, it->second)))
          return rc;
      }
    }
    it = cache.find(kr);
    if (it != cache.end() && shape_ok(it->second)) {
      std::vector<Tile> t;
      make_tiles(l0.info, it->second, it->second.lx, false, t);
      if (t.size() <= l0.cap_cell && (rc = apply_shape(s, it->second, false))) return rc;
    }
    it = s->rr_fold ? cache.find(krr) : cache.end();
    if (it != cache.end()) {
      bool cand = false;
      for (Shape c : rr_candidates())
        cand = cand || (c.lx == it->second.lx && c.ly == it->second.ly && c.tz == it->second.tz);
      if (cand && (rc = apply_rr_shape(s, Shape{it->second.lx, it->second.ly, it->second.tz, 2})))
        return rc;
    }
    return MG_OK;
  }
  if (s->opts.tune != 2) return MG_OK;
  // data: the scratch array (ng 1) as phi, level-0 coefficients as rhs-sized input
  const Shape g0 = l0.s_gsrb, c0 = l0.s_cell, w0 = l0.s_sweep;
  Shape best_g = g0, best_c = c0, best_w = w0;
  float tg = 1e30f, tr = 1e30f, tw = 1e30f, t;
  if (f32) {
    float* phi = (float*)s->tune_scratch;
    HIPTRY(hipMemsetAsync(phi, 0, sizeof(float) * l0.n_g1, s->st));
    const StencilArgs<float> op = stencil_of<float>(s, l0, true);
    if (l0.fused)
      for (Shape sh : sweep_candidates()) {
        if ((rc = time_sweep<float>(s, sh, phi, l0.rhs32, op, &t))) return rc;
        if (t < tw) { tw = t; best_w = sh; }
      }
    std::vector<std::pair<float, Shape>> fg, fr;
    for (Shape sh : gsrb_candidates()) {
      if ((rc = time_gsrb<float>(s, sh, phi, l0.rhs32, op, &t))) return rc;
      fg.push_back({t, sh});
    }
    // one x-quad per lane where the level streams through buffer loads
    if (quad_ok(s))
      for (Shape sh : quad_candidates()) {
        if ((rc = time_gsrb<float>(s, sh, phi, l0.rhs32, op, &t))) return rc;
        fg.push_back({t, sh});
      }
    if ((rc = pick_finalist(fg, [&](Shape sh, float* ms) {
           return time_gsrb<float>(s, sh, phi, l0.rhs32, op, ms);
         }, &best_g, &tg)))
      return rc;
    for (Shape sh : cell_candidates()) {
      if ((rc = time_resid<float>(s, sh, phi, l0.rhs32, op, l0.r32, false, &t))) return rc;
      fr.push_back({t, sh});
    }
    if ((rc = pick_finalist(fr, [&](Shape sh, float* ms) {
           return time_resid<float>(s, sh, phi, l0.rhs32, op, l0.r32, false, ms);
         }, &best_c, &tr)))
      return rc;
  } else {
    double* phi = s->tune_scratch;
    HIPTRY(hipMemsetAsync(phi, 0, sizeof(double) * l0.n_g1, s->st));
    const StencilArgs<double> op = stencil_of<double>(s, l0, false);
    if (l0.fused)
      for (Shape sh : sweep_candidates()) {
        if ((rc = time_sweep<double>(s, sh, phi, l0.r64, op, &t))) return rc;
        if (t < tw) { tw = t; best_w = sh; }
      }
    std::vector<std::pair<float, Shape>> fg, fr;
    for (Shape sh : gsrb_candidates()) {
      if ((rc = time_gsrb<double>(s, sh, phi, l0.r64, op, &t))) return rc;
      fg.push_back({t, sh});
    }
    if ((rc = pick_finalist(fg, [&](Shape sh, float* ms) {
           return time_gsrb<double>(s, sh, phi, l0.r64, op, ms);
         }, &best_g, &tg)))
      return rc;
    for (Shape sh : cell_candidates()) {
      if ((rc = time_resid<double>(s, sh, phi, l0.r64, op, l0.r64, true, &t))) return rc;
      fr.push_back({t, sh});
    }
    if ((rc = pick_finalist(fr, [&](Shape sh, float* ms) {
           return time_resid<double>(s, sh, phi, l0.r64, op, l0.r64, true, ms);
         }, &best_c, &tr)))
      return rc;
  }
  if ((rc = apply_shape(s, best_g, true))) return rc;
  if ((rc = apply_shape(s, best_c, false))) return rc;
  if (s->rr_fold) {
    std::vector<std::pair<float, Shape>> fq;
    Shape best_q = l0.s_rr;
    float tq = 1e30f;
    Level& l1 = s->L[1];
    auto time_q = [&](Shape sh, float* ms) {
      return f32 ? time_rr<float>(s, sh, (const float*)s->tune_scratch, l0.rhs32,
                                  stencil_of<float>(s, l0, true), l1.rhs32, ms)
                 : time_rr<double>(s, sh, s->tune_scratch, l0.r64,
                                   stencil_of<double>(s, l0, false), l1.rhs64, ms);
    };
    for (Shape sh : rr_candidates()) {
      if ((rc = time_q(sh, &t))) return rc;
      fq.push_back({t, sh});
    }
    if ((rc = pick_finalist(fq, time_q, &best_q, &tq))) return rc;
    if ((rc = apply_rr_shape(s, best_q))) return rc;
    cache[krr] = best_q;
  }
  std::map<int, Shape> cls;
  float tu = 0, tcl = 0;
  rc = f32 ? tune_classes<float>(s, best_g, (float*)s->tune_scratch, l0.rhs32,
                                 stencil_of<float>(s, l0, true), &cls, &tu, &tcl)
           : tune_classes<double>(s, best_g, s->tune_scratch, l0.r64,
                                  stencil_of<double>(s, l0, false), &cls, &tu, &tcl);
  if (rc) return rc;
  {
    // a class entry per x extent; a class that keeps best_g is stored as
    // best_g, so loading the cache rebuilds the same table (or none)
    std::set<int> xs;
    for (const BoxInfo& b : l0.info) xs.insert(b.hi[0] - b.lo[0] + 1);
    for (int x : xs) {
      auto it = cls.find(x);
      if (it != cls.end())
        cache[class_key(s, f32, x)] = it->second;
      else
        cache.erase(class_key(s, f32, x));
    }
    if (s->opts.verbose && xs.size() >= 2) {
      fprintf(stderr, "amrmg tune classes: uniform %.4f ms, per class %.4f ms (%s)\n", tu, tcl,
              cls.empty() ? "uniform kept" : "classes kept");
      for (const auto& kv : cls)
        fprintf(stderr, "  x extent %d: %dx%dx%d\n", kv.first, kv.second.lx, kv.second.ly,
                kv.second.tz);
    }
  }
  Shape g1 = t1 ? s->L[1].s_gsrb : Shape{}, c1 = t1 ? s->L[1].s_cell : Shape{};
  float tg1 = 0, tr1 = 0;
  if (t1) {
    rc = f32 ? tune_level1<float>(s, true, (float*)s->tune_scratch, &g1, &c1, &tg1, &tr1)
             : tune_level1<double>(s, false, s->tune_scratch, &g1, &c1, &tg1, &tr1);
    if (rc) return rc;
    cache[kg1] = g1;
    cache[kr1] = c1;
  }
  float tsep = 0, tfold = 0;
  if (tf) {
    // with level 1's tiles as chosen above; best of three interleaved
    float a = 1e30f, b = 1e30f, t;
    for (int r = 0; r < 3; ++r) {
      rc = f32 ? time_rfold<float>(s, true, false, (float*)s->tune_scratch, &t)
               : time_rfold<double>(s, false, false, s->tune_scratch, &t);
      if (rc) return rc;
      a = std::min(a, t);
      rc = f32 ? time_rfold<float>(s, true, true, (float*)s->tune_scratch, &t)
               : time_rfold<double>(s, false, true, s->tune_scratch, &t);
      if (rc) return rc;
      b = std::min(b, t);
    }
    tsep = a;
    tfold = b;
    s->L[1].fold_rs = tfold < tsep;
    cache[kf] = Shape{1, 1, 1, s->L[1].fold_rs ? 1 : 0, 0};
  }
  if (l0.fused) {
    if ((rc = apply_sweep_shape(s, best_w))) return rc;
    // a fused sweep also saves nothing on exchanges, so it must beat the two
    // half-sweeps it replaces on its own
    best_w.u = tw < 2 * tg ? 1 : 0;
    l0.fused = best_w.u == 1;
    cache[ks] = best_w;
  }
  if (s->opts.verbose)
    fprintf(stderr,
            "amrmg tune: gsrb %dx%dx%d u%d wp%d %.4f ms, resid %dx%dx%d u%d %.4f ms, "
            "sweep %dx%dx%d %.4f ms (%s)\n",
            best_g.lx, best_g.ly, best_g.tz, best_g.u, best_g.wp, tg, best_c.lx, best_c.ly,
            best_c.tz, best_c.u, tr, best_w.lx, best_w.ly, best_w.tz, tw,
            l0.fused ? "fused" : "half-sweeps");
  if (s->opts.verbose && t1)
    fprintf(stderr,
            "amrmg tune level 1: gsrb %dx%dx%d u%d wp%d %.4f ms, resid %dx%dx%d u%d %.4f ms, "
            "restriction + first half-sweep %.4f ms, folded %.4f ms\n",
            g1.lx, g1.ly, g1.tz, g1.u, g1.wp, tg1, c1.lx, c1.ly, c1.tz, c1.u, tr1, tsep, tfold);
  cache[kg] = best_g;
  cache[kr] = best_c;
  write_cache(cache);
  return MG_OK;
}

template <typename T>
TailPlan<T> tail_plan(mg_solver* s, bool f32) {
  TailPlan<T> tp{};
  const int nl = (int)s->L.size(), t = s->tail_lev;
  tp.nlev = nl - 1 - t;
  tp.nu1 = s->opts.nu1;
  tp.nu2 = s->opts.nu2;
  tp.reverse = s->opts.krylov != 0;
  Level& up = s->L[t - 1];
  tp.rf = ldata<T>(up, f32).r;
  tp.finfo = up.d_info;
  tp.fnbox = up.nbox;
  tp.rcells = up.d_trc;
  // level 0's residual pass already restricted into the first tail level
  tp.nrc = t == 1 && s->rr_fold ? 0 : (int)up.h_trc.size();
  for (int i = 0; i < tp.nlev; ++i) {
    Level& lv = s->L[t + i];
    const LevelData<T> D = ldata<T>(lv, f32);
    TailLevel<T>& L = tp.lev[i];
    L.op = stencil_of<T>(s, lv, f32);
    L.e = D.e;
    L.rhs = D.rhs;
    L.r = D.r;
    L.wtb = lv.d_wtbox;
    L.wte = lv.d_wt;
    L.cells = lv.d_tcells;
    L.nred = lv.tail_nred;
    L.ncell = (int)lv.h_tcells.size();
    L.nbox = lv.nbox;
    L.rcells = lv.d_trc;
    L.nrc = (int)lv.h_trc.size();
    L.cinfo = s->L[t + i + 1].d_info;
  }
  const LevelData<T> B = ldata<T>(s->L.back(), f32);
  tp.binfo = s->L.back().d_info;
  tp.bnbox = s->L.back().nbox;
  tail_lds_layout<T>(s, t, &tp);
  tp.bt = bottom_tables(s);
  tp.bdiag = f32 ? (const T*)s->bdiag32 : (const T*)s->bdiag64;
  tp.bcoef = f32 ? (const T*)s->bcoef32 : (const T*)s->bcoef64;
  tp.be = B.e;
  tp.brhs = B.rhs;
  tp.tol = s->opts.bottom_rel_tol;
  tp.maxiter = s->opts.bottom_max_iter > 0 ? s->opts.bottom_max_iter : s->nb;
  tp.singular = s->singular ? 1 : 0;
  tp.iters = s->d_iters;
  return tp;
}

// The tail's device plan (pinned staging, then a copy on the solver stream,
// which the caller synchronises before the staging goes).
template <typename T>
int upload_tail_plan(mg_solver* s, bool f32) {
  const TailPlan<T> tp = tail_plan<T>(s, f32);
  TailPlan<T>* h = nullptr;
  HIPTRY(hipHostMalloc((void**)&h, sizeof(TailPlan<T>), hipHostMallocDefault));
  *h = tp;
  hipError_t e = hipMemcpyAsync(s->d_tail, h, sizeof(TailPlan<T>), hipMemcpyHostToDevice, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  hipHostFree(h);
  HIPTRY(e);
  return MG_OK;
}

int upload_tables(mg_solver* s) {
  for (Level& lv : s->L) {
    HIPTRY(hipMemcpyAsync(lv.d_info, lv.info.data(), sizeof(BoxInfo) * lv.info.size(),
                          hipMemcpyHostToDevice, s->st));
    if (!lv.t_gsrb.empty())
      HIPTRY(hipMemcpyAsync(lv.d_gsrb, lv.t_gsrb.data(), sizeof(Tile) * lv.t_gsrb.size(),
                            hipMemcpyHostToDevice, s->st));
    if (!lv.t_cell.empty())
      HIPTRY(hipMemcpyAsync(lv.d_cell, lv.t_cell.data(), sizeof(Tile) * lv.t_cell.size(),
                            hipMemcpyHostToDevice, s->st));
    if (!lv.t_rst.empty())
      HIPTRY(hipMemcpyAsync(lv.d_rst, lv.t_rst.data(), sizeof(Tile) * lv.t_rst.size(),
                            hipMemcpyHostToDevice, s->st));
    if (!lv.t_vec.empty())
      HIPTRY(hipMemcpyAsync(lv.d_vec, lv.t_vec.data(), sizeof(Tile) * lv.t_vec.size(),
                            hipMemcpyHostToDevice, s->st));
    if (!lv.t_rr.empty())
      HIPTRY(hipMemcpyAsync(lv.d_rr, lv.t_rr.data(), sizeof(Tile) * lv.t_rr.size(),
                            hipMemcpyHostToDevice, s->st));
    if (lv.wt) {
      if (!lv.h_wt.empty())
        HIPTRY(hipMemcpyAsync(lv.d_wt, lv.h_wt.data(), sizeof(WtEntry) * lv.h_wt.size(),
                              hipMemcpyHostToDevice, s->st));
      HIPTRY(hipMemcpyAsync(lv.d_wtbox, lv.h_wtbox.data(), sizeof(WtBox) * lv.h_wtbox.size(),
                            hipMemcpyHostToDevice, s->st));
    }
    if (lv.fused) {
      HIPTRY(hipMemcpyAsync(lv.d_sweep, lv.t_sweep.data(), sizeof(Tile) * lv.t_sweep.size(),
                            hipMemcpyHostToDevice, s->st));
      if (!lv.t_rim.empty())
        HIPTRY(hipMemcpyAsync(lv.d_rim, lv.t_rim.data(), sizeof(RimTile) * lv.t_rim.size(),
                              hipMemcpyHostToDevice, s->st));
    }
    if (!lv.tags.empty())
      HIPTRY(hipMemcpyAsync(lv.d_tags, lv.tags.data(), sizeof(FbTag) * lv.tags.size(),
                            hipMemcpyHostToDevice, s->st));
    if (!lv.chunks.empty())
      HIPTRY(hipMemcpyAsync(lv.d_chunks, lv.chunks.data(), sizeof(FbChunk) * lv.chunks.size(),
                            hipMemcpyHostToDevice, s->st));
  }
  const size_t nb = s->nb;
  HIPTRY(hipMemcpyAsync(s->d_nbr, s->h_nbr.data(), sizeof(int) * 6 * nb, hipMemcpyHostToDevice, s->st));
  HIPTRY(hipMemcpyAsync(s->d_fidx, s->h_fidx.data(), sizeof(int) * 6 * nb, hipMemcpyHostToDevice, s->st));
  HIPTRY(hipMemcpyAsync(s->d_aidx, s->h_aidx.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s->st));
  HIPTRY(hipMemcpyAsync(s->d_map_rhs, s->h_map_rhs.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s->st));
  HIPTRY(hipMemcpyAsync(s->d_map_out, s->h_map_out.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s->st));
  if (s->tail_lev > 0) {
    for (Level& lv : s->L) {
      if (!lv.h_tcells.empty())
        HIPTRY(hipMemcpyAsync(lv.d_tcells, lv.h_tcells.data(), sizeof(unsigned) * lv.h_tcells.size(),
                              hipMemcpyHostToDevice, s->st));
      if (!lv.h_trc.empty())
        HIPTRY(hipMemcpyAsync(lv.d_trc, lv.h_trc.data(), sizeof(unsigned) * lv.h_trc.size(),
                              hipMemcpyHostToDevice, s->st));
    }
    const int rc = s->opts.precision == MG_PREC_F32_REFINE ? upload_tail_plan<float>(s, true)
                                                           : upload_tail_plan<double>(s, false);
    if (rc) return rc;
  }
  return MG_OK;
}

bool is_singular_problem(const mg_solver* s) {
  return s->periodic[0] && s->periodic[1] && s->periodic[2] && s->alpha == 0.0;
}

// ---------------------------------------------------------------------------
// Two-level composite: plan and cycle.
//
// Fine boxes live in the index space of the coarse level refined by 2; each is
// a union of whole coarse cells inside one coarse box.  The fine level gets
// its own box table, tiles and exchange tags; the coarse/fine coupling is
// three tables built here: fine ghosts to interpolate, and per uncovered
// coarse cell the coarse/fine faces whose coarse flux is replaced by the mean
// fine flux.

struct CoarseIndex {
  IBox dom;
  int n[3];
  std::vector<int> owner;  // coarse cell -> box
  const std::vector<BoxInfo>* info;
  explicit CoarseIndex(const Level& lv) : dom(lv.domain), info(&lv.info) {
    for (int d = 0; d < 3; ++d) n[d] = ext(dom, d);
    owner.assign((size_t)n[0] * n[1] * n[2], -1);
    for (int b = 0; b < lv.nbox; ++b) {
      const IBox& B = lv.boxes[b];
      for (int k = B.lo[2]; k <= B.hi[2]; ++k)
        for (int j = B.lo[1]; j <= B.hi[1]; ++j)
          for (int i = B.lo[0]; i <= B.hi[0]; ++i) owner[lin(i, j, k)] = b;
    }
  }
  size_t lin(int i, int j, int k) const {
    return (size_t)(i - dom.lo[0]) + (size_t)n[0] * ((j - dom.lo[1]) + (size_t)n[1] * (k - dom.lo[2]));
  }
  bool inside(const int p[3]) const {
    for (int d = 0; d < 3; ++d)
      if (p[d] < dom.lo[d] || p[d] > dom.hi[d]) return false;
    return true;
  }
  long long elem(const int p[3], int ng) const {
    const BoxInfo& B = (*info)[owner[lin(p[0], p[1], p[2])]];
    const long long nx = B.hi[0] - B.lo[0] + 1 + 2 * ng, ny = B.hi[1] - B.lo[1] + 1 + 2 * ng;
    return (ng ? B.off_g1 : B.off_g0) + (p[0] - B.lo[0] + ng) + nx * ((p[1] - B.lo[1] + ng) +
                                                                      ny * (p[2] - B.lo[2] + ng));
  }
  long long face_elem(const int p[3], int d, int f) const {  // face f along d of cell p's box
    const BoxInfo& B = (*info)[owner[lin(p[0], p[1], p[2])]];
    int q[3] = {p[0], p[1], p[2]};
    q[d] = f;
    const long long fx = B.hi[0] - B.lo[0] + 1 + (d == 0), fy = B.hi[1] - B.lo[1] + 1 + (d == 1);
    return B.off_f[d] + (q[0] - B.lo[0]) + fx * ((q[1] - B.lo[1]) + fy * (long long)(q[2] - B.lo[2]));
  }
};

long long fine_elem(const BoxInfo& B, const int q[3]) {
  const long long nx = B.hi[0] - B.lo[0] + 3, ny = B.hi[1] - B.lo[1] + 3;
  return B.off_g1 + (q[0] - B.lo[0] + 1) + nx * ((q[1] - B.lo[1] + 1) + ny * (q[2] - B.lo[2] + 1));
}
long long fine_face_elem(const BoxInfo& B, int d, const int q[3]) {
  const long long fx = B.hi[0] - B.lo[0] + 1 + (d == 0), fy = B.hi[1] - B.lo[1] + 1 + (d == 1);
  return B.off_f[d] + (q[0] - B.lo[0]) + fx * ((q[1] - B.lo[1]) + fy * (long long)(q[2] - B.lo[2]));
}

int build_composite(mg_solver* s, const std::vector<IBox>& fboxes, Bump& bump) {
  const Level& L0 = s->L[0];
  IBox fdom;
  for (int d = 0; d < 3; ++d) {
    fdom.lo[d] = 2 * s->domain.lo[d];
    fdom.hi[d] = 2 * s->domain.hi[d] + 1;
  }
  std::string err;
  if (!validate_boxes(fboxes, fdom, false, &err)) return fail(MG_ERR_INVALID_BOXARRAY, "fine: " + err);
  Level& F = s->F;
  F.boxes = fboxes;
  F.domain = fdom;
  F.merged = false;
  fill_info(F, fdom, s->periodic);
  for (int b = 0; b < F.nbox; ++b) {
    const IBox& B = fboxes[b];
    for (int d = 0; d < 3; ++d)
      if (((B.lo[d] % 2) + 2) % 2 != 0 || ext(B, d) % 2 != 0)
        return fail(MG_ERR_INVALID_BOXARRAY, "fine box " + std::to_string(b) +
                                                 " is not a union of whole coarse cells");
    const IBox cb = coarsen(B, 2);
    int par = -1;
    for (int c = 0; c < L0.nbox; ++c)
      if (same(intersect(L0.boxes[c], cb), cb)) par = c;
    if (par < 0)
      return fail(MG_ERR_INVALID_BOXARRAY, "fine box " + std::to_string(b) +
                                               " does not lie inside one coarse box");
    F.info[b].parent = par;
    if (grown_volume(B, 1, 0) >= (int64_t(1) << 31))
      return fail(MG_ERR_INVALID_BOXARRAY, "a fine box holds 2^31 or more cells");
  }
  int mx[3] = {1, 1, 1};
  for (const IBox& b : F.boxes)
    for (int d = 0; d < 3; ++d) mx[d] = std::max(mx[d], ext(b, d));
  F.s_gsrb = fit_tz(F.info, shape_gsrb(mx[0], mx[1], mx[2]), 2, false);
  F.s_cell = fit_tz(F.info, shape_cell(mx[0], mx[1], mx[2]), 1, false);
  make_tiles(F.info, F.s_gsrb, 2 * F.s_gsrb.lx, false, F.t_gsrb);
  make_tiles(F.info, F.s_cell, F.s_cell.lx, false, F.t_cell);
  F.cap_gsrb = F.t_gsrb.size();
  F.cap_cell = F.t_cell.size();
  build_fb(F, s->periodic, 1);
  s->s_fcov = fit_tz(F.info, shape_cell(std::max(1, mx[0] / 2), std::max(1, mx[1] / 2),
                                        std::max(1, mx[2] / 2)), 1, true);
  make_tiles(F.info, s->s_fcov, s->s_fcov.lx, true, s->t_fcov);

  // coverage of the coarse level
  CoarseIndex ci(L0);
  std::vector<char> covered(ci.owner.size(), 0);
  for (const IBox& B : fboxes) {
    const IBox cb = coarsen(B, 2);
    for (int k = cb.lo[2]; k <= cb.hi[2]; ++k)
      for (int j = cb.lo[1]; j <= cb.hi[1]; ++j)
        for (int i = cb.lo[0]; i <= cb.hi[0]; ++i) covered[ci.lin(i, j, k)] = 1;
  }
  // fine ghosts no fine box supplies: face slabs of each box, inside the domain,
  // whose coarse parent is uncovered (fine boxes are unions of coarse cells)
  s->h_ghost.clear();
  for (int b = 0; b < F.nbox; ++b) {
    const IBox& B = fboxes[b];
    for (int d = 0; d < 3; ++d)
      for (int side = -1; side <= 1; side += 2) {
        IBox slab = B;
        slab.lo[d] = slab.hi[d] = side < 0 ? B.lo[d] - 1 : B.hi[d] + 1;
        for (int k = slab.lo[2]; k <= slab.hi[2]; ++k)
          for (int j = slab.lo[1]; j <= slab.hi[1]; ++j)
            for (int i = slab.lo[0]; i <= slab.hi[0]; ++i) {
              const int g[3] = {i, j, k};
              bool in = true;
              for (int a = 0; a < 3; ++a)
                if (g[a] < fdom.lo[a] || g[a] > fdom.hi[a]) in = false;
              if (!in) continue;
              const int C[3] = {floordiv(i, 2), floordiv(j, 2), floordiv(k, 2)};
              if (covered[ci.lin(C[0], C[1], C[2])]) continue;
              CfGhost e;
              e.dst = fine_elem(F.info[b], g);
              e.c = ci.elem(C, 1);
              e.sign = 0;
              e.pad = 0;
              for (int a = 0; a < 3; ++a) {
                for (int o = 0; o < 2; ++o) {
                  int q[3] = {C[0], C[1], C[2]};
                  q[a] += o ? 1 : -1;
                  e.nb[2 * a + o] = ci.inside(q) ? ci.elem(q, 1) : -1;
                }
                if (((g[a] % 2) + 2) % 2 == 1) e.sign |= 1 << a;
              }
              s->h_ghost.push_back(e);
            }
      }
  }
  // coarse/fine faces grouped by uncovered coarse cell (ordered by cell index)
  std::map<size_t, std::vector<CfFace>> byI;
  std::map<size_t, std::pair<long long, long long>> cellIdx;
  for (int b = 0; b < F.nbox; ++b) {
    const IBox cb = coarsen(fboxes[b], 2);
    for (int d = 0; d < 3; ++d)
      for (int side = -1; side <= 1; side += 2) {
        IBox slab = cb;
        slab.lo[d] = slab.hi[d] = side < 0 ? cb.lo[d] - 1 : cb.hi[d] + 1;
        for (int k = slab.lo[2]; k <= slab.hi[2]; ++k)
          for (int j = slab.lo[1]; j <= slab.hi[1]; ++j)
            for (int i = slab.lo[0]; i <= slab.hi[0]; ++i) {
              const int I[3] = {i, j, k};
              if (!ci.inside(I) || covered[ci.lin(i, j, k)]) continue;
              int J[3] = {i, j, k};
              J[d] -= side;
              CfFace f;
              f.d = d;
              f.pad = 0;
              f.j_idx = ci.elem(J, 1);
              f.cb_idx = ci.face_elem(I, d, side > 0 ? I[d] : I[d] + 1);
              int tr[2], t = 0;
              for (int a = 0; a < 3; ++a)
                if (a != d) tr[t++] = a;
              int q = 0;
              for (int o1 = 0; o1 < 2; ++o1)
                for (int o2 = 0; o2 < 2; ++o2, ++q) {
                  int fc[3];
                  fc[tr[0]] = 2 * J[tr[0]] + o1;
                  fc[tr[1]] = 2 * J[tr[1]] + o2;
                  fc[d] = 2 * J[d] + (side < 0 ? 0 : 1);
                  int gc[3] = {fc[0], fc[1], fc[2]};
                  gc[d] += side;
                  int face[3] = {fc[0], fc[1], fc[2]};
                  if (side > 0) face[d] += 1;
                  f.fv[q] = fine_elem(F.info[b], fc);
                  f.fg[q] = fine_elem(F.info[b], gc);
                  f.fb[q] = fine_face_elem(F.info[b], d, face);
                }
              const size_t key = ci.lin(i, j, k);
              byI[key].push_back(f);
              cellIdx[key] = {ci.elem(I, 0), ci.elem(I, 1)};
            }
      }
  }
  s->h_cfcell.clear();
  s->h_cfface.clear();
  for (auto& kv : byI) {
    CfCell c;
    c.r_idx = cellIdx[kv.first].first;
    c.phi_idx = cellIdx[kv.first].second;
    c.first = (int)s->h_cfface.size();
    c.count = (int)kv.second.size();
    s->h_cfcell.push_back(c);
    for (const CfFace& f : kv.second) s->h_cfface.push_back(f);
  }
  // workspace
  F.d_info = bump.take<BoxInfo>(F.info.size());
  F.d_gsrb = bump.take<Tile>(F.t_gsrb.size());
  F.d_cell = bump.take<Tile>(F.t_cell.size());
  F.d_tags = bump.take<FbTag>(F.tags.size());
  F.d_chunks = bump.take<FbChunk>(F.chunks.size());
  for (int d = 0; d < 3; ++d) F.b64[d] = bump.take<double>(F.n_f[d]);
  s->d_fcov = bump.take<Tile>(s->t_fcov.size());
  s->d_ghost = bump.take<CfGhost>(s->h_ghost.size());
  s->d_cfcell = bump.take<CfCell>(s->h_cfcell.size());
  s->d_cfface = bump.take<CfFace>(s->h_cfface.size());
  s->Rc = bump.take<double>(L0.n_g0);
  s->ef = bump.take<double>(F.n_g1);
  s->Rf = bump.take<double>(F.n_g0);
  s->rf2 = bump.take<double>(F.n_g0);
  if (s->opts.krylov) {
    const int m = s->gm_m;
    s->gm_Vf = bump.take<double>((size_t)(m + 1) * F.n_g0);
    s->gm_Vc = bump.take<double>((size_t)(m + 1) * L0.n_g0);
    s->gm_Zf = bump.take<double>((size_t)m * F.n_g1);
    s->gm_Zc = bump.take<double>((size_t)m * L0.n_g1);
    s->gm_Wf = bump.take<double>(F.n_g0);
    s->gm_Wc = bump.take<double>(L0.n_g0);
    s->gm_zero_f = bump.take<double>(F.n_g0);
    s->gm_zero_c = bump.take<double>(L0.n_g0);
    s->gm_part = bump.take<double>((size_t)(m + 1) * (F.t_cell.size() + L0.t_vec.size()));
    s->d_gm = bump.take<double>(m + 2);
  }
  if (s->opts.precision == MG_PREC_F32_REFINE) {
    for (int d = 0; d < 3; ++d) F.b32[d] = bump.take<float>(F.n_f[d]);
    s->Rc32 = bump.take<float>(L0.n_g0);
    s->ef32 = bump.take<float>(F.n_g1);
    s->Rf32 = bump.take<float>(F.n_g0);
    s->rf2_32 = bump.take<float>(F.n_g0);
  }
  s->ws_need = bump.off + 256;
  return MG_OK;
}

int upload_composite(mg_solver* s) {
  Level& F = s->F;
  auto up = [&](void* d, const void* h, size_t n) -> hipError_t {
    return n ? hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, s->st) : hipSuccess;
  };
  HIPTRY(up(F.d_info, F.info.data(), sizeof(BoxInfo) * F.info.size()));
  HIPTRY(up(F.d_gsrb, F.t_gsrb.data(), sizeof(Tile) * F.t_gsrb.size()));
  HIPTRY(up(F.d_cell, F.t_cell.data(), sizeof(Tile) * F.t_cell.size()));
  HIPTRY(up(F.d_tags, F.tags.data(), sizeof(FbTag) * F.tags.size()));
  HIPTRY(up(F.d_chunks, F.chunks.data(), sizeof(FbChunk) * F.chunks.size()));
  HIPTRY(up(s->d_fcov, s->t_fcov.data(), sizeof(Tile) * s->t_fcov.size()));
  HIPTRY(up(s->d_ghost, s->h_ghost.data(), sizeof(CfGhost) * s->h_ghost.size()));
  HIPTRY(up(s->d_cfcell, s->h_cfcell.data(), sizeof(CfCell) * s->h_cfcell.size()));
  HIPTRY(up(s->d_cfface, s->h_cfface.data(), sizeof(CfFace) * s->h_cfface.size()));
  return MG_OK;
}

// fine ghosts: other fine boxes, then coarse interpolation (covered coarse
// cells must already hold the average of their children)
template <typename T>
int fine_ghosts(mg_solver* s, T* fine, const T* coarse) {
  int rc;
  if ((rc = exchange<T>(s, s->F, fine, false))) return rc;
  HIPTRY(launch_cf_ghost<T>(s->st, s->d_ghost, (int)s->h_ghost.size(), coarse, fine));
  return MG_OK;
}

template <typename T>
int avgdown(mg_solver* s, const T* f, int fng, T* c, int cng, int zero_only) {
  HIPTRY(launch_avgdown<T>(s->st, s->d_fcov, (int)s->t_fcov.size(), s->s_fcov, s->F.d_info,
                           s->L[0].d_info, f, fng, c, cng, zero_only));
  return MG_OK;
}

template <typename T>
const T* bcoef(const Level& lv, int d);
template <>
const double* bcoef<double>(const Level& lv, int d) { return lv.b64[d]; }
template <>
const float* bcoef<float>(const Level& lv, int d) { return lv.b32[d]; }

// composite residual: Rf = ff - A_f phi_f, Rc = fc - A_c phi_c with refluxing,
// covered Rc = 0 (or, with cover_from, the mean of cover_from's children).
// Norms (when normbits != null) over fine cells and uncovered coarse cells.
template <typename T>
int composite_residual(mg_solver* s, T* phic, T* phif, const T* fc, int fc_ng, const T* ff,
                       int ff_ng, T* Rc, T* Rf, unsigned long long* normbits, const T* cover_from) {
  Level& L0 = s->L[0];
  Level& F = s->F;
  const bool f32 = sizeof(T) == 4;
  int rc;
  if ((rc = avgdown<T>(s, phif, 1, phic, 1, 0))) return rc;
  if ((rc = exchange<T>(s, L0, phic, false))) return rc;
  if ((rc = fine_ghosts<T>(s, phif, phic))) return rc;
  const StencilArgs<T> opf = stencil_of<T>(s, F, f32);
  const StencilArgs<T> opc = stencil_of<T>(s, L0, f32);
  HIPTRY((launch_residual<T, T>(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, opf, phif, ff,
                                ff_ng, Rf, normbits, 0)));
  HIPTRY((launch_residual<T, T>(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, opc, phic, fc,
                                fc_ng, Rc, nullptr, 0)));
  double ihc[3], ihf[3];
  for (int d = 0; d < 3; ++d) {
    ihc[d] = 1.0 / (L0.h[d] * L0.h[d]);
    ihf[d] = 1.0 / (F.h[d] * L0.h[d]);
  }
  HIPTRY(launch_cf_reflux<T>(s->st, s->d_cfcell, (int)s->h_cfcell.size(), s->d_cfface, phic,
                             phif, bcoef<T>(L0, 0), bcoef<T>(L0, 1), bcoef<T>(L0, 2),
                             bcoef<T>(F, 0), bcoef<T>(F, 1), bcoef<T>(F, 2), s->beta, ihc, ihf,
                             Rc));
  if (cover_from) {
    if ((rc = avgdown<T>(s, cover_from, 0, Rc, 0, 0))) return rc;
  } else {
    if ((rc = avgdown<T>(s, nullptr, 0, Rc, 0, 1))) return rc;
  }
  if (normbits)
    HIPTRY(launch_maxabs<T>(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info, Rc, 0,
                            normbits));
  return MG_OK;
}

template <typename T>
int fine_sweeps(mg_solver* s, T* ef, T* ec, const T* rhs, int sweeps) {
  Level& F = s->F;
  const StencilArgs<T> opf = stencil_of<T>(s, F, sizeof(T) == 4);
  int rc;
  for (int k = 0; k < sweeps; ++k)
    for (int colour = 0; colour < 2; ++colour) {
      if ((rc = avgdown<T>(s, ef, 1, ec, 1, 0))) return rc;
      if ((rc = fine_ghosts<T>(s, ef, ec))) return rc;
      HIPTRY(launch_gsrb<T>(s->st, F.d_gsrb, (int)F.t_gsrb.size(), F.s_gsrb, opf, ef, rhs, 0,
                            colour, 0));
    }
  return MG_OK;
}

// The two-level correction of a composite residual (vc, vf) from zero, in
// FP32 on (vc, vf) rounded once: result in ef32 (fine) and L0.e32 (coarse).
int correction_core32(mg_solver* s, const double* vc, const double* vf) {
  Level& L0 = s->L[0];
  Level& F = s->F;
  int rc;
  HIPTRY((launch_convert<double, float>(s->st, vc, s->Rc32, L0.n_g0)));
  HIPTRY((launch_convert<double, float>(s->st, vf, s->Rf32, F.n_g0)));
  HIPTRY(launch_zero_valid<float>(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info,
                                  s->ef32, 1));
  HIPTRY(launch_zero_valid<float>(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info,
                                  L0.e32, 1));
  if ((rc = fine_sweeps<float>(s, s->ef32, L0.e32, s->Rf32, 2 * s->opts.nu1))) return rc;
  if ((rc = composite_residual<float>(s, L0.e32, s->ef32, s->Rc32, 0, s->Rf32, 0, L0.rhs32,
                                      s->rf2_32, nullptr, s->rf2_32)))
    return rc;
  if ((rc = coarse_cycle<float>(s, 0, true))) return rc;
  HIPTRY(launch_prolong_add<float>(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info,
                                   L0.d_info, s->ef32, L0.e32));
  return fine_sweeps<float>(s, s->ef32, L0.e32, s->Rf32, 2 * s->opts.nu2);
}

// The same in FP64: result in ef (fine, ng 1) and L0.e64 (coarse).
int correction_core64(mg_solver* s, const double* vc, const double* vf, double* ef) {
  Level& L0 = s->L[0];
  Level& F = s->F;
  int rc;
  HIPTRY(launch_zero_valid<double>(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info, ef,
                                   1));
  HIPTRY(launch_zero_valid<double>(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info,
                                   L0.e64, 1));
  // the fine level gets twice the sweeps of the coarse V-cycle on each side: it
  // is a small share of the cells, and two sweeps leave its error decaying at
  // about 0.5 per correction against about 0.35 with four
  if ((rc = fine_sweeps<double>(s, ef, L0.e64, vf, 2 * s->opts.nu1))) return rc;
  // residual the fine correction leaves: fine part into rf2, coarse part into
  // L0.rhs64 with covered cells = mean of rf2's children
  if ((rc = composite_residual<double>(s, L0.e64, ef, vc, 0, vf, 0, L0.rhs64, s->rf2, nullptr,
                                       s->rf2)))
    return rc;
  // one coarse V-cycle from zero on the whole coarse level
  if ((rc = coarse_cycle<double>(s, 0, false))) return rc;
  HIPTRY(launch_prolong_add<double>(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info,
                                    L0.d_info, ef, L0.e64));
  return fine_sweeps<double>(s, ef, L0.e64, vf, 2 * s->opts.nu2);
}

// One two-level correction of the composite residual (Rc, Rf) applied to phi
// (FP32 correction: phi updated in FP64).
int composite_correction(mg_solver* s, double* phic, double* phif) {
  Level& L0 = s->L[0];
  Level& F = s->F;
  int rc;
  if (s->opts.precision == MG_PREC_F32_REFINE) {
    if ((rc = correction_core32(s, s->Rc, s->Rf))) return rc;
    HIPTRY(launch_update(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info, phif,
                         s->ef32));
    HIPTRY(launch_update(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info, phic,
                         L0.e32));
  } else {
    if ((rc = correction_core64(s, s->Rc, s->Rf, s->ef))) return rc;
    HIPTRY(launch_axpy_valid(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info, phif,
                             s->ef));
    HIPTRY(launch_axpy_valid(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info, phic,
                             L0.e64));
  }
  return avgdown<double>(s, phif, 1, phic, 1, 0);
}

// Flexible GMRES on the composite system, right-preconditioned by the
// two-level correction (z_j = M v_j kept, as the correction's bottom CG makes
// M vary slightly).  Basis vectors are ghost-free pairs (fine, coarse) with
// covered coarse entries zero; dot products run over fine cells and coarse
// cells.  Each cycle starts from the true composite residual (its max norm
// is the stop test and the history entry) and ends when the Givens estimate
// of the residual's 2-norm reaches tol times the cycle's starting 2-norm /
// max-norm ratio, at the restart length or when max_iter corrections are
// used; then phi += sum y_j z_j and covered coarse cells are averaged down.
int solve_amr_fgmres(mg_solver* s, double* Pc, double* Pf, const double* Fc, int fc_ng,
                     const double* Ff, int ff_ng, double tol, mg_info_t* inf,
                     double* resid_history) {
  Level& L0 = s->L[0];
  Level& F = s->F;
  const int m = s->gm_m;
  const bool f32 = s->opts.precision == MG_PREC_F32_REFINE;
  const int ntf = (int)F.t_cell.size(), ntc = (int)L0.t_vec.size(), np = ntf + ntc;
  const long long sf = F.n_g0, sc = L0.n_g0, zf = F.n_g1, zc = L0.n_g1;
  int rc;
  int total = 0, hist = 0, status = MG_OK;
  double rn = 0;
  std::vector<double> H((m + 1) * m), g(m + 1), cs(m), sn(m), y(m);
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  // dots of w (fine wf, coarse wc) with basis vectors 0..n-1 -> s->d_gm[0..n)
  auto mdot = [&](const double* wf, const double* wc, const double* Vf, const double* Vc,
                  int n) -> int {
    HIPTRY(launch_mdot(s->st, F.d_cell, ntf, F.s_cell, F.d_info, wf, Vf, sf, n, s->gm_part, np,
                       0));
    HIPTRY(launch_mdot(s->st, L0.d_vec, ntc, L0.s_vec, L0.d_info, wc, Vc, sc, n, s->gm_part, np,
                       ntf));
    HIPTRY(launch_sum_rows(s->st, s->gm_part, n, np, s->d_gm));
    return MG_OK;
  };
  auto readback = [&](int n) -> int {
    HIPTRY(hipMemcpyAsync(s->h_gm, s->d_gm, sizeof(double) * n, hipMemcpyDeviceToHost, s->st));
    HIPTRY(hipStreamSynchronize(s->st));
    return MG_OK;
  };
  while (true) {
    HIPTRY(launch_fill_u64(s->st, norm_slot(s, 1), kNormSlot, 0ull));
    if ((rc = composite_residual<double>(s, Pc, Pf, Fc, fc_ng, Ff, ff_ng, s->Rc, s->Rf,
                                         norm_slot(s, 1), nullptr)))
      return rc;
    if ((rc = read_norm(s, 1, &rn))) return rc;
    if (resid_history) resid_history[hist] = rn;
    ++hist;
    if (s->opts.verbose) fprintf(stderr, "amrmg composite fgmres %d  max|R| = %.6e\n", total, rn);
    if (!std::isfinite(rn)) {
      status = fail(MG_ERR_NAN, "residual norm is not finite");
      break;
    }
    if (rn <= tol) {
      inf->converged = 1;
      break;
    }
    if (total >= s->opts.max_iter) {
      status = fail(MG_ERR_NOT_CONVERGED, "max_iter reached");
      break;
    }
    // v_0 = R / ||R||
    if ((rc = mdot(s->Rf, s->Rc, s->Rf, s->Rc, 1))) return rc;
    HIPTRY(launch_vnormalise(s->st, F.d_cell, ntf, F.s_cell, F.d_info, s->Rf, s->gm_Vf, s->d_gm));
    HIPTRY(launch_vnormalise(s->st, L0.d_vec, ntc, L0.s_vec, L0.d_info, s->Rc, s->gm_Vc, s->d_gm));
    if ((rc = readback(1))) return rc;
    const double beta = std::sqrt(s->h_gm[0]);
    const double target = tol * beta / rn;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double* Zfj = s->gm_Zf + j * zf;
      double* Zcj = s->gm_Zc + j * zc;
      const double* Vfj = s->gm_Vf + j * sf;
      const double* Vcj = s->gm_Vc + j * sc;
      // z_j = M v_j
      if (f32) {
        if ((rc = correction_core32(s, Vcj, Vfj))) return rc;
        HIPTRY((launch_convert<float, double>(s->st, s->ef32, Zfj, F.n_g1)));
        HIPTRY((launch_convert<float, double>(s->st, L0.e32, Zcj, L0.n_g1)));
      } else {
        if ((rc = correction_core64(s, Vcj, Vfj, Zfj))) return rc;
        HIPTRY(hipMemcpyAsync(Zcj, L0.e64, sizeof(double) * L0.n_g1, hipMemcpyDeviceToDevice,
                              s->st));
      }
      // W = 0 - A z_j (covered coarse entries zero), then classical
      // Gram-Schmidt of A z_j = -W against v_0..v_j into slot j+1
      if ((rc = composite_residual<double>(s, Zcj, Zfj, s->gm_zero_c, 0, s->gm_zero_f, 0,
                                           s->gm_Wc, s->gm_Wf, nullptr, nullptr)))
        return rc;
      if ((rc = mdot(s->gm_Wf, s->gm_Wc, s->gm_Vf, s->gm_Vc, j + 1))) return rc;
      double* Vf1 = s->gm_Vf + (j + 1) * sf;
      double* Vc1 = s->gm_Vc + (j + 1) * sc;
      HIPTRY(launch_maxpy(s->st, F.d_cell, ntf, F.s_cell, F.d_info, s->gm_Wf, s->gm_Vf, sf, j + 1,
                          s->d_gm, -1.0, Vf1, s->gm_part, 0));
      HIPTRY(launch_maxpy(s->st, L0.d_vec, ntc, L0.s_vec, L0.d_info, s->gm_Wc, s->gm_Vc, sc, j + 1,
                          s->d_gm, -1.0, Vc1, s->gm_part, ntf));
      HIPTRY(launch_sum_rows(s->st, s->gm_part, 1, np, s->d_gm + m + 1));
      HIPTRY(hipMemcpyAsync(s->h_gm, s->d_gm, sizeof(double) * (m + 2), hipMemcpyDeviceToHost,
                            s->st));
      HIPTRY(hipStreamSynchronize(s->st));
      const double hn = std::sqrt(s->h_gm[m + 1]);
      for (int i = 0; i <= j; ++i) Hij(i, j) = -s->h_gm[i];
      Hij(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
        Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
        Hij(i, j) = t;
      }
      const double r = std::hypot(Hij(j, j), Hij(j + 1, j));
      cs[j] = Hij(j, j) / r;
      sn[j] = Hij(j + 1, j) / r;
      Hij(j, j) = r;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      k = j + 1;
      if (hn == 0.0 || std::fabs(g[j + 1]) <= target || total >= s->opts.max_iter) break;
      HIPTRY(launch_vnormalise(s->st, F.d_cell, ntf, F.s_cell, F.d_info, Vf1, Vf1,
                               s->d_gm + m + 1));
      HIPTRY(launch_vnormalise(s->st, L0.d_vec, ntc, L0.s_vec, L0.d_info, Vc1, Vc1,
                               s->d_gm + m + 1));
    }
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= Hij(i, l) * y[l];
      y[i] = acc / Hij(i, i);
    }
    std::memcpy(s->h_gm, y.data(), sizeof(double) * k);
    HIPTRY(hipMemcpyAsync(s->d_gm, s->h_gm, sizeof(double) * k, hipMemcpyHostToDevice, s->st));
    HIPTRY(launch_zaxpy(s->st, F.d_cell, ntf, F.s_cell, F.d_info, Pf, s->gm_Zf, zf, k, s->d_gm));
    HIPTRY(launch_zaxpy(s->st, L0.d_vec, ntc, L0.s_vec, L0.d_info, Pc, s->gm_Zc, zc, k, s->d_gm));
    if ((rc = avgdown<double>(s, Pf, 1, Pc, 1, 0))) return rc;
    HIPTRY(hipStreamSynchronize(s->st));  // h_gm is reused by the next cycle
  }
  inf->iters = total;
  inf->abs_resid = rn;
  return status;
}

int check_mf_boxes(const std::vector<IBox>& boxes, const mg_multifab_t* mf, int ng_min, int ng_max,
                   int face_d, const char* what) {
  if (!mf) return fail(MG_ERR_ARG, std::string(what) + " is null");
  if (mf->nbox != (int)boxes.size() || !mf->boxes || !mf->offsets || !mf->data)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": box count or pointers differ");
  if (mf->dtype != MG_F64 || mf->ncomp != 1)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": must be MG_F64 with one component");
  if (mf->ngrow < ng_min || mf->ngrow > ng_max)
    return fail(MG_ERR_MISMATCH, std::string(what) + ": unsupported ngrow");
  for (int d = 0; d < 3; ++d)
    if (mf->ixtype[d] != (d == face_d ? 1 : 0))
      return fail(MG_ERR_MISMATCH, std::string(what) + ": wrong index type");
  int64_t off = 0;
  for (size_t b = 0; b < boxes.size(); ++b) {
    if (!same(to_ibox(mf->boxes[b]), boxes[b]))
      return fail(MG_ERR_MISMATCH, std::string(what) + ": box " + std::to_string(b) + " differs");
    if (mf->offsets[b] != off)
      return fail(MG_ERR_MISMATCH, std::string(what) + ": non-canonical offsets");
    off += grown_volume(boxes[b], mf->ngrow, face_d);
  }
  return MG_OK;
}

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

void mg_default_opts(mg_opts_t* o) {
  if (!o) return;
  o->nu1 = 2;
  o->nu2 = 2;
  o->max_iter = 100;
  o->bottom_max_iter = 0;
  o->min_bottom_edge = 4;
  o->precision = MG_PREC_F64;
  o->use_graph = 1;
  o->tune = 1;
  o->verbose = 0;
  o->aggregate = 0;
  o->bottom_rel_tol = 1e-4;
  o->fused_min_edge = 0;
  o->krylov = 0;
  o->ghost_write = 1;
  o->interp_fold = 1;
  o->bottom_solver = 0;
  o->restrict_fold = 1;
  o->stop_fold = 1;
  o->coarse_tail = 1024;
}

static int check_opts(const mg_opts_t* o) {
  if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 == 0) return fail(MG_ERR_ARG, "bad nu1/nu2");
  if (o->max_iter < 0) return fail(MG_ERR_ARG, "max_iter < 0");
  if (o->min_bottom_edge < 1) return fail(MG_ERR_ARG, "min_bottom_edge < 1");
  if (o->precision != MG_PREC_F64 && o->precision != MG_PREC_F32_REFINE)
    return fail(MG_ERR_ARG, "bad precision");
  if (o->tune < 0 || o->tune > 2) return fail(MG_ERR_ARG, "bad tune");
  if (!(o->bottom_rel_tol >= 0)) return fail(MG_ERR_ARG, "bad bottom_rel_tol");
  if (o->fused_min_edge < 0) return fail(MG_ERR_ARG, "fused_min_edge < 0");
  if (o->krylov != 0 && o->krylov != 1) return fail(MG_ERR_ARG, "bad krylov");
  if (o->ghost_write != 0 && o->ghost_write != 1) return fail(MG_ERR_ARG, "bad ghost_write");
  if (o->interp_fold != 0 && o->interp_fold != 1) return fail(MG_ERR_ARG, "bad interp_fold");
  if (o->bottom_solver != 0 && o->bottom_solver != 1) return fail(MG_ERR_ARG, "bad bottom_solver");
  if (o->restrict_fold < 0 || o->restrict_fold > 2) return fail(MG_ERR_ARG, "bad restrict_fold");
  if (o->stop_fold != 0 && o->stop_fold != 1) return fail(MG_ERR_ARG, "bad stop_fold");
  if (o->coarse_tail < 0) return fail(MG_ERR_ARG, "coarse_tail < 0");
  return MG_OK;
}

int mg_query_workspace(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                       const mg_opts_t* opts, int32_t has_acoef, size_t* bytes) {
  if (!boxes || nbox <= 0 || !bytes) return fail(MG_ERR_ARG, "null boxes or size pointer");
  std::unique_ptr<mg_solver> s(new mg_solver());
  if (opts)
    s->opts = *opts;
  else
    mg_default_opts(&s->opts);
  int rc;
  if ((rc = check_opts(&s->opts))) return rc;
  if ((rc = check_geom(geom, nullptr, nullptr, s.get()))) return rc;
  s->has_a = has_acoef != 0;
  std::vector<IBox> bx(nbox);
  for (int i = 0; i < nbox; ++i) bx[i] = to_ibox(boxes[i]);
  Bump bump{nullptr};
  if ((rc = build_plan(s.get(), bx, bump))) return rc;
  *bytes = s->ws_need;
  return MG_OK;
}

int mg_num_levels(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom,
                  const mg_opts_t* opts, int32_t* nlevels) {
  if (!boxes || nbox <= 0 || !nlevels || !geom) return fail(MG_ERR_ARG, "null argument");
  mg_opts_t o;
  if (opts)
    o = *opts;
  else
    mg_default_opts(&o);
  std::vector<IBox> bx(nbox);
  for (int i = 0; i < nbox; ++i) bx[i] = to_ibox(boxes[i]);
  std::string err;
  const IBox dom = to_ibox(geom->domain);
  if (!validate_boxes(bx, dom, true, &err)) return fail(MG_ERR_INVALID_BOXARRAY, err);
  *nlevels = (int32_t)hierarchy(bx, dom, o.min_bottom_edge, o.aggregate != 0).size();
  return MG_OK;
}

int mg_create(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom, const int32_t bc_lo[3],
              const int32_t bc_hi[3], double alpha, double beta, const mg_multifab_t* acoef,
              const mg_multifab_t* const* bcoef, const mg_opts_t* opts, void* workspace,
              size_t ws_bytes, void* hip_stream, mg_solver_t** out) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!out) return fail(MG_ERR_ARG, "out is null");
  *out = nullptr;
  if (!boxes || nbox <= 0) return fail(MG_ERR_ARG, "no boxes");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(MG_ERR_ARG, "alpha/beta not finite");
  std::unique_ptr<mg_solver> s(new mg_solver());
  if (opts)
    s->opts = *opts;
  else
    mg_default_opts(&s->opts);
  int rc;
  if ((rc = check_opts(&s->opts))) return rc;
  if ((rc = check_geom(geom, bc_lo, bc_hi, s.get()))) return rc;
  s->alpha = alpha;
  s->beta = beta;
  s->has_a = acoef != nullptr;
  std::vector<IBox> bx(nbox);
  for (int i = 0; i < nbox; ++i) bx[i] = to_ibox(boxes[i]);
  {
    Bump measure{nullptr};
    if ((rc = build_plan(s.get(), bx, measure))) return rc;
  }
  if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is null");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(MG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < s->ws_need)
    return fail(MG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(s->ws_need) +
                                      " bytes, got " + std::to_string(ws_bytes));
  {
    Bump real{static_cast<char*>(workspace)};
    if ((rc = build_plan(s.get(), bx, real))) return rc;
  }
  set_h(s.get(), geom);
  s->ws = static_cast<char*>(workspace);
  s->ws_bytes = ws_bytes;
  s->singular = is_singular_problem(s.get());
  // coefficient MultiFabs
  if (acoef && (rc = check_mf(s.get(), acoef, MG_F64, 0, 0, -1, "acoef"))) return rc;
  if (bcoef)
    for (int d = 0; d < 3; ++d)
      if ((rc = check_mf(s.get(), bcoef[d], MG_F64, 0, 0, d, "bcoef"))) return rc;
  s->user = static_cast<hipStream_t>(hip_stream);
  HIPTRY(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
  HIPTRY(hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
  HIPTRY(hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
  for (hipEvent_t& e : s->ev_norm) HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPTRY(hipHostMalloc((void**)&s->h_norm, sizeof(unsigned long long) * (3 * kNormSlot + 8),
                       hipHostMallocDefault));
  s->h_iters = reinterpret_cast<int*>(s->h_norm + 3 * kNormSlot);
  {
    CallScope call(s.get());
    if ((rc = call.rc())) return rc;
    if ((rc = upload_tables(s.get()))) return rc;
    if ((rc = setup_coefficients(s.get(), acoef, bcoef))) return rc;
    if ((rc = coarsen_all(s.get()))) return rc;
    if ((rc = autotune(s.get()))) return rc;
    if ((rc = capture_graphs(s.get()))) return rc;
    HIPTRY(hipStreamSynchronize(s->st));
    if ((rc = call.finish())) return rc;
  }
  s->setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = s.release();
  return MG_OK;
}

int mg_set_coefficients(mg_solver_t* s, const mg_multifab_t* acoef,
                        const mg_multifab_t* const* bcoef) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  if ((acoef != nullptr) != s->has_a)
    return fail(MG_ERR_ARG, "acoef presence must match mg_create");
  int rc;
  if (acoef && (rc = check_mf(s, acoef, MG_F64, 0, 0, -1, "acoef"))) return rc;
  if (bcoef)
    for (int d = 0; d < 3; ++d)
      if ((rc = check_mf(s, bcoef[d], MG_F64, 0, 0, d, "bcoef"))) return rc;
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  if ((rc = setup_coefficients(s, acoef, bcoef))) return rc;
  if ((rc = coarsen_all(s))) return rc;
  return call.finish();
}

int mg_set_coefficients_global(mg_solver_t* s, const void* acoef_global,
                               const void* const* bface_global, int32_t is_log) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  if ((acoef_global != nullptr) != s->has_a)
    return fail(MG_ERR_ARG, "acoef presence must match mg_create");
  if (!bface_global) return fail(MG_ERR_ARG, "bface_global is null");
  for (int d = 0; d < 3; ++d)
    if (!bface_global[d]) return fail(MG_ERR_ARG, "bface_global entry is null");
  int rc;
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  Level& l0 = s->L[0];
  const int dlo[3] = {s->domain.lo[0], s->domain.lo[1], s->domain.lo[2]};
  const int dn[3] = {ext(s->domain, 0), ext(s->domain, 1), ext(s->domain, 2)};
  for (int d = 0; d < 3; ++d) {
    HIPTRY(launch_scatter_faces(s->st, l0.d_info, l0.nbox, d, dlo, dn,
                                (const double*)bface_global[d], l0.b64[d], is_log ? 1 : 0,
                                l0.max_faces));
  }
  if (acoef_global)
    HIPTRY(launch_scatter_cells(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, l0.d_info, dlo,
                                dn, (const double*)acoef_global, l0.a64));
  if ((rc = coarsen_all(s))) return rc;
  return call.finish();
}

// Preconditioned conjugate gradients on level 0 with one symmetric V-cycle
// (zero guess, post-smoothing black then red) as the preconditioner: the
// paper's Krylov CG with its multigrid inside.  x = P (ng 1) in place;
// r = L0.rhs64 (the V-cycle's right-hand side), z = L0.e64 (its result),
// p = L0.p64, q = A p in L0.r64 (free again once the V-cycle has returned).
// The max-norm stop test runs on the recurrence residual and is confirmed on
// the true one; if that is still above tol, r is replaced by it and the
// recurrence restarts from p = M r.  Scalars stay on the device: d_cg[0..1]
// hold rho = r.z of alternate iterations, d_cg[2] = p.q.
int solve_pcg(mg_solver* s, double* P, const double* F, int rng, double tol, mg_info_t* inf,
              double* resid_history) {
  Level& l0 = s->L[0];
  const StencilArgs<double> op = stencil_of<double>(s, l0, false);
  const int nt = (int)l0.t_cell.size();
  const Shape sh = l0.s_cell;
  // vector kernels (dots, updates, shifts) on the deep tiles
  const Tile* vt = l0.d_vec;
  const int nv = (int)l0.t_vec.size();
  const Shape sv = l0.s_vec;
  double* r = l0.rhs64;
  double* z = l0.e64;
  double* p = l0.p64;
  double* q = l0.r64;
  int rc;
  // r = f - A x (into buf), mean taken out when singular; max |r| read back
  auto true_residual = [&](double* buf, double* norm) -> int {
    HIPTRY(launch_fill_u64(s->st, norm_slot(s, 2), kNormSlot, 0ull));
    if ((rc = exchange<double>(s, l0, P, false))) return rc;
    {
      ProfScope ps(s, 1, true);
      HIPTRY((launch_residual<double, double>(s->st, l0.d_cell, nt, sh, op, P, F, rng, buf,
                                              s->singular ? nullptr : norm_slot(s, 2), 0)));
    }
    if (s->singular) {
      HIPTRY(launch_sum_valid(s->st, vt, nv, sv, l0.d_info, buf, 0, s->d_partials, s->d_sum));
      HIPTRY(launch_shift_valid(s->st, vt, nv, sv, l0.d_info, buf, 0, s->d_sum, l0.ncell));
      HIPTRY(launch_maxabs<double>(s->st, vt, nv, sv, l0.d_info, buf, 0, norm_slot(s, 2)));
    }
    return read_norm(s, 2, norm);
  };
  const bool f32 = s->opts.precision == MG_PREC_F32_REFINE;
  double rn;
  if ((rc = true_residual(r, &rn))) return rc;
  int it = 0, status = MG_OK;
  bool restart = true;
  bool r32_current = false;  // FP32 copy of r written by the last update
  while (true) {
    if (resid_history) resid_history[it] = rn;
    if (s->opts.verbose) fprintf(stderr, "amrmg pcg %d  max|r| = %.6e\n", it, rn);
    if (!std::isfinite(rn)) {
      status = fail(MG_ERR_NAN, "residual norm is not finite");
      break;
    }
    if (rn <= tol) {
      double rt;
      if ((rc = true_residual(q, &rt))) return rc;
      if (rt <= tol) {
        inf->converged = 1;
        break;
      }
      HIPTRY(hipMemcpyAsync(r, q, sizeof(double) * l0.n_g0, hipMemcpyDeviceToDevice, s->st));
      restart = true;
      r32_current = false;
    }
    if (it == s->opts.max_iter) {
      status = fail(MG_ERR_NOT_CONVERGED, "max_iter reached");
      break;
    }
    // z = M r, the V-cycle in FP64, or in FP32 on r rounded to FP32 (the
    // mixed-precision preconditioner; CG itself stays in FP64)
    double* rho_new = s->d_cg + (it & 1);
    double* rho_old = s->d_cg + ((it + 1) & 1);
    if (f32) {
      if (!r32_current) HIPTRY((launch_convert<double, float>(s->st, r, l0.rhs32, l0.n_g0)));
      if ((rc = coarse_cycle<float>(s, 0, true))) return rc;
    } else {
      if ((rc = coarse_cycle<double>(s, 0, false))) return rc;
    }
    {
      ProfScope ps_dot(s, 6, true);
      if (s->singular) {
        if (f32) HIPTRY((launch_convert<float, double>(s->st, l0.e32, z, l0.n_g1)));
        HIPTRY(launch_sum_valid(s->st, vt, nv, sv, l0.d_info, z, 1, s->d_partials, s->d_sum));
        HIPTRY(launch_shift_valid(s->st, vt, nv, sv, l0.d_info, z, 1, s->d_sum, l0.ncell));
        HIPTRY(launch_dot(s->st, vt, nv, sv, l0.d_info, r, 0, z, 1, s->d_partials, rho_new));
      } else if (f32) {
        // z = FP64 of the FP32 V-cycle result and rho = r.z in one pass
        HIPTRY(launch_widen_dot(s->st, vt, nv, sv, l0.d_info, l0.e32, z, r, s->d_partials,
                                rho_new));
      } else {
        HIPTRY(launch_dot(s->st, vt, nv, sv, l0.d_info, r, 0, z, 1, s->d_partials, rho_new));
      }
    }
    {
      ProfScope ps(s, 6, true);
      HIPTRY(launch_cg_p(s->st, vt, nv, sv, l0.d_info, p, z, rho_new, rho_old, restart ? 1 : 0));
    }
    restart = false;
    // q = A p, alpha = rho_new / p.q
    if ((rc = exchange<double>(s, l0, p, true))) return rc;
    {
      // q = A p with the per-tile partials of p.q from the same pass
      ProfScope ps(s, 1, true);
      HIPTRY((launch_residual<double, double>(s->st, l0.d_cell, nt, sh, op, p, nullptr, 0, q,
                                              nullptr, 1, s->d_partials)));
    }
    {
      ProfScope ps(s, 6, true);
      HIPTRY(launch_sum_final(s->st, s->d_partials, nt, s->d_cg + 2));
    }
    HIPTRY(launch_fill_u64(s->st, norm_slot(s, 2), kNormSlot, 0ull));
    {
      ProfScope ps(s, 6, true);
      HIPTRY(launch_cg_xr(s->st, vt, nv, sv, l0.d_info, P, p, r, q, rho_new, s->d_cg + 2,
                          norm_slot(s, 2), f32 ? l0.rhs32 : nullptr));
      r32_current = f32;
    }
    ++it;
    if ((rc = read_norm(s, 2, &rn))) return rc;
  }
  inf->iters = it;
  inf->abs_resid = rn;
  return status;
}

// FP64 V-cycles with the stop test's residual folded into the next cycle's
// first half-sweep: one pass computes max|f - A phi| of the current iterate
// and writes that iterate after a red half-sweep into the other level-0
// array, where the cycle goes on, so the iterates alternate between the
// caller's phi and next64.  The norm is copied to the host while the rest
// of the cycle runs and read before the next pass (which overwrites the
// iterate it was taken of); while the norms' geometric trend puts the next
// one well above the tolerance the cycle is queued before the norm is read,
// else after (a converged solve would otherwise run one cycle for nothing).
// Same iterates, norms, decisions and result as the plain loop.
int solve_folded(mg_solver* s, double* P, const double* F, int rng, double tol, mg_info_t* inf,
                 double* hist, int* status) {
  Level& l0 = s->L[0];
  const StencilArgs<double> op = stencil_of<double>(s, l0, false);
  double* cur = P;
  double* nxt = l0.next64;
  int rc;
  int it = 0, rising = 0;
  double rn = 0, first = 0, prev = 0, prev2 = 0;
  *status = MG_OK;
  // 1 = stop, 0 = go on
  auto decide = [&]() -> int {
    if (hipEventSynchronize(s->ev_norm[it & 1]) != hipSuccess) return -1;
    const unsigned long long* h = s->h_norm + (size_t)(1 + (it & 1)) * kNormSlot;
    unsigned long long m = 0;
    for (int w = 0; w < kNormWays; ++w) m = std::max(m, h[w * kNormStride]);
    std::memcpy(&rn, &m, sizeof(double));
    if (hist) hist[it] = rn;
    if (s->opts.verbose) fprintf(stderr, "amrmg cycle %d  max|r| = %.6e\n", it, rn);
    if (!std::isfinite(rn)) {
      *status = fail(MG_ERR_NAN, "residual norm is not finite");
      return 1;
    }
    if (it == 0) first = rn;
    if (rn <= tol) {
      inf->converged = 1;
      return 1;
    }
    if (it == s->opts.max_iter) {
      *status = fail(MG_ERR_NOT_CONVERGED, "max_iter reached");
      return 1;
    }
    if (it > 0) rising = rn > prev ? rising + 1 : 0;
    if (rising >= 3 && rn > first) {
      *status = fail(MG_ERR_DIVERGED, "residual grew for 3 cycles");
      return 1;
    }
    prev2 = prev;
    prev = rn;
    return 0;
  };
  while (true) {
    // the caller's ghosts may be stale; after a cycle they are current where
    // its post-smoothing wrote through
    if ((it == 0 || !l0.wt || s->opts.nu2 == 0) && (rc = exchange<double>(s, l0, cur, false)))
      return rc;
    const int slot = 1 + (it & 1);
    HIPTRY(launch_fill_u64(s->st, norm_slot(s, slot), kNormSlot, 0ull));
    {
      ProfScope ps(s, 1, true);
      // with write-through the pass also puts its red values into nxt's face
      // ghosts, and the black half-sweep that follows reads nothing else
      HIPTRY((launch_residual<double, double>(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell,
                                              op, cur, F, rng, nullptr, norm_slot(s, slot), 0,
                                              nullptr, nxt, l0.wt ? l0.d_wtbox : nullptr,
                                              l0.wt ? l0.d_wt : nullptr)));
    }
    HIPTRY(hipMemcpyAsync(s->h_norm + (size_t)slot * kNormSlot, norm_slot(s, slot),
                          sizeof(unsigned long long) * kNormSlot, hipMemcpyDeviceToHost, s->st));
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
    if (!l0.wt && (rc = exchange<double>(s, l0, nxt, false))) return rc;
    if ((rc = vcycle64(s, nxt, F, rng, true))) return rc;
    if (!wait) {
      const int d = decide();
      if (d < 0) return fail(MG_ERR_HIP, "norm read-back failed");
      if (d) break;
    }
    std::swap(cur, nxt);
    ++it;
  }
  if (cur != P)
    HIPTRY(hipMemcpyAsync(P, cur, sizeof(double) * l0.n_g1, hipMemcpyDeviceToDevice, s->st));
  inf->iters = it;
  inf->abs_resid = rn;
  return MG_OK;
}

int mg_solve(mg_solver_t* s, mg_multifab_t* phi, const mg_multifab_t* rhs, double rel_tol,
             double abs_tol, mg_info_t* info, double* resid_history) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!s) return fail(MG_ERR_ARG, "null solver");
  int rc;
  if ((rc = check_mf(s, phi, MG_F64, 1, 1, -1, "phi"))) return rc;
  if ((rc = check_mf(s, rhs, MG_F64, 0, 1, -1, "rhs"))) return rc;
  if (!(rel_tol >= 0) || !(abs_tol >= 0)) return fail(MG_ERR_ARG, "negative tolerance");
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  Level& l0 = s->L[0];
  double* P = static_cast<double*>(phi->data);
  const double* F = static_cast<const double*>(rhs->data);
  const int rng = rhs->ngrow;
  const bool f32 = s->opts.precision == MG_PREC_F32_REFINE;
  const StencilArgs<double> op = stencil_of<double>(s, l0, false);
  mg_info_t inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.nlevels = (int)s->L.size();
  inf.tail_level = std::max(s->tail_lev, 0);
  inf.setup_ms = s->setup_ms;

  HIPTRY(launch_fill_u64(s->st, s->d_norm, 4 * kNormSlot, 0ull));
  HIPTRY(launch_maxabs<double>(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, l0.d_info, F,
                               rng, s->d_norm));
  double normf;
  if ((rc = read_norm(s, 0, &normf))) return rc;
  int status = MG_OK;
  if (!std::isfinite(normf)) return fail(MG_ERR_NAN, "rhs holds a non-finite value");
  if (normf == 0.0) {
    HIPTRY(launch_zero_valid<double>(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, l0.d_info,
                                     P, 1));
    HIPTRY(hipStreamSynchronize(s->st));
    inf.converged = 1;
    if (resid_history) resid_history[0] = 0.0;
  } else if (s->opts.krylov) {
    status = solve_pcg(s, P, F, rng, std::max(rel_tol * normf, abs_tol), &inf, resid_history);
    inf.rel_resid = inf.abs_resid / normf;
  } else if (l0.next64) {
    if ((rc = solve_folded(s, P, F, rng, std::max(rel_tol * normf, abs_tol), &inf, resid_history,
                           &status)))
      return rc;
    inf.rel_resid = inf.abs_resid / normf;
  } else {
    const double tol = std::max(rel_tol * normf, abs_tol);
    int it = 0, rising = 0;
    double rn = 0, first = 0, prev = 0;
    while (true) {
      HIPTRY(launch_fill_u64(s->st, norm_slot(s, 1), kNormSlot, 0ull));
      // after an FP64 V-cycle whose post-smoothing wrote through, phi's face
      // ghosts are current; the refinement update touches valid cells only
      if ((f32 || it == 0 || !l0.wt || s->opts.nu2 == 0) &&
          (rc = exchange<double>(s, l0, P, false)))
        return rc;
      {
        ProfScope ps(s, 1, true);
        if (f32)
          HIPTRY((launch_residual<double, float>(s->st, l0.d_cell, (int)l0.t_cell.size(),
                                                 l0.s_cell, op, P, F, rng, l0.rhs32, norm_slot(s, 1),
                                                 0)));
        else
          HIPTRY((launch_residual<double, double>(s->st, l0.d_cell, (int)l0.t_cell.size(),
                                                  l0.s_cell, op, P, F, rng, nullptr,
                                                  norm_slot(s, 1), 0)));
      }
      if ((rc = read_norm(s, 1, &rn))) return rc;
      if (resid_history) resid_history[it] = rn;
      if (s->opts.verbose) fprintf(stderr, "amrmg cycle %d  max|r| = %.6e\n", it, rn);
      if (!std::isfinite(rn)) {
        status = fail(MG_ERR_NAN, "residual norm is not finite");
        break;
      }
      if (it == 0) first = rn;
      if (rn <= tol) {
        inf.converged = 1;
        break;
      }
      if (it == s->opts.max_iter) {
        status = fail(MG_ERR_NOT_CONVERGED, "max_iter reached");
        break;
      }
      if (it > 0) rising = rn > prev ? rising + 1 : 0;
      if (rising >= 3 && rn > first) {
        status = fail(MG_ERR_DIVERGED, "residual grew for 3 cycles");
        break;
      }
      prev = rn;
      if (f32) {
        if ((rc = coarse_cycle<float>(s, 0, true))) return rc;
        ProfScope ps(s, 6, true);
        HIPTRY(launch_update(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, l0.d_info, P,
                             l0.e32));
      } else {
        if ((rc = vcycle64(s, P, F, rng))) return rc;
      }
      ++it;
    }
    inf.iters = it;
    inf.abs_resid = rn;
    inf.rel_resid = rn / normf;
  }
  if (s->singular) {
    HIPTRY(launch_sum_valid(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, l0.d_info, P, 1,
                            s->d_partials, s->d_sum));
    HIPTRY(launch_shift_valid(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, l0.d_info, P, 1,
                              s->d_sum, l0.ncell));
  }
  HIPTRY(hipMemcpyAsync(s->h_iters, s->d_iters, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPTRY(hipStreamSynchronize(s->st));
  inf.bottom_iters = *s->h_iters;
  if ((rc = call.finish())) return rc;
  inf.solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

int mg_apply(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* out) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  int rc;
  if ((rc = check_mf(s, phi, MG_F64, 1, 1, -1, "phi"))) return rc;
  if ((rc = check_mf(s, out, MG_F64, 0, 0, -1, "out"))) return rc;
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  Level& l0 = s->L[0];
  if ((rc = exchange<double>(s, l0, (double*)phi->data, false))) return rc;
  HIPTRY((launch_residual<double, double>(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell,
                                          stencil_of<double>(s, l0, false),
                                          (const double*)phi->data, nullptr, 0,
                                          (double*)out->data, nullptr, 1)));
  return call.finish();
}

static int face_grad_check(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* lam) {
  int rc;
  if ((rc = check_mf(s, phi, MG_F64, 1, 1, -1, "phi"))) return rc;
  if ((rc = check_mf(s, lam, MG_F64, 1, 1, -1, "lam"))) return rc;
  return MG_OK;
}

// Ghost exchange of phi and lambda, then the face-gradient launches.
static int face_grad_run(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* lam, void* const* out,
                         int mode) {
  int rc;
  Level& l0 = s->L[0];
  if ((rc = exchange<double>(s, l0, (double*)phi->data, false))) return rc;
  if ((rc = exchange<double>(s, l0, (double*)lam->data, false))) return rc;
  const int dlo[3] = {s->domain.lo[0], s->domain.lo[1], s->domain.lo[2]};
  const int dn[3] = {ext(s->domain, 0), ext(s->domain, 1), ext(s->domain, 2)};
  int max_n[3] = {0, 0, 0};
  for (const IBox& b : l0.boxes)
    for (int d = 0; d < 3; ++d) max_n[d] = std::max(max_n[d], ext(b, d));
  // 32-bit offsets inside a box's face arrays
  if ((int64_t)(max_n[0] + 1) * (max_n[1] + 1) * (max_n[2] + 1) >= (int64_t(1) << 31))
    return fail(MG_ERR_ARG, "face gradient: a box is too large for 32-bit face offsets");
  const int perbits = (s->periodic[0] ? 1 : 0) | (s->periodic[1] ? 2 : 0) |
                      (s->periodic[2] ? 4 : 0);
  double* const o[3] = {(double*)out[0], (double*)out[1], (double*)out[2]};
  ProfScope ps(s, 8, true);
  HIPTRY(launch_face_grad(s->st, l0.nbox, stencil_of<double>(s, l0, false),
                          (const double*)phi->data, (const double*)lam->data, o, mode, dlo, dn,
                          perbits, max_n));
  return MG_OK;
}

int mg_face_grad_logb(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* lam,
                      mg_multifab_t* const* grad) {
  if (!s || !grad) return fail(MG_ERR_ARG, "null argument");
  int rc;
  for (int d = 0; d < 3; ++d)
    if ((rc = check_mf(s, grad[d], MG_F64, 0, 0, d, "grad"))) return rc;
  if ((rc = face_grad_check(s, phi, lam))) return rc;
  void* out[3] = {grad[0]->data, grad[1]->data, grad[2]->data};
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  if ((rc = face_grad_run(s, phi, lam, out, 0))) return rc;
  return call.finish();
}

int mg_face_grad_logb_global(mg_solver_t* s, mg_multifab_t* phi, mg_multifab_t* lam,
                             void* const* grad_global) {
  if (!s || !grad_global) return fail(MG_ERR_ARG, "null argument");
  for (int d = 0; d < 3; ++d)
    if (!grad_global[d]) return fail(MG_ERR_ARG, "null gradient array");
  int rc;
  if ((rc = face_grad_check(s, phi, lam))) return rc;
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  if ((rc = face_grad_run(s, phi, lam, grad_global, 1))) return rc;
  return call.finish();
}

int mg_copy_valid(mg_solver_t* s, const mg_multifab_t* src, mg_multifab_t* dst) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  int rc;
  if ((rc = check_mf(s, src, MG_F64, 0, 1, -1, "src"))) return rc;
  if ((rc = check_mf(s, dst, MG_F64, 0, 1, -1, "dst"))) return rc;
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  Level& l0 = s->L[0];
  HIPTRY(launch_copy_valid(s->st, l0.d_cell, (int)l0.t_cell.size(), l0.s_cell, l0.d_info,
                           (const double*)src->data, src->ngrow, (double*)dst->data, dst->ngrow));
  return call.finish();
}

void mg_destroy(mg_solver_t* s) {
  if (!s) return;
  if (s->st) hipStreamSynchronize(s->st);
  if (s->graph64) hipGraphExecDestroy(s->graph64);
  if (s->graph32) hipGraphExecDestroy(s->graph32);
  for (hipEvent_t e : s->ev_pool) hipEventDestroy(e);
  if (s->ev_in) hipEventDestroy(s->ev_in);
  if (s->ev_out) hipEventDestroy(s->ev_out);
  for (hipEvent_t e : s->ev_norm)
    if (e) hipEventDestroy(e);
  if (s->h_norm) hipHostFree(s->h_norm);
  if (s->h_gm) hipHostFree(s->h_gm);
  if (s->st) hipStreamDestroy(s->st);
  delete s;
}

int mg_profile(mg_solver_t* s, int32_t enable) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  HIPTRY(hipStreamSynchronize(s->st));
  s->prof.clear();
  s->ev_used = 0;
  s->profile = enable != 0;
  return MG_OK;
}

int mg_kernel_stats(mg_solver_t* s, int32_t family, double* total_ms, int64_t* launches) {
  if (!s || !total_ms || !launches) return fail(MG_ERR_ARG, "null argument");
  HIPTRY(hipStreamSynchronize(s->st));
  double t = 0;
  int64_t n = 0;
  for (const ProfRec& r : s->prof) {
    if (r.fam != family) continue;
    float ms = 0;
    HIPTRY(hipEventElapsedTime(&ms, r.a, r.b));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return MG_OK;
}

int mg_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 ||
      reinterpret_cast<uintptr_t>(src) % 16)
    return fail(MG_ERR_ARG, "mg_stream_copy: null pointer, or size or address not 16-byte aligned");
  HIPTRY(launch_stream_copy(static_cast<hipStream_t>(hip_stream), src, dst,
                            static_cast<long long>(bytes / 16)));
  return MG_OK;
}

int mg_time_smoother(mg_solver_t* s, mg_multifab_t* phi, const mg_multifab_t* rhs, int32_t reps,
                     double* mean_ms) {
  if (!s || !mean_ms || reps <= 0) return fail(MG_ERR_ARG, "bad argument");
  int rc;
  if ((rc = check_mf(s, phi, MG_F64, 1, 1, -1, "phi"))) return rc;
  if ((rc = check_mf(s, rhs, MG_F64, 0, 1, -1, "rhs"))) return rc;
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  Level& l0 = s->L[0];
  const StencilArgs<double> op = stencil_of<double>(s, l0, false);
  hipEvent_t a, b;
  HIPTRY(hipEventCreate(&a));
  HIPTRY(hipEventCreate(&b));
  HIPTRY(hipEventRecord(a, s->st));
  for (int k = 0; k < reps; ++k)
    HIPTRY(launch_gsrb<double>(s->st, l0.d_gsrb, (int)l0.t_gsrb.size(), l0.s_gsrb, op,
                               (double*)phi->data, (const double*)rhs->data, rhs->ngrow, k & 1, 0));
  HIPTRY(hipEventRecord(b, s->st));
  HIPTRY(hipEventSynchronize(b));
  float ms;
  HIPTRY(hipEventElapsedTime(&ms, a, b));
  hipEventDestroy(a);
  hipEventDestroy(b);
  *mean_ms = ms / reps;
  return call.finish();
}

static int amr_plan(mg_solver* s, const mg_box_t* cboxes, int32_t ncb, const mg_box_t* fboxes,
                    int32_t nfb, const mg_geom_t* geom, const mg_opts_t* opts, char* ws) {
  if (!cboxes || ncb <= 0 || !fboxes || nfb <= 0) return fail(MG_ERR_ARG, "no boxes");
  if (opts)
    s->opts = *opts;
  else
    mg_default_opts(&s->opts);
  int rc;
  if ((rc = check_opts(&s->opts))) return rc;
  if ((rc = check_geom(geom, nullptr, nullptr, s))) return rc;
  for (int d = 0; d < 3; ++d)
    if (s->periodic[d]) return fail(MG_ERR_ARG, "the composite solve needs Dirichlet walls");
  s->composite = true;
  s->has_a = false;
  std::vector<IBox> cb(ncb), fb(nfb);
  for (int i = 0; i < ncb; ++i) cb[i] = to_ibox(cboxes[i]);
  for (int i = 0; i < nfb; ++i) fb[i] = to_ibox(fboxes[i]);
  Bump bump{ws};
  if ((rc = build_plan(s, cb, bump))) return rc;
  if ((rc = build_composite(s, fb, bump))) return rc;
  return MG_OK;
}

int mg_query_workspace_amr(const mg_box_t* cboxes, int32_t ncb, const mg_box_t* fboxes,
                           int32_t nfb, const mg_geom_t* geom, const mg_opts_t* opts,
                           size_t* bytes) {
  if (!bytes) return fail(MG_ERR_ARG, "bytes is null");
  std::unique_ptr<mg_solver> s(new mg_solver());
  int rc;
  if ((rc = amr_plan(s.get(), cboxes, ncb, fboxes, nfb, geom, opts, nullptr))) return rc;
  *bytes = s->ws_need;
  return MG_OK;
}

int mg_create_amr(const mg_box_t* cboxes, int32_t ncb, const mg_box_t* fboxes, int32_t nfb,
                  const mg_geom_t* geom, double alpha, double beta,
                  const mg_multifab_t* const* bcoef_c, const mg_multifab_t* const* bcoef_f,
                  const mg_opts_t* opts, void* workspace, size_t ws_bytes, void* hip_stream,
                  mg_solver_t** out) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!out) return fail(MG_ERR_ARG, "out is null");
  *out = nullptr;
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(MG_ERR_ARG, "alpha/beta not finite");
  std::unique_ptr<mg_solver> s(new mg_solver());
  int rc;
  if ((rc = amr_plan(s.get(), cboxes, ncb, fboxes, nfb, geom, opts, nullptr))) return rc;
  if (!workspace) return fail(MG_ERR_WORKSPACE, "workspace is null");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(MG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < s->ws_need)
    return fail(MG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(s->ws_need) +
                                      " bytes, got " + std::to_string(ws_bytes));
  std::unique_ptr<mg_solver> r(new mg_solver());
  if ((rc = amr_plan(r.get(), cboxes, ncb, fboxes, nfb, geom, opts, (char*)workspace))) return rc;
  s.swap(r);
  set_h(s.get(), geom);
  for (int d = 0; d < 3; ++d) s->F.h[d] = 0.5 * s->L[0].h[d];
  s->alpha = alpha;
  s->beta = beta;
  s->singular = false;
  s->ws = static_cast<char*>(workspace);
  s->ws_bytes = ws_bytes;
  if (bcoef_c)
    for (int d = 0; d < 3; ++d)
      if ((rc = check_mf(s.get(), bcoef_c[d], MG_F64, 0, 0, d, "bcoef_c"))) return rc;
  if (bcoef_f)
    for (int d = 0; d < 3; ++d)
      if ((rc = check_mf_boxes(s->F.boxes, bcoef_f[d], 0, 0, d, "bcoef_f"))) return rc;
  s->user = static_cast<hipStream_t>(hip_stream);
  HIPTRY(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
  HIPTRY(hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
  HIPTRY(hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
  HIPTRY(hipHostMalloc((void**)&s->h_norm, sizeof(unsigned long long) * (3 * kNormSlot + 8),
                       hipHostMallocDefault));
  s->h_iters = reinterpret_cast<int*>(s->h_norm + 3 * kNormSlot);
  {
    CallScope call(s.get());
    if ((rc = call.rc())) return rc;
    if ((rc = upload_tables(s.get()))) return rc;
    if ((rc = upload_composite(s.get()))) return rc;
    if (s->opts.krylov) {
      HIPTRY(hipHostMalloc((void**)&s->h_gm, sizeof(double) * (s->gm_m + 2), hipHostMallocDefault));
      HIPTRY(hipMemsetAsync(s->gm_zero_f, 0, sizeof(double) * s->F.n_g0, s->st));
      HIPTRY(hipMemsetAsync(s->gm_zero_c, 0, sizeof(double) * s->L[0].n_g0, s->st));
    }
    if ((rc = setup_coefficients(s.get(), nullptr, bcoef_c))) return rc;
    for (int d = 0; d < 3; ++d) {
      HIPTRY(launch_scale_faces(s->st, bcoef_f ? (const double*)bcoef_f[d]->data : nullptr,
                                s->F.b64[d], s->F.n_f[d], 1.0));
      if (s->F.b32[d])
        HIPTRY((launch_convert<double, float>(s->st, s->F.b64[d], s->F.b32[d], s->F.n_f[d])));
    }
    if ((rc = coarsen_all(s.get()))) return rc;
    if ((rc = autotune(s.get()))) return rc;
    if ((rc = capture_graphs(s.get()))) return rc;
    HIPTRY(hipStreamSynchronize(s->st));
    if ((rc = call.finish())) return rc;
  }
  s->setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = s.release();
  return MG_OK;
}

int mg_solve_amr(mg_solver_t* s, mg_multifab_t* phi_c, mg_multifab_t* phi_f,
                 const mg_multifab_t* rhs_c, const mg_multifab_t* rhs_f, double rel_tol,
                 double abs_tol, mg_info_t* info, double* resid_history) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!s || !s->composite) return fail(MG_ERR_ARG, "not a composite solver");
  int rc;
  if ((rc = check_mf(s, phi_c, MG_F64, 1, 1, -1, "phi_c"))) return rc;
  if ((rc = check_mf(s, rhs_c, MG_F64, 0, 1, -1, "rhs_c"))) return rc;
  if ((rc = check_mf_boxes(s->F.boxes, phi_f, 1, 1, -1, "phi_f"))) return rc;
  if ((rc = check_mf_boxes(s->F.boxes, rhs_f, 0, 1, -1, "rhs_f"))) return rc;
  if (!(rel_tol >= 0) || !(abs_tol >= 0)) return fail(MG_ERR_ARG, "negative tolerance");
  CallScope call(s);
  if ((rc = call.rc())) return rc;
  Level& L0 = s->L[0];
  Level& F = s->F;
  double* Pc = (double*)phi_c->data;
  double* Pf = (double*)phi_f->data;
  const double* Fc = (const double*)rhs_c->data;
  const double* Ff = (const double*)rhs_f->data;
  mg_info_t inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.nlevels = (int)s->L.size() + 1;
  inf.tail_level = s->tail_lev > 0 ? s->tail_lev + 1 : 0;
  inf.setup_ms = s->setup_ms;
  HIPTRY(launch_fill_u64(s->st, s->d_norm, 4 * kNormSlot, 0ull));
  HIPTRY(launch_copy_valid(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info, Fc,
                           rhs_c->ngrow, s->Rc, 0));
  if ((rc = avgdown<double>(s, nullptr, 0, s->Rc, 0, 1))) return rc;
  HIPTRY(launch_maxabs<double>(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info, s->Rc,
                               0, s->d_norm));
  HIPTRY(launch_maxabs<double>(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info, Ff,
                               rhs_f->ngrow, s->d_norm));
  double normf;
  if ((rc = read_norm(s, 0, &normf))) return rc;
  int status = MG_OK;
  if (!std::isfinite(normf)) return fail(MG_ERR_NAN, "rhs holds a non-finite value");
  if (normf == 0.0) {
    HIPTRY(launch_zero_valid<double>(s->st, L0.d_cell, (int)L0.t_cell.size(), L0.s_cell, L0.d_info,
                                     Pc, 1));
    HIPTRY(launch_zero_valid<double>(s->st, F.d_cell, (int)F.t_cell.size(), F.s_cell, F.d_info, Pf,
                                     1));
    inf.converged = 1;
    if (resid_history) resid_history[0] = 0.0;
  } else if (s->opts.krylov) {
    status = solve_amr_fgmres(s, Pc, Pf, Fc, rhs_c->ngrow, Ff, rhs_f->ngrow,
                              std::max(rel_tol * normf, abs_tol), &inf, resid_history);
    inf.rel_resid = inf.abs_resid / normf;
  } else {
    const double tol = std::max(rel_tol * normf, abs_tol);
    int it = 0;
    double rn = 0;
    while (true) {
      HIPTRY(launch_fill_u64(s->st, norm_slot(s, 1), kNormSlot, 0ull));
      if ((rc = composite_residual<double>(s, Pc, Pf, Fc, rhs_c->ngrow, Ff, rhs_f->ngrow, s->Rc,
                                           s->Rf, norm_slot(s, 1), nullptr)))
        return rc;
      if ((rc = read_norm(s, 1, &rn))) return rc;
      if (resid_history) resid_history[it] = rn;
      if (s->opts.verbose) fprintf(stderr, "amrmg composite cycle %d  max|R| = %.6e\n", it, rn);
      if (!std::isfinite(rn)) {
        status = fail(MG_ERR_NAN, "residual norm is not finite");
        break;
      }
      if (rn <= tol) {
        inf.converged = 1;
        break;
      }
      if (it == s->opts.max_iter) {
        status = fail(MG_ERR_NOT_CONVERGED, "max_iter reached");
        break;
      }
      if ((rc = composite_correction(s, Pc, Pf))) return rc;
      ++it;
    }
    inf.iters = it;
    inf.abs_resid = rn;
    inf.rel_resid = rn / normf;
  }
  HIPTRY(hipMemcpyAsync(s->h_iters, s->d_iters, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPTRY(hipStreamSynchronize(s->st));
  inf.bottom_iters = *s->h_iters;
  if ((rc = call.finish())) return rc;
  inf.solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

int mg_set_tile_shape(mg_solver_t* s, int32_t kernel, int32_t lx, int32_t ly, int32_t tz,
                      int32_t unroll) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  if (kernel == 3) {
    bool ok = false;
    for (Shape c : sweep_candidates())
      if (c.lx == lx && c.ly == ly && c.tz == tz) ok = true;
    if (!ok) return fail(MG_ERR_ARG, "shape is not a candidate");
    return apply_sweep_shape(s, Shape{lx, ly, tz});
  }
  if (kernel == 5) {
    bool ok = false;
    for (Shape c : quad_candidates())
      if (c.lx == lx && c.ly == ly && c.tz == tz && c.u == unroll) ok = true;
    if (!ok || !quad_ok(s)) return fail(MG_ERR_ARG, "shape is not a candidate");
    return apply_shape(s, Shape{lx, ly, tz, unroll, 2}, true);
  }
  if (kernel == 4) {
    bool ok = false;
    for (Shape c : rr_candidates())
      if (c.lx == lx && c.ly == ly && c.tz == tz) ok = true;
    if (!ok || !s->rr_fold) return fail(MG_ERR_ARG, "shape is not a candidate");
    return apply_rr_shape(s, Shape{lx, ly, tz, 2});
  }
  // kernel 2: the smoother storing whole x-pairs
  const int wp = kernel == 2 ? 1 : 0;
  if (kernel == 2) kernel = 0;
  const Shape sh{lx, ly, tz, unroll, wp};
  bool found = false;
  for (Shape c : kernel == 0 ? gsrb_candidates() : cell_candidates())
    if (c.lx == lx && c.ly == ly && c.tz == tz && c.u == unroll && c.wp == wp) found = true;
  if (!found) return fail(MG_ERR_ARG, "shape is not a candidate");
  return apply_shape(s, sh, kernel == 0);
}

int mg_set_class_tile_shape(mg_solver_t* s, int32_t x_extent, int32_t lx, int32_t ly,
                            int32_t tz) {
  if (!s) return fail(MG_ERR_ARG, "null solver");
  Level& l0 = s->L[0];
  if (l0.fused) return fail(MG_ERR_ARG, "level 0 uses fused sweeps");
  if (l0.cls.empty() && l0.s_gsrb.wp == 2)
    return fail(MG_ERR_ARG, "level 0 uses the quad smoother mapping (no class tables)");
  bool have = false;
  for (const BoxInfo& b : l0.info) have = have || b.hi[0] - b.lo[0] + 1 == x_extent;
  if (!have) return fail(MG_ERR_ARG, "no level-0 box has that x extent");
  const Shape base = l0.cls.empty() ? l0.s_gsrb : l0.cls_base;
  bool ok = false;
  for (Shape c : class_candidates(base.lx * base.ly, base.u, base.wp))
    if (c.lx == lx && c.ly == ly && c.tz == tz) ok = true;
  if (!ok) return fail(MG_ERR_ARG, "shape is not a class candidate of the current launch");
  std::map<int, Shape> cls = l0.cls;
  cls[x_extent] = Shape{lx, ly, tz, base.u, base.wp};
  std::vector<Tile> t;
  make_class_tiles(l0.info, cls, base, {}, t);
  if (t.size() > l0.cap_gsrb) return fail(MG_ERR_ARG, "tile table larger than its reservation");
  return apply_class_tiles(s, cls, base);
}

int mg_get_tile_shape(mg_solver_t* s, int32_t kernel, int32_t* shape) {
  if (!s || !shape) return fail(MG_ERR_ARG, "null argument");
  const Level& l0 = s->L[0];
  if (kernel == 0) {
    const Shape& g = l0.s_gsrb;
    const int32_t v[5] = {g.lx, g.ly, g.tz, g.u, g.wp};
    std::memcpy(shape, v, sizeof(v));
  } else if (kernel == 1) {
    const Shape& c = l0.s_cell;
    const int32_t v[5] = {c.lx, c.ly, c.tz, c.u, 0};
    std::memcpy(shape, v, sizeof(v));
  } else if (kernel == 3) {
    const Shape& w = l0.s_sweep;
    const bool has = !l0.t_sweep.empty();
    const int32_t v[5] = {has ? w.lx : 0, has ? w.ly : 0, has ? w.tz : 0, l0.fused ? 1 : 0, 0};
    std::memcpy(shape, v, sizeof(v));
  } else if (kernel == 4) {
    const Shape& q = l0.s_rr;
    const int32_t v[5] = {q.lx, q.ly, q.tz, s->rr_fold ? 1 : 0, 0};
    std::memcpy(shape, v, sizeof(v));
  } else {
    return fail(MG_ERR_ARG, "kernel must be 0, 1, 3 or 4");
  }
  return MG_OK;
}

int mg_get_class_tile_shapes(mg_solver_t* s, int32_t* out, int32_t cap, int32_t* n) {
  if (!s || !n) return fail(MG_ERR_ARG, "null argument");
  const Level& l0 = s->L[0];
  *n = (int32_t)l0.cls.size();
  if (!out) return MG_OK;
  if (cap < *n) return fail(MG_ERR_ARG, "capacity too small");
  int i = 0;
  for (const auto& kv : l0.cls) {
    out[4 * i] = kv.first;
    out[4 * i + 1] = kv.second.lx;
    out[4 * i + 2] = kv.second.ly;
    out[4 * i + 3] = kv.second.tz;
    ++i;
  }
  return MG_OK;
}

const char* mg_last_error(void) { return amrmg::last_error(); }

}  // extern "C"
