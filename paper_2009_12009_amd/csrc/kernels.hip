// gfx950 kernels of the multigrid solve.
//
// Operator (the cell-centred equation of the paper's "Linear Solvers"
// section, alpha*a*phi - beta*div(b grad phi) = f, 7-point discretisation):
//   (A phi)_i = diag_i phi_i - sum_{faces f not on a wall} c_f phi_nbr(f),
//   c_f = (beta b_f) / h_d^2,  diag_i = alpha a_i + sum_f w_f c_f,
// w_f = 2 on a homogeneous Dirichlet wall (linear ghost phi_g = -phi_i folded
// in), 1 elsewhere.  Faces are visited in the order xlo, xhi, ylo, yhi, zlo,
// zhi everywhere, so the diagonal is the same number in every kernel.
//
// All kernels work on box-list tile tables: one launch covers every box of a
// level; a work-group takes one tile of one box and marches along z, so
// consecutive planes of the same arrays stay in L2 between iterations.  Every
// access is x-contiguous across the lanes of a wavefront.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "kernels.hpp"

namespace amrmg {

namespace {

struct BoxDims {
  int nx, ny, nz;
};

__device__ __forceinline__ BoxDims dims(const BoxInfo& b) {
  return {b.hi[0] - b.lo[0] + 1, b.hi[1] - b.lo[1] + 1, b.hi[2] - b.lo[2] + 1};
}

// Element index of valid cell (il, jl, kl) in a cell array with ng ghosts.
__device__ __forceinline__ long long cidx(const BoxDims& d, int ng, int il, int jl, int kl) {
  const long long sy = d.nx + 2 * ng;
  const long long sz = sy * (d.ny + 2 * ng);
  return (il + ng) + sy * (jl + ng) + sz * (kl + ng);
}

__device__ __forceinline__ unsigned long long absbits(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}
__device__ __forceinline__ unsigned long long absbits(float v) { return absbits((double)v); }

// Fold a per-lane value into the norm slot at dst as an unsigned max over
// the block, into the block's way of the slot (kNormWays words on separate
// cache lines, so the blocks of a launch do not all meet on one line).  The
// block's atomic is skipped when its way already holds at least its value:
// a way only grows, so a value read at any time that is >= m makes the
// atomic a no-op.
__device__ void block_max_u64(unsigned long long v, unsigned long long* dst) {
  dst += kNormStride * (blockIdx.x % kNormWays);
  __shared__ unsigned long long red[16];
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = (unsigned long long)__shfl_xor((long long)v, o);
    v = w > v ? w : v;
  }
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int nw = (blockDim.x * blockDim.y + 63) / 64;
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    unsigned long long m = red[0];
    for (int w = 1; w < nw; ++w) m = red[w] > m ? red[w] : m;
    if (m > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, m);
  }
}

// floor(a / 2) for any sign: the coarse index of fine index a.
__device__ __forceinline__ int fdiv2(int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

// The stencil at one valid cell.  Returns diag and the neighbour sum.
template <typename T>
struct Cell {
  T diag, off;
};

// Values one cell's stencil needs, gathered before any arithmetic so that a
// lane can have the loads of several cells in flight at once.
template <typename T>
struct Nbr {
  T f, a, bxl, bxh, byl, byh, bzl, bzh, pc, pxl, pxh, pyl, pyh, pzl, pzh;
};

// 32-bit strides of one box's arrays (a box's grown array holds < 2^31 cells).
struct Strides {
  int nx, ny, nz, sy, sz, rsy, rsz;
};

__device__ __forceinline__ Strides strides_of(const BoxInfo& B, int rhs_ng) {
  Strides s;
  s.nx = B.hi[0] - B.lo[0] + 1;
  s.ny = B.hi[1] - B.lo[1] + 1;
  s.nz = B.hi[2] - B.lo[2] + 1;
  s.sy = s.nx + 2;
  s.sz = s.sy * (s.ny + 2);
  s.rsy = s.nx + 2 * rhs_ng;
  s.rsz = s.rsy * (s.ny + 2 * rhs_ng);
  return s;
}

template <typename T, bool READ_PHI, bool READ_CENTRE>
__device__ __forceinline__ void gather(Nbr<T>& v, const Strides& s, const T* P, const T* R,
                                       int rhs_ng, const T* BX, const T* BY, const T* BZ,
                                       const T* A, int il, int jl, int kl, int pc) {
  if (R) v.f = R[(il + rhs_ng) + s.rsy * (jl + rhs_ng) + s.rsz * (kl + rhs_ng)];
  const int fx = il + (s.nx + 1) * (jl + s.ny * kl);
  const int fy = il + s.nx * (jl + (s.ny + 1) * kl);
  const int fz = il + s.nx * (jl + s.ny * kl);
  v.bxl = BX[fx];
  v.bxh = BX[fx + 1];
  v.byl = BY[fy];
  v.byh = BY[fy + s.nx];
  v.bzl = BZ[fz];
  v.bzh = BZ[fz + s.nx * s.ny];
  if (A) v.a = A[fz];
  if (READ_CENTRE) v.pc = P[pc];
  if (READ_PHI) {
    v.pxl = P[pc - 1];
    v.pxh = P[pc + 1];
    v.pyl = P[pc - s.sy];
    v.pyh = P[pc + s.sy];
    v.pzl = P[pc - s.sz];
    v.pzh = P[pc + s.sz];
  }
}

// Buffer descriptors of one box's arrays (phi with one ghost layer, rhs,
// face coefficients, cell coefficient): a load through them takes the base
// from SGPRs and a 32-bit byte offset per lane, and loads of the read-once
// arrays carry the non-temporal hint.  Offsets past a descriptor's size
// read 0 (none occur: the indexing is the same as gather's).
struct BoxBufs {
  __amdgpu_buffer_rsrc_t p, r, x, y, z, a;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* base, long long elems,
                                                          int word) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0,
                                           (int)(unsigned)(elems * word), 0x00020000);
}

// aux 2: non-temporal
template <typename T, int AUX>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int idx) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)((unsigned)idx * 8u),
                                                                      0, AUX));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)((unsigned)idx * 4u),
                                                                      0, AUX));
  }
}

// Elements idx and idx + 1 in one load (8 bytes FP32, 16 bytes FP64).  The
// load's vector is cast whole to an integer and split by shifts: taking its
// 32-bit elements one by one lets the compiler shrink the load to its first
// element while still reading the second.
template <typename T, int AUX>
__device__ __forceinline__ void bload_pair(__amdgpu_buffer_rsrc_t r, int idx, T& lo, T& hi) {
  if constexpr (sizeof(T) == 8) {
    const unsigned __int128 u = __builtin_bit_cast(
        unsigned __int128, __builtin_amdgcn_raw_buffer_load_b128(r, (int)((unsigned)idx * 8u), 0, AUX));
    lo = __builtin_bit_cast(T, (unsigned long long)u);
    hi = __builtin_bit_cast(T, (unsigned long long)(u >> 64));
  } else {
    const unsigned long long u = __builtin_bit_cast(
        unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, (int)((unsigned)idx * 4u), 0, AUX));
    lo = __builtin_bit_cast(T, (unsigned)u);
    hi = __builtin_bit_cast(T, (unsigned)(u >> 32));
  }
}

template <typename T>
__device__ __forceinline__ BoxBufs bufs_of(const StencilArgs<T>& op, const BoxInfo& B,
                                           const Strides& s, const T* P, const T* R, int rhs_ng,
                                           const T* BX, const T* BY, const T* BZ, const T* A) {
  BoxBufs b;
  const int w = (int)sizeof(T);
  const long long ncell = (long long)s.nx * s.ny * s.nz;
  b.p = rsrc_of(P, (long long)s.sz * (s.nz + 2), w);
  b.r = rsrc_of(R ? R : P, R ? (long long)s.rsz * (s.nz + 2 * rhs_ng) : 0, w);
  b.x = rsrc_of(BX, ncell + (long long)s.ny * s.nz, w);
  b.y = rsrc_of(BY, ncell + (long long)s.nx * s.nz, w);
  b.z = rsrc_of(BZ, ncell + (long long)s.nx * s.ny, w);
  b.a = rsrc_of(A ? A : P, A ? ncell : 0, w);
  return b;
}

// gather through buffer descriptors (same indices, same values).  HI: aux
// of the high-side y and z face loads, the rows and planes that the next
// tile along y or z reads again as its low side (measured: the half-sweep
// is fastest with them cached, 0; the residual with them non-temporal, 2).
template <typename T, bool READ_PHI, bool READ_CENTRE, int HI>
__device__ __forceinline__ void gather_buf(Nbr<T>& v, const Strides& s, const BoxBufs& b,
                                           int rhs_ng, bool has_r, bool has_a, int il, int jl,
                                           int kl, int pc) {
  if (has_r)
    v.f = bload<T, 2>(b.r, (il + rhs_ng) + s.rsy * (jl + rhs_ng) + s.rsz * (kl + rhs_ng));
  const int fx = il + (s.nx + 1) * (jl + s.ny * kl);
  const int fy = il + s.nx * (jl + (s.ny + 1) * kl);
  const int fz = il + s.nx * (jl + s.ny * kl);
  // the cell's two x faces are adjacent: one load of both (only 4-byte
  // alignment is needed)
  bload_pair<T, 2>(b.x, fx, v.bxl, v.bxh);
  v.byl = bload<T, 2>(b.y, fy);
  v.byh = bload<T, HI>(b.y, fy + s.nx);
  v.bzl = bload<T, 2>(b.z, fz);
  v.bzh = bload<T, HI>(b.z, fz + s.nx * s.ny);
  if (has_a) v.a = bload<T, 2>(b.a, fz);
  if constexpr (READ_PHI && READ_CENTRE) {
    // the low x neighbour and the cell in one load
    bload_pair<T, 0>(b.p, pc - 1, v.pxl, v.pc);
    v.pxh = bload<T, 0>(b.p, pc + 1);
  } else {
    if (READ_CENTRE) v.pc = bload<T, 0>(b.p, pc);
    if (READ_PHI) {
      v.pxl = bload<T, 0>(b.p, pc - 1);
      v.pxh = bload<T, 0>(b.p, pc + 1);
    }
  }
  if (READ_PHI) {
    v.pyl = bload<T, 0>(b.p, pc - s.sy);
    v.pyh = bload<T, 0>(b.p, pc + s.sy);
    v.pzl = bload<T, 0>(b.p, pc - s.sz);
    v.pzh = bload<T, 0>(b.p, pc + s.sz);
  }
}

// diag and neighbour sum from gathered values.  Every kernel that applies
// the operator goes through this one function, so all of them compute the
// same numbers for a cell.
template <typename T, bool READ_PHI>
__device__ __forceinline__ Cell<T> eval(const StencilArgs<T>& op, const Nbr<T>& v, bool has_a,
                                        int m, const Strides& s, int il, int jl, int kl) {
  const T cxl = (op.beta * v.bxl) * op.ih0;
  const T cxh = (op.beta * v.bxh) * op.ih0;
  const T cyl = (op.beta * v.byl) * op.ih1;
  const T cyh = (op.beta * v.byh) * op.ih1;
  const T czl = (op.beta * v.bzl) * op.ih2;
  const T czh = (op.beta * v.bzh) * op.ih2;
  const bool wxl = (m & 1) && il == 0, wxh = (m & 2) && il == s.nx - 1;
  const bool wyl = (m & 4) && jl == 0, wyh = (m & 8) && jl == s.ny - 1;
  const bool wzl = (m & 16) && kl == 0, wzh = (m & 32) && kl == s.nz - 1;
  T diag = has_a ? op.alpha * v.a : op.alpha;
  diag = diag + (wxl ? T(2) * cxl : cxl);
  diag = diag + (wxh ? T(2) * cxh : cxh);
  diag = diag + (wyl ? T(2) * cyl : cyl);
  diag = diag + (wyh ? T(2) * cyh : cyh);
  diag = diag + (wzl ? T(2) * czl : czl);
  diag = diag + (wzh ? T(2) * czh : czh);
  T off = T(0);
  if (READ_PHI) {
    off = wxl ? T(0) : cxl * v.pxl;
    off = off + (wxh ? T(0) : cxh * v.pxh);
    off = off + (wyl ? T(0) : cyl * v.pyl);
    off = off + (wyh ? T(0) : cyh * v.pyh);
    off = off + (wzl ? T(0) : czl * v.pzl);
    off = off + (wzh ? T(0) : czh * v.pzh);
  }
  return {diag, off};
}

// Store a new value of a cell on its box's boundary layer into the face
// ghosts of the boxes that see it (at most one entry per face in a uniform
// box array, a few where faces are shared unevenly).  wb is the box's entry
// range and ex[0..1] its x faces' entries, loaded once per work-group when a
// face has exactly one (every row of a tile has x-face cells, so these must
// not wait on dependent loads inside the loop).
template <typename T>
__device__ __forceinline__ void wt_store(const WtEntry& w, T* phi, int il, int jl, int kl, T v) {
  if (il >= w.lo[0] && il <= w.hi[0] && jl >= w.lo[1] && jl <= w.hi[1] && kl >= w.lo[2] &&
      kl <= w.hi[2])
    phi[w.base + il + (long long)jl * w.sy + (long long)kl * w.sz] = v;
}

// y and z faces only (whole rows and planes of a tile); x faces go through
// the work-group's end-of-tile pass.
template <typename T>
__device__ __forceinline__ void write_through_yz(const WtBox& wb, const WtEntry* __restrict__ wte,
                                                 T* phi, const Strides& s, int il, int jl, int kl,
                                                 T v) {
  const bool on[6] = {false, false, jl == 0, jl == s.ny - 1, kl == 0, kl == s.nz - 1};
  if (!(on[2] | on[3] | on[4] | on[5])) return;
  for (int f = 2; f < 6; ++f) {
    if (!on[f]) continue;
    for (int e = wb.first[f]; e < wb.first[f] + wb.count[f]; ++e)
      wt_store<T>(wte[e], phi, il, jl, kl, v);
  }
}

template <typename T>
__device__ __forceinline__ void write_through(const WtBox& wb, const WtEntry* ex,
                                              const WtEntry* __restrict__ wte, T* phi,
                                              const Strides& s, int il, int jl, int kl, T v) {
  const bool on[6] = {il == 0, il == s.nx - 1, jl == 0, jl == s.ny - 1, kl == 0, kl == s.nz - 1};
  if (!(on[0] | on[1] | on[2] | on[3] | on[4] | on[5])) return;
  for (int f = 0; f < 6; ++f) {
    if (!on[f]) continue;
    if (f < 2 && wb.count[f] == 1) {
      wt_store<T>(ex[f], phi, il, jl, kl, v);
      continue;
    }
    for (int e = wb.first[f]; e < wb.first[f] + wb.count[f]; ++e)
      wt_store<T>(wte[e], phi, il, jl, kl, v);
  }
}

// Red/black half-sweep.  Cells of one colour never read each other, so a lane
// gathers the inputs of U planes first and then updates them: U independent
// load groups in flight per lane instead of one.
// WP: also store the unchanged other cell of the lane's x-pair (its value was
// read as an x-neighbour), so that every cache line is written whole instead
// of one double in two.  No other lane writes that cell in a half-sweep, so
// the result is the same either way.
// WT: each new value is also written into the face ghosts of the boxes that
// see the cell (wtb/wte), so the next half-sweep needs no exchange.  Only
// cells of the active colour are written, into ghosts of that colour, and a
// half-sweep reads only ghosts of the other colour (even periodic extents),
// so no lane reads what another writes.  Rows of y/z-face cells write as
// they go; x-face cells (one or two lanes per row) park their values in LDS
// and the work-group stores them after its z-march, so the march itself
// carries no per-row divergent stores.
// PE: interpolation folded in.  The half-sweep first in line after the
// coarse correction ec (cell data of the next coarser level, boxes cinfo)
// would have been added to every cell: it reads only the other colour, so
// each neighbour value it loads gets its coarse parent's correction added
// (the same single addition), and the other colour is never stored, since
// the next half-sweep overwrites it without reading it (hence never WP,
// whose partner store would race with the lanes adding the correction to
// that cell).  Neighbours on the box's ghost layer take the correction from
// the coarse box's ghost layer, which the caller keeps current.
// BUF: loads through buffer descriptors (gather_buf), for levels whose
// arrays fit 32-bit offsets and are too large to stay in the last-level
// cache between sweeps (the non-temporal hint would cost re-reads there).
template <typename T, int U, bool ZG, bool WP, bool WT, bool PE, bool BUF, bool RS>
__global__ void __launch_bounds__(256)
    k_gsrb(const Tile* __restrict__ tiles, StencilArgs<T> op, T* __restrict__ phi,
           const T* __restrict__ rhs, int rhs_ng, int colour, int tz_launch,
           const WtBox* __restrict__ wtb, const WtEntry* __restrict__ wte,
           const BoxInfo* __restrict__ cinfo, const T* __restrict__ ec,
           const BoxInfo* __restrict__ finfo, const T* __restrict__ rf, T* __restrict__ rout) {
  static_assert(!(PE && (WP || ZG || !WT)), "folded interpolation: write-through half-sweeps only");
  static_assert(!(RS && (!ZG || WP || PE || BUF)), "folded restriction: zero-guess half-sweeps only");
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = op.boxes[t.box];
  // the tile's lane layout (its box class's shape): lx x ly lanes over the
  // work-group's threads (lx a power of two), tz planes
  int lxl, ly, tz;
  if (t.shape) {
    lxl = t.shape & 15;
    ly = (t.shape >> 4) & 255;
    tz = t.shape >> 16;
  } else {
    lxl = __builtin_ctz(blockDim.x);
    ly = blockDim.y;
    tz = tz_launch;
  }
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int tx = tid & ((1 << lxl) - 1), ty = tid >> lxl;
  const int j = t.y0 + ty;
  if (!WT && (ty >= ly || j > B.hi[1])) return;  // with WT every lane reaches the barrier below
  const bool row_ok = ty < ly && j <= B.hi[1];
  const Strides s = strides_of(B, rhs_ng);
  const int jl = j - B.lo[1];
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  T* P = phi + B.off_g1;
  extern __shared__ double lds_gsrb[];
  T* XS = reinterpret_cast<T*>(lds_gsrb);  // [2][ly][tz] x-face values (WT)
  const T* R = rhs + (rhs_ng ? B.off_g1 : B.off_g0);
  const T* BX = op.b0 + B.off_f[0];
  const T* BY = op.b1 + B.off_f[1];
  const T* BZ = op.b2 + B.off_f[2];
  const T* A = op.a ? op.a + B.off_g0 : nullptr;
  const int m = B.bcmask;
  BoxBufs bb;
  if (BUF) bb = bufs_of<T>(op, B, s, P, R, rhs_ng, BX, BY, BZ, A);
  WtBox wb;
  WtEntry ex[2];
  if (WT) {
    wb = wtb[t.box];
    for (int f = 0; f < 2; ++f)
      if (wb.count[f] == 1) ex[f] = wte[wb.first[f]];
  }
  // PE: the coarse parent box (ghost layer 1) and this row's parent index
  const T* EC = nullptr;
  int csy = 0, csz = 0, cbase = 0;
  __amdgpu_buffer_rsrc_t ecr;
  if (PE) {
    const BoxInfo C = cinfo[B.parent];
    csy = C.hi[0] - C.lo[0] + 3;
    csz = csy * (C.hi[1] - C.lo[1] + 3);
    EC = ec + C.off_g1;
    cbase = (1 - C.lo[0]) + csy * (fdiv2(j) - C.lo[1] + 1) + csz * (1 - C.lo[2]);
    // each parent value serves eight fine cells: cached loads
    if (BUF) ecr = rsrc_of(EC, (long long)csz * (C.hi[2] - C.lo[2] + 3), sizeof(T));
  }
  // RS: box b of this level is the coarsening of box b of the finer level
  // (finfo), whose residual rf this half-sweep restricts into rout (ng 0)
  BoxInfo F;
  const T* RF = nullptr;
  T* RO = nullptr;
  long long fsy = 0, fsz = 0;
  if (RS) {
    F = finfo[t.box];
    RF = rf + F.off_g0;
    RO = rout + B.off_g0;
    fsy = F.hi[0] - F.lo[0] + 1;
    fsz = fsy * (F.hi[1] - F.lo[1] + 1);
  }
  for (int k0 = t.z0; k0 <= kend; k0 += U) {
    Nbr<T> v[U];
    T ev[U][PE ? 4 : 1];
    T rv[U][RS ? 2 : 1];
    int il[U], pc[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u;
      const int i = t.x0 + 2 * tx + ((colour + t.x0 + j + k) & 1);
      ok[u] = row_ok && k <= kend && i <= B.hi[0];
      il[u] = i - B.lo[0];
      pc[u] = (il[u] + 1) + s.sy * (jl + 1) + s.sz * (k - B.lo[2] + 1);
      if (RS && row_ok && k <= kend) {
        // the average of the 2x2x2 fine children of both cells of the
        // lane's x-pair (either colour), summed in the restriction's order;
        // a child pair along x is one aligned two-element load (fine boxes
        // have even extents and start at even offsets, so b is even)
        using V2 = T __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int ic = t.x0 + 2 * tx + c;
          if (ic > B.hi[0]) continue;
          const long long b =
              (2 * ic - F.lo[0]) + fsy * (2 * j - F.lo[1]) + fsz * (2 * k - F.lo[2]);
          const V2 q00 = *reinterpret_cast<const V2*>(RF + b);
          const V2 q01 = *reinterpret_cast<const V2*>(RF + b + fsy);
          const V2 q10 = *reinterpret_cast<const V2*>(RF + b + fsz);
          const V2 q11 = *reinterpret_cast<const V2*>(RF + b + fsz + fsy);
          const T z0 = (q00.x + q00.y) + (q01.x + q01.y);
          const T z1 = (q10.x + q10.y) + (q11.x + q11.y);
          rv[u][c] = (z0 + z1) * T(0.125);
          RO[(ic - B.lo[0]) + s.rsy * jl + s.rsz * (k - B.lo[2])] = rv[u][c];
        }
      }
      if (ok[u]) {
        if (BUF)
          gather_buf<T, !ZG, false, 0>(v[u], s, bb, rhs_ng, true, A != nullptr, il[u], jl,
                                       k - B.lo[2], pc[u]);
        else
          gather<T, !ZG, false>(v[u], s, P, RS ? nullptr : R, rhs_ng, BX, BY, BZ, A, il[u], jl,
                                k - B.lo[2], pc[u]);
        if (RS) v[u].f = rv[u][(i - t.x0) & 1];
        if (PE) {
          // the parent of (i, j, k) and, per axis, the parent of the
          // neighbour that lies in the next coarse cell
          const int cc = cbase + fdiv2(i) + csz * fdiv2(k);
          const int c1 = cc + ((i & 1) ? 1 : -1);
          const int c2 = cc + ((j & 1) ? csy : -csy);
          const int c3 = cc + ((k & 1) ? csz : -csz);
          if (BUF) {
            ev[u][0] = bload<T, 0>(ecr, cc);
            ev[u][1] = bload<T, 0>(ecr, c1);
            ev[u][2] = bload<T, 0>(ecr, c2);
            ev[u][3] = bload<T, 0>(ecr, c3);
          } else {
            ev[u][0] = EC[cc];
            ev[u][1] = EC[c1];
            ev[u][2] = EC[c2];
            ev[u][3] = EC[c3];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      if (PE) {
        const bool ox = (il[u] + B.lo[0]) & 1, oy = j & 1, oz = (k0 + u) & 1;
        v[u].pxl = v[u].pxl + (ox ? ev[u][0] : ev[u][1]);
        v[u].pxh = v[u].pxh + (ox ? ev[u][1] : ev[u][0]);
        v[u].pyl = v[u].pyl + (oy ? ev[u][0] : ev[u][2]);
        v[u].pyh = v[u].pyh + (oy ? ev[u][2] : ev[u][0]);
        v[u].pzl = v[u].pzl + (oz ? ev[u][0] : ev[u][3]);
        v[u].pzh = v[u].pzh + (oz ? ev[u][3] : ev[u][0]);
      }
      const Cell<T> c = eval<T, !ZG>(op, v[u], A != nullptr, m, s, il[u], jl, k0 + u - B.lo[2]);
      const T nv = ZG ? v[u].f / c.diag : (v[u].f + c.off) / c.diag;
      P[pc[u]] = nv;
      if (WT) {
        const int kk = k0 + u - t.z0;
        if (il[u] == 0) XS[(0 * ly + ty) * tz + kk] = nv;
        if (il[u] == s.nx - 1) XS[(1 * ly + ty) * tz + kk] = nv;
        write_through_yz<T>(wb, wte, phi, s, il[u], jl, k0 + u - B.lo[2], nv);
      }
      if (WP && !ZG) {
        // partner = the pair's other cell: x+1 when the active cell is the pair's first
        const bool first = ((il[u] + B.lo[0] - t.x0) & 1) == 0;
        const int pil = first ? il[u] + 1 : il[u] - 1;
        if (pil >= 0 && pil < s.nx) P[first ? pc[u] + 1 : pc[u] - 1] = first ? v[u].pxh : v[u].pxl;
      }
    }
  }
  if (WT) {
    // x faces of this tile: cells of the active colour in column 0 (tile
    // starts at the box's low x) and column nx-1 (tile reaches its high x)
    const bool has_lo = t.x0 == B.lo[0] && wb.count[0] > 0;
    const bool has_hi = B.hi[0] <= t.x0 + 2 * (1 << lxl) - 1 && wb.count[1] > 0;
    if (has_lo || has_hi) {
      __syncthreads();
      const int nz_t = kend - t.z0 + 1;
      const int n = ly * nz_t;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        if (!(f ? has_hi : has_lo)) continue;
        const int ilf = f ? s.nx - 1 : 0;
        for (int q = tid; q < n; q += blockDim.x * blockDim.y) {
          const int ty = q / nz_t, kk = q - ty * nz_t;
          const int jj = t.y0 + ty, k = t.z0 + kk;
          if (jj > B.hi[1] || ((B.lo[0] + ilf + jj + k) & 1) != colour) continue;
          const T xv = XS[(f * ly + ty) * tz + kk];
          const int jlf = jj - B.lo[1], klf = k - B.lo[2];
          if (wb.count[f] == 1) {
            wt_store<T>(ex[f], phi, ilf, jlf, klf, xv);
          } else {
            for (int e = wb.first[f]; e < wb.first[f] + wb.count[f]; ++e)
              wt_store<T>(wte[e], phi, ilf, jlf, klf, xv);
          }
        }
      }
    }
  }
}

// FP32 half-sweep with two cells of the active colour per lane: lane tx of
// a tile row covers the x-quad t.x0 + 4 tx .. + 3 and updates its cells i0
// and i0 + 2 of that colour, each with the pair kernel's arithmetic (eval,
// the same update).  The quad's values come in 16-byte buffer loads (dword
// alignment; loads past a row read other cells and are not used, past the
// array they read 0), so a lane issues about half the loads per cell of the
// pair mapping.  Streaming levels (buffer descriptors) with write-through
// only, every box's x extent a multiple of 4 (no quad reaches past the end of
// an array); ZG and PE as in k_gsrb.
// A quad stays a 128-bit integer value; an element is a constant shift of
// it.  (Kept as an array or a struct, a choice between two elements by the
// lane's colour parity became an indexed access to a copy in scratch.)
typedef unsigned __int128 Quad;

__device__ __forceinline__ Quad qload(__amdgpu_buffer_rsrc_t r, int idx, int aux_nt) {
  // the vector is cast whole (element-wise extraction let the compiler
  // shrink wide buffer loads)
  return aux_nt ? __builtin_bit_cast(Quad, __builtin_amdgcn_raw_buffer_load_b128(
                                               r, (int)((unsigned)idx * 4u), 0, 2))
                : __builtin_bit_cast(Quad, __builtin_amdgcn_raw_buffer_load_b128(
                                               r, (int)((unsigned)idx * 4u), 0, 0));
}

template <int E>
__device__ __forceinline__ float qel(Quad q) {
  return __builtin_bit_cast(float, (unsigned)(q >> (32 * E)));
}

// element 2c + p (p = 0 or 1): the select is on values, not on addresses
__device__ __forceinline__ float qpick(Quad q, int c, int p) {
  const unsigned lo = (unsigned)(q >> (c ? 64 : 0)), hi = (unsigned)(q >> (c ? 96 : 32));
  return __builtin_bit_cast(float, p ? hi : lo);
}

template <int U, bool ZG, bool PE>
__global__ void __launch_bounds__(256)
    k_gsrb_quad(const Tile* __restrict__ tiles, StencilArgs<float> op, float* __restrict__ phi,
                const float* __restrict__ rhs, int rhs_ng, int colour, int tz_launch,
                const WtBox* __restrict__ wtb, const WtEntry* __restrict__ wte,
                const BoxInfo* __restrict__ cinfo, const float* __restrict__ ec) {
  static_assert(!(PE && ZG), "folded interpolation: not from zero");
  using T = float;
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = op.boxes[t.box];
  const int lxl = __builtin_ctz(blockDim.x);
  const int ly = blockDim.y;
  const int tz = tz_launch;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int j = t.y0 + ty;
  const bool row_ok = j <= B.hi[1];
  const Strides s = strides_of(B, rhs_ng);
  const int jl = j - B.lo[1];
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  T* P = phi + B.off_g1;
  extern __shared__ double lds_gsrb[];
  T* XS = reinterpret_cast<T*>(lds_gsrb);  // [2][ly][tz] x-face values
  const T* R = rhs + (rhs_ng ? B.off_g1 : B.off_g0);
  const T* BX = op.b0 + B.off_f[0];
  const T* BY = op.b1 + B.off_f[1];
  const T* BZ = op.b2 + B.off_f[2];
  const T* A = op.a ? op.a + B.off_g0 : nullptr;
  const int m = B.bcmask;
  const BoxBufs bb = bufs_of<T>(op, B, s, P, R, rhs_ng, BX, BY, BZ, A);
  WtBox wb = wtb[t.box];
  WtEntry ex[2];
  for (int f = 0; f < 2; ++f)
    if (wb.count[f] == 1) ex[f] = wte[wb.first[f]];
  const T* EC = nullptr;
  int csy = 0, csz = 0, cbase = 0;
  __amdgpu_buffer_rsrc_t ecr;
  if (PE) {
    const BoxInfo C = cinfo[B.parent];
    csy = C.hi[0] - C.lo[0] + 3;
    csz = csy * (C.hi[1] - C.lo[1] + 3);
    EC = ec + C.off_g1;
    cbase = (1 - C.lo[0]) + csy * (fdiv2(j) - C.lo[1] + 1) + csz * (1 - C.lo[2]);
    ecr = rsrc_of(EC, (long long)csz * (C.hi[2] - C.lo[2] + 3), sizeof(T));
  }
  const int xq = t.x0 + 4 * tx;
  const int ilq = xq - B.lo[0];
  for (int k0 = t.z0; k0 <= kend; k0 += U) {
    Nbr<T> v[U][2];
    T ev[U][2][PE ? 4 : 1];
    int pc[U], par[U];
    bool ok[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u;
      const int p = (colour + t.x0 + j + k) & 1;
      par[u] = p;
      ok[u][0] = row_ok && k <= kend && ilq + p <= s.nx - 1;
      ok[u][1] = row_ok && k <= kend && ilq + p + 2 <= s.nx - 1;
      const int kl = k - B.lo[2];
      pc[u] = (ilq + 1) + s.sy * (jl + 1) + s.sz * (kl + 1);
      if (!ok[u][0]) continue;
      const int fxq = ilq + (s.nx + 1) * (jl + s.ny * kl);
      const int fyq = ilq + s.nx * (jl + (s.ny + 1) * kl);
      const int fzq = ilq + s.nx * (jl + s.ny * kl);
      const Quad qf = qload(bb.r, (ilq + rhs_ng) + s.rsy * (jl + rhs_ng) + s.rsz * (kl + rhs_ng), 1);
      const Quad qx = qload(bb.x, fxq + p, 1);
      const Quad qyl = qload(bb.y, fyq, 1);
      const Quad qyh = qload(bb.y, fyq + s.nx, 0);
      const Quad qzl = qload(bb.z, fzq, 1);
      const Quad qzh = qload(bb.z, fzq + s.nx * s.ny, 0);
      Quad qa = 0;
      if (A) qa = qload(bb.a, fzq, 1);
      // element p + 2c of a quad, picked with constant indices (an index
      // that depends on the lane's parity would put the quad in scratch)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        v[u][c].f = qpick(qf, c, p);
        v[u][c].bxl = c ? qel<2>(qx) : qel<0>(qx);
        v[u][c].bxh = c ? qel<3>(qx) : qel<1>(qx);
        v[u][c].byl = qpick(qyl, c, p);
        v[u][c].byh = qpick(qyh, c, p);
        v[u][c].bzl = qpick(qzl, c, p);
        v[u][c].bzh = qpick(qzh, c, p);
        if (A) v[u][c].a = qpick(qa, c, p);
      }
      if (!ZG) {
        // x neighbours: pc-1 .. pc+2 and pc+3 .. pc+6 of the quad's row
        const Quad qp0 = qload(bb.p, pc[u] - 1, 0);
        const Quad qp1 = qload(bb.p, pc[u] + 3, 0);
        const Quad qyl_ = qload(bb.p, pc[u] - s.sy, 0);
        const Quad qyh_ = qload(bb.p, pc[u] + s.sy, 0);
        const Quad qzl_ = qload(bb.p, pc[u] - s.sz, 0);
        const Quad qzh_ = qload(bb.p, pc[u] + s.sz, 0);
        // the row from the quad's low neighbour on: x0..x5 = qp0's four
        // values and qp1's first two; quad cell e has x_e below, x_(e+2) above
        const T x0 = qel<0>(qp0), x1 = qel<1>(qp0), x2 = qel<2>(qp0), x3 = qel<3>(qp0);
        const T x4 = qel<0>(qp1), x5 = qel<1>(qp1);
        v[u][0].pxl = p ? x1 : x0;
        v[u][0].pxh = p ? x3 : x2;
        v[u][1].pxl = p ? x3 : x2;
        v[u][1].pxh = p ? x5 : x4;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          v[u][c].pyl = qpick(qyl_, c, p);
          v[u][c].pyh = qpick(qyh_, c, p);
          v[u][c].pzl = qpick(qzl_, c, p);
          v[u][c].pzh = qpick(qzh_, c, p);
        }
      }
      if (PE) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (!ok[u][c]) continue;
          const int i = xq + p + 2 * c;
          const int cc = cbase + fdiv2(i) + csz * fdiv2(k);
          ev[u][c][0] = bload<T, 0>(ecr, cc);
          ev[u][c][1] = bload<T, 0>(ecr, cc + ((i & 1) ? 1 : -1));
          ev[u][c][2] = bload<T, 0>(ecr, cc + ((j & 1) ? csy : -csy));
          ev[u][c][3] = bload<T, 0>(ecr, cc + ((k & 1) ? csz : -csz));
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (!ok[u][c]) continue;
        const int il = ilq + par[u] + 2 * c;
        const int kl = k0 + u - B.lo[2];
        Nbr<T>& w = v[u][c];
        if (PE) {
          const bool ox = (il + B.lo[0]) & 1, oy = j & 1, oz = (k0 + u) & 1;
          w.pxl = w.pxl + (ox ? ev[u][c][0] : ev[u][c][1]);
          w.pxh = w.pxh + (ox ? ev[u][c][1] : ev[u][c][0]);
          w.pyl = w.pyl + (oy ? ev[u][c][0] : ev[u][c][2]);
          w.pyh = w.pyh + (oy ? ev[u][c][2] : ev[u][c][0]);
          w.pzl = w.pzl + (oz ? ev[u][c][0] : ev[u][c][3]);
          w.pzh = w.pzh + (oz ? ev[u][c][3] : ev[u][c][0]);
        }
        const Cell<T> cl = eval<T, !ZG>(op, w, A != nullptr, m, s, il, jl, kl);
        const T nv = ZG ? w.f / cl.diag : (w.f + cl.off) / cl.diag;
        P[pc[u] + par[u] + 2 * c] = nv;
        const int kk = k0 + u - t.z0;
        if (il == 0) XS[(0 * ly + ty) * tz + kk] = nv;
        if (il == s.nx - 1) XS[(1 * ly + ty) * tz + kk] = nv;
        write_through_yz<T>(wb, wte, phi, s, il, jl, kl, nv);
      }
    }
  }
  // x faces of this tile, as in k_gsrb
  const bool has_lo = t.x0 == B.lo[0] && wb.count[0] > 0;
  const bool has_hi = B.hi[0] <= t.x0 + 4 * (1 << lxl) - 1 && wb.count[1] > 0;
  if (has_lo || has_hi) {
    __syncthreads();
    const int nz_t = kend - t.z0 + 1;
    const int n = ly * nz_t;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      if (!(f ? has_hi : has_lo)) continue;
      const int ilf = f ? s.nx - 1 : 0;
      for (int q = tx + blockDim.x * ty; q < n; q += blockDim.x * blockDim.y) {
        const int tyq = q / nz_t, kk = q - tyq * nz_t;
        const int jj = t.y0 + tyq, k = t.z0 + kk;
        if (jj > B.hi[1] || ((B.lo[0] + ilf + jj + k) & 1) != colour) continue;
        const T xv = XS[(f * ly + tyq) * tz + kk];
        const int jlf = jj - B.lo[1], klf = k - B.lo[2];
        if (wb.count[f] == 1) {
          wt_store<T>(ex[f], phi, ilf, jlf, klf, xv);
        } else {
          for (int e = wb.first[f]; e < wb.first[f] + wb.count[f]; ++e)
            wt_store<T>(wte[e], phi, ilf, jlf, klf, xv);
        }
      }
    }
  }
}

// One full red/black sweep, out of place (see launch_sweep).  Box-local
// coordinates throughout; colour of local cell (i, j, k) = (i+j+k+par) & 1,
// red = 0.  LDS holds a ring of 5 old planes over the tile grown by 2 in x
// and y (old values of both colours, ghosts included) and a ring of 3 planes
// of new red values over the tile grown by 1.  Step k computes red on plane
// k over the grown tile (needs old planes k-1..k+1), then black on plane
// k-1 over the tile (needs new red on planes k-2..k) and writes plane k-1.
// Every global load of a step (old plane k+1, red and black coefficients) is
// issued before its first barrier, so a step waits for memory once.
// Ring sizes make two barriers per step enough: the old slot loaded at step
// k+1 last held plane k-4, read at step k-1 at the latest, and the red slot
// written at step k+1 last held plane k-2, read at step k before the
// barrier that opens step k+1's red phase.
template <typename T, int LX, int LY, bool ZG, bool NORM>
__global__ void __launch_bounds__(LX / 2 * LY)
    k_sweep(const Tile* __restrict__ tiles, StencilArgs<T> op, const T* __restrict__ pin,
            T* __restrict__ pout, const T* __restrict__ rhs, int rhs_ng, int tz,
            unsigned long long* normbits) {
  constexpr int NT = LX / 2 * LY;
  constexpr int W2 = LX + 4, P2 = W2 * (LY + 4);
  constexpr int W1 = LX + 2, P1 = W1 * (LY + 2);
  constexpr int HP = W1 / 2, NRP = HP * (LY + 2);  // red pair slots of the grown tile
  constexpr int R1 = (P2 + NT - 1) / NT, R2 = (NRP + NT - 1) / NT;
  extern __shared__ double lds_sweep[];
  T* OLD = reinterpret_cast<T*>(lds_sweep);
  T* RED = OLD + 5 * P2;
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = op.boxes[t.box];
  const Strides s = strides_of(B, rhs_ng);
  const int tid = threadIdx.x;
  const int x0 = t.x0 - B.lo[0], y0 = t.y0 - B.lo[1], z0 = t.z0 - B.lo[2];
  const int x1 = min(x0 + LX, s.nx) - 1, y1 = min(y0 + LY, s.ny) - 1, z1 = min(z0 + tz, s.nz) - 1;
  const int par = (B.lo[0] + B.lo[1] + B.lo[2]) & 1;
  const T* Pin = pin + B.off_g1;
  T* Pout = pout + B.off_g1;
  const T* R = rhs + (rhs_ng ? B.off_g1 : B.off_g0);
  const T* BX = op.b0 + B.off_f[0];
  const T* BY = op.b1 + B.off_f[1];
  const T* BZ = op.b2 + B.off_f[2];
  const T* A = op.a ? op.a + B.off_g0 : nullptr;
  const int m = B.bcmask;
  unsigned long long mx = 0;

  // this lane's old-plane positions (fixed for the whole z-march)
  int o_off[R1];  // element offset in the grown box array without the plane term, -1 = skip
#pragma unroll
  for (int r = 0; r < R1; ++r) {
    const int q = tid + r * NT;
    const int il = x0 - 2 + q % W2, jl = y0 - 2 + q / W2;
    o_off[r] = (q < P2 && il >= -1 && il <= s.nx && jl >= -1 && jl <= s.ny)
                   ? (il + 1) + s.sy * (jl + 1)
                   : -1;
  }
  // this lane's red pair slots and black pair
  int r_jl[R2], r_i0[R2];
#pragma unroll
  for (int r = 0; r < R2; ++r) {
    const int q = tid + r * NT;
    r_jl[r] = q < NRP ? y0 - 1 + q / HP : -2;
    r_i0[r] = x0 - 1 + 2 * (q % HP);
  }
  const int b_jl = y0 + tid / (LX / 2), b_i0 = x0 + 2 * (tid % (LX / 2));
  const bool b_ok = b_jl <= y1 && b_i0 <= x1;

  auto oslot = [](int k) { return ((k % 5) + 5) % 5; };
  auto rslot = [](int k) { return ((k % 3) + 3) % 3; };
  auto old_at = [&](int il, int jl, int k) -> T {
    return OLD[oslot(k) * P2 + (jl - y0 + 2) * W2 + (il - x0 + 2)];
  };
  auto red_at = [&](int il, int jl, int k) -> T {
    return RED[rslot(k) * P1 + (jl - y0 + 1) * W1 + (il - x0 + 1)];
  };
  auto load_now = [&](int k) {  // direct load of old plane k (prologue only)
    T* dst = OLD + oslot(k) * P2;
#pragma unroll
    for (int r = 0; r < R1; ++r)
      if (o_off[r] >= 0) dst[tid + r * NT] = ZG ? T(0) : Pin[o_off[r] + s.sz * (k + 1)];
  };

  const int kb = z0 - 1, ke = z1 + 1;
  for (int k = kb - 1; k <= kb; ++k)
    if (k >= -1 && k <= s.nz) load_now(k);
  for (int k = kb; k <= ke; ++k) {
    // ---- issue this step's global loads
    T ov[R1];
    const bool load_next = k + 1 <= s.nz;
#pragma unroll
    for (int r = 0; r < R1; ++r)
      if (!ZG && load_next && o_off[r] >= 0) ov[r] = Pin[o_off[r] + s.sz * (k + 2)];
    Nbr<T> vr[R2];
    int r_il[R2];
    bool r_ok[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int jl = r_jl[r];
      const int il = r_i0[r] + ((r_i0[r] + jl + k + par) & 1);
      r_il[r] = il;
      r_ok[r] = k >= 0 && k < s.nz && il >= 0 && il < s.nx && jl >= 0 && jl < s.ny;
      if (r_ok[r]) gather<T, false, false>(vr[r], s, nullptr, R, rhs_ng, BX, BY, BZ, A, il, jl, k, 0);
    }
    const int kk = k - 1;
    const bool first_black = ((b_i0 + b_jl + kk + par) & 1) == 1;
    const int ib = first_black ? b_i0 : b_i0 + 1;
    const int ir = first_black ? b_i0 + 1 : b_i0;
    const bool bk = b_ok && kk >= z0 && kk <= z1;
    const bool bb = bk && ib <= x1;
    const bool rim = ib == 0 || ib == s.nx - 1 || b_jl == 0 || b_jl == s.ny - 1 || kk == 0 ||
                     kk == s.nz - 1;
    Nbr<T> vb;
    if (bb && (!rim || NORM))
      gather<T, false, false>(vb, s, nullptr, R, rhs_ng, BX, BY, BZ, A, ib, b_jl, kk, 0);
    // ---- old plane k+1 into LDS
    if (load_next) {
      T* dst = OLD + oslot(k + 1) * P2;
#pragma unroll
      for (int r = 0; r < R1; ++r)
        if (o_off[r] >= 0) dst[tid + r * NT] = ZG ? T(0) : ov[r];
    }
    __syncthreads();
    // ---- red on plane k over the tile grown by 1
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      if (!r_ok[r]) continue;
      const int il = r_il[r], jl = r_jl[r];
      Nbr<T>& v = vr[r];
      v.pxl = old_at(il - 1, jl, k);
      v.pxh = old_at(il + 1, jl, k);
      v.pyl = old_at(il, jl - 1, k);
      v.pyh = old_at(il, jl + 1, k);
      v.pzl = old_at(il, jl, k - 1);
      v.pzh = old_at(il, jl, k + 1);
      const Cell<T> c = eval<T, true>(op, v, A != nullptr, m, s, il, jl, k);
      RED[rslot(k) * P1 + (jl - y0 + 1) * W1 + (il - x0 + 1)] = (v.f + c.off) / c.diag;
      if (NORM && il >= x0 && il <= x1 && jl >= y0 && jl <= y1 && k >= z0 && k <= z1) {
        const T res = v.f - (c.diag * old_at(il, jl, k) - c.off);
        const unsigned long long bits = absbits(res);
        mx = bits > mx ? bits : mx;
      }
    }
    __syncthreads();
    // ---- black on plane k-1 over the tile; write both cells of the pair
    if (bk) {
      const int jl = b_jl;
      const int base = s.sy * (jl + 1) + s.sz * (kk + 1) + 1;
      if (ir <= x1) Pout[base + ir] = red_at(ir, jl, kk);
      if (bb) {
        T out = old_at(ib, jl, kk);
        if (!rim) {
          vb.pxl = red_at(ib - 1, jl, kk);
          vb.pxh = red_at(ib + 1, jl, kk);
          vb.pyl = red_at(ib, jl - 1, kk);
          vb.pyh = red_at(ib, jl + 1, kk);
          vb.pzl = red_at(ib, jl, kk - 1);
          vb.pzh = red_at(ib, jl, kk + 1);
          const Cell<T> c = eval<T, true>(op, vb, A != nullptr, m, s, ib, jl, kk);
          out = (vb.f + c.off) / c.diag;
        }
        if (NORM) {
          vb.pxl = old_at(ib - 1, jl, kk);
          vb.pxh = old_at(ib + 1, jl, kk);
          vb.pyl = old_at(ib, jl - 1, kk);
          vb.pyh = old_at(ib, jl + 1, kk);
          vb.pzl = old_at(ib, jl, kk - 1);
          vb.pzh = old_at(ib, jl, kk + 1);
          const Cell<T> c = eval<T, true>(op, vb, A != nullptr, m, s, ib, jl, kk);
          const T res = vb.f - (c.diag * old_at(ib, jl, kk) - c.off);
          const unsigned long long bits = absbits(res);
          mx = bits > mx ? bits : mx;
        }
        Pout[base + ib] = out;
      }
    }
  }
  if (NORM) block_max_u64(mx, normbits);
}

// Black update of the rim cells left by k_sweep (phi holds new red values,
// ghosts included).  One lane per cell of a rim tile; red lanes idle.
template <typename T>
__global__ void __launch_bounds__(256)
    k_rim(const RimTile* __restrict__ tiles, StencilArgs<T> op, T* __restrict__ phi,
          const T* __restrict__ rhs, int rhs_ng) {
  const RimTile t = tiles[blockIdx.x];
  const int q = threadIdx.x;
  if (q >= t.ni * t.nj * t.nk) return;
  const BoxInfo B = op.boxes[t.box];
  const int il = t.i0 + q % t.ni;
  const int jl = t.j0 + (q / t.ni) % t.nj;
  const int kl = t.k0 + q / (t.ni * t.nj);
  if (((il + jl + kl + B.lo[0] + B.lo[1] + B.lo[2]) & 1) != 1) return;
  const Strides s = strides_of(B, rhs_ng);
  T* P = phi + B.off_g1;
  const T* R = rhs + (rhs_ng ? B.off_g1 : B.off_g0);
  const T* A = op.a ? op.a + B.off_g0 : nullptr;
  const int pc = (il + 1) + s.sy * (jl + 1) + s.sz * (kl + 1);
  Nbr<T> v;
  gather<T, true, false>(v, s, P, R, rhs_ng, op.b0 + B.off_f[0], op.b1 + B.off_f[1],
                         op.b2 + B.off_f[2], A, il, jl, kl, pc);
  const Cell<T> c = eval<T, true>(op, v, A != nullptr, B.bcmask, s, il, jl, kl);
  P[pc] = (v.f + c.off) / c.diag;
}

__device__ double block_sum(double v, double* red, int& phase);

// out = rhs - A phi (mode 0) or A phi (mode 1), one lane per cell, U planes
// gathered at a time; optional NaN-propagating max |out|.
// NX (mode 0): also write phi after a red half-sweep into pnext (same ghost
// layout as phi, valid cells only): a red cell gets (f + off) / diag from
// the same gathered values, the same expression as the half-sweep, and a
// black cell its old value.  The residual is that of phi, before the update.
// With wtb/wte (non-null) each new red value on the box's boundary layer is
// also stored into the face ghosts of pnext that mirror it, as the
// half-sweep's write-through does: the next half-sweep (black) reads only
// red values, so pnext then needs no exchange.
template <typename T, typename TO, int U, bool BUF, bool NX>
__global__ void __launch_bounds__(256)
    k_residual(const Tile* __restrict__ tiles, StencilArgs<T> op, const T* __restrict__ phi,
               const T* __restrict__ rhs, int rhs_ng, TO* __restrict__ out,
               unsigned long long* normbits, int tz, int mode, double* __restrict__ dot_partials,
               T* __restrict__ pnext, const WtBox* __restrict__ wtb,
               const WtEntry* __restrict__ wte) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = op.boxes[t.box];
  const int i = t.x0 + threadIdx.x;
  const int j = t.y0 + threadIdx.y;
  const bool act = i <= B.hi[0] && j <= B.hi[1];
  unsigned long long mx = 0;
  double dot = 0.0;
  WtBox wb;
  WtEntry ex[2];
  if (NX && wtb) {
    wb = wtb[t.box];
    for (int f = 0; f < 2; ++f)
      if (wb.count[f] == 1) ex[f] = wte[wb.first[f]];
  }
  if (act) {
    const Strides s = strides_of(B, rhs_ng);
    const int kend = min(t.z0 + tz - 1, B.hi[2]);
    const T* P = phi + B.off_g1;
    const T* R = mode == 0 ? rhs + (rhs_ng ? B.off_g1 : B.off_g0) : nullptr;
    const T* BX = op.b0 + B.off_f[0];
    const T* BY = op.b1 + B.off_f[1];
    const T* BZ = op.b2 + B.off_f[2];
    const T* A = op.a ? op.a + B.off_g0 : nullptr;
    TO* O = out ? out + B.off_g0 : nullptr;
    const int il = i - B.lo[0], jl = j - B.lo[1];
    const int m = B.bcmask;
    BoxBufs bb;
    if (BUF) bb = bufs_of<T>(op, B, s, P, R, rhs_ng, BX, BY, BZ, A);
    for (int k0 = t.z0; k0 <= kend; k0 += U) {
      Nbr<T> v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int kl = k0 + u - B.lo[2];
        const int pc = (il + 1) + s.sy * (jl + 1) + s.sz * (kl + 1);
        if (k0 + u > kend) continue;
        if (BUF)
          gather_buf<T, true, true, 2>(v[u], s, bb, rhs_ng, R != nullptr, A != nullptr, il, jl,
                                       kl, pc);
        else
          gather<T, true, true>(v[u], s, P, R, rhs_ng, BX, BY, BZ, A, il, jl, kl, pc);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u > kend) continue;
        const int kl = k0 + u - B.lo[2];
        const Cell<T> c = eval<T, true>(op, v[u], A != nullptr, m, s, il, jl, kl);
        const T Aphi = c.diag * v[u].pc - c.off;
        const T r = mode == 0 ? v[u].f - Aphi : Aphi;
        if (O) O[il + s.nx * (jl + s.ny * kl)] = (TO)r;
        if (NX) {
          const bool red = ((i + j + k0 + u) & 1) == 0;
          const T nv = red ? (v[u].f + c.off) / c.diag : v[u].pc;
          pnext[B.off_g1 + (il + 1) + s.sy * (jl + 1) + s.sz * (kl + 1)] = nv;
          if (wtb && red) write_through<T>(wb, ex, wte, pnext, s, il, jl, kl, nv);
        }
        const unsigned long long bits = absbits(r);
        mx = bits > mx ? bits : mx;
        if (dot_partials) dot += (double)v[u].pc * (double)r;
      }
    }
  }
  if (normbits) block_max_u64(mx, normbits);
  if (dot_partials) {
    __shared__ double red[32];
    int phase = 0;
    dot = block_sum(dot, red, phase);
    if (threadIdx.x == 0 && threadIdx.y == 0) dot_partials[blockIdx.x] = dot;
  }
}

// rc = R (rhs - A phi): the residual of each cell, computed as k_residual
// computes it (mode 0), summed over 2x2x2 blocks in k_restrict's order and
// scaled, so the coarse right-hand side gets the bits that a residual pass
// and a restriction pass store, without the fine residual reaching memory.
// Tiles (lx x ly lanes, tz planes) start at even cells with lx, ly, tz
// even, box extents even: a lane gathers its cell on two planes, x-pairs
// are adjacent lanes, y-pairs go through LDS.  cinfo: the coarse level's
// boxes (box b's parent); rc without ghosts.
template <typename T, bool BUF>
__global__ void __launch_bounds__(256)
    k_resid_restrict(const Tile* __restrict__ tiles, StencilArgs<T> op, const T* __restrict__ phi,
                     const T* __restrict__ rhs, int rhs_ng, int tz,
                     const BoxInfo* __restrict__ cinfo, T* __restrict__ rc) {
  __shared__ T ypair[2][128];
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = op.boxes[t.box];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = t.x0 + tx, j = t.y0 + ty;
  // x-pairs and y-pairs lie wholly inside or outside the box (even extents)
  const bool act = i <= B.hi[0] && j <= B.hi[1];
  const Strides s = strides_of(B, rhs_ng);
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  const T* P = phi + B.off_g1;
  const T* R = rhs + (rhs_ng ? B.off_g1 : B.off_g0);
  const T* BX = op.b0 + B.off_f[0];
  const T* BY = op.b1 + B.off_f[1];
  const T* BZ = op.b2 + B.off_f[2];
  const T* A = op.a ? op.a + B.off_g0 : nullptr;
  const int il = i - B.lo[0], jl = j - B.lo[1];
  BoxBufs bb;
  if (BUF) bb = bufs_of<T>(op, B, s, P, R, rhs_ng, BX, BY, BZ, A);
  const BoxInfo C = cinfo[B.parent];
  const BoxDims dc = dims(C);
  const int slot = (ty >> 1) * (blockDim.x >> 1) + (tx >> 1);
  for (int k0 = t.z0; k0 <= kend; k0 += 2) {
    T r[2] = {T(0), T(0)};
    if (act) {
      Nbr<T> v[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int kl = k0 + u - B.lo[2];
        const int pc = (il + 1) + s.sy * (jl + 1) + s.sz * (kl + 1);
        if (BUF)
          gather_buf<T, true, true, 2>(v[u], s, bb, rhs_ng, true, A != nullptr, il, jl, kl, pc);
        else
          gather<T, true, true>(v[u], s, P, R, rhs_ng, BX, BY, BZ, A, il, jl, kl, pc);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int kl = k0 + u - B.lo[2];
        const Cell<T> c = eval<T, true>(op, v[u], A != nullptr, B.bcmask, s, il, jl, kl);
        const T Aphi = c.diag * v[u].pc - c.off;
        r[u] = v[u].f - Aphi;
      }
    }
    // x-pair sums (both lanes of a pair get the same bits)
    T sx[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) sx[u] = r[u] + __shfl_xor(r[u], 1);
    if ((tx & 1) == 0 && (ty & 1) == 1) {
      ypair[0][slot] = sx[0];
      ypair[1][slot] = sx[1];
    }
    __syncthreads();
    if ((tx & 1) == 0 && (ty & 1) == 0 && act) {
      const T z0 = sx[0] + ypair[0][slot];
      const T z1 = sx[1] + ypair[1][slot];
      const int I = fdiv2(i), J = fdiv2(j), K = fdiv2(k0);
      rc[C.off_g0 + cidx(dc, 0, I - C.lo[0], J - C.lo[1], K - C.lo[2])] = (z0 + z1) * T(0.125);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_maxabs(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
             const T* __restrict__ v, int ng, unsigned long long* normbits, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  unsigned long long mx = 0;
  if (i <= B.hi[0] && j <= B.hi[1]) {
    const int kend = min(t.z0 + tz - 1, B.hi[2]);
    const T* V = v + (ng ? B.off_g1 : B.off_g0);
    for (int k = t.z0; k <= kend; ++k) {
      const unsigned long long bits =
          absbits(V[cidx(d, ng, i - B.lo[0], j - B.lo[1], k - B.lo[2])]);
      mx = bits > mx ? bits : mx;
    }
  }
  block_max_u64(mx, normbits);
}

// Tiles index coarse cells of coarsen(fine box t.box).
template <typename T>
__global__ void __launch_bounds__(256)
    k_restrict(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ fine,
               const BoxInfo* __restrict__ coarse, const T* __restrict__ rf,
               T* __restrict__ rc, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo F = fine[t.box];
  const BoxInfo C = coarse[F.parent];
  const BoxDims df = dims(F), dc = dims(C);
  const int I = t.x0 + threadIdx.x, J = t.y0 + threadIdx.y;
  const int chx = fdiv2(F.hi[0]), chy = fdiv2(F.hi[1]), chz = fdiv2(F.hi[2]);
  if (I > chx || J > chy) return;
  const int kend = min(t.z0 + tz - 1, chz);
  const T* R = rf + F.off_g0;
  T* Q = rc + C.off_g0;
  const long long sy = df.nx, sz = (long long)df.nx * df.ny;
  for (int K = t.z0; K <= kend; ++K) {
    const long long b = cidx(df, 0, 2 * I - F.lo[0], 2 * J - F.lo[1], 2 * K - F.lo[2]);
    const T z0 = (R[b] + R[b + 1]) + (R[b + sy] + R[b + sy + 1]);
    const T z1 = (R[b + sz] + R[b + sz + 1]) + (R[b + sz + sy] + R[b + sz + sy + 1]);
    Q[cidx(dc, 0, I - C.lo[0], J - C.lo[1], K - C.lo[2])] = (z0 + z1) * T(0.125);
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_prolong_add(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ fine,
                  const BoxInfo* __restrict__ coarse, T* __restrict__ ef,
                  const T* __restrict__ ec, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo F = fine[t.box];
  const BoxInfo C = coarse[F.parent];
  const BoxDims df = dims(F), dc = dims(C);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > F.hi[0] || j > F.hi[1]) return;
  const int kend = min(t.z0 + tz - 1, F.hi[2]);
  T* E = ef + F.off_g1;
  const T* EC = ec + C.off_g1;
  for (int k = t.z0; k <= kend; ++k) {
    const long long p = cidx(df, 1, i - F.lo[0], j - F.lo[1], k - F.lo[2]);
    E[p] += EC[cidx(dc, 1, fdiv2(i) - C.lo[0], fdiv2(j) - C.lo[1], fdiv2(k) - C.lo[2])];
  }
}

__global__ void __launch_bounds__(256)
    k_update(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
             double* __restrict__ phi, const float* __restrict__ e, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  for (int k = t.z0; k <= kend; ++k) {
    const long long p = B.off_g1 + cidx(d, 1, i - B.lo[0], j - B.lo[1], k - B.lo[2]);
    phi[p] += (double)e[p];
  }
}

__global__ void __launch_bounds__(256)
    k_copy_valid(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                 const double* __restrict__ src, int sng, double* __restrict__ dst, int dng,
                 int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  const double* S = src + (sng ? B.off_g1 : B.off_g0);
  double* D = dst + (dng ? B.off_g1 : B.off_g0);
  for (int k = t.z0; k <= kend; ++k) {
    const int il = i - B.lo[0], jl = j - B.lo[1], kl = k - B.lo[2];
    D[cidx(d, dng, il, jl, kl)] = S[cidx(d, sng, il, jl, kl)];
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_zero_valid(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                 T* __restrict__ v, int ng, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  T* V = v + (ng ? B.off_g1 : B.off_g0);
  for (int k = t.z0; k <= kend; ++k) V[cidx(d, ng, i - B.lo[0], j - B.lo[1], k - B.lo[2])] = T(0);
}

// Block sum in a fixed order: lanes by butterfly (every lane ends with the
// same bits), then the first nw waves in index order (every wave of the
// work-group takes part in the barrier; later waves' sums are left out).
__device__ double block_sum_w(double v, double* red, int& phase, int nw) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  double* buf = red + phase * 16;
  phase ^= 1;
  if ((tid & 63) == 0) buf[tid >> 6] = v;
  __syncthreads();
  double s = buf[0];
  for (int w = 1; w < nw; ++w) s += buf[w];
  return s;
}

// ... over every wave of the work-group.
__device__ double block_sum(double v, double* red, int& phase) {
  return block_sum_w(v, red, phase, (blockDim.x * blockDim.y + 63) / 64);
}

__global__ void __launch_bounds__(256)
    k_sum_partial(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                  const double* __restrict__ v, int ng, double* __restrict__ partials, int tz) {
  __shared__ double red[32];
  int phase = 0;
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  double s = 0.0;
  if (i <= B.hi[0] && j <= B.hi[1]) {
    const int kend = min(t.z0 + tz - 1, B.hi[2]);
    const double* V = v + (ng ? B.off_g1 : B.off_g0);
    for (int k = t.z0; k <= kend; ++k) s += V[cidx(d, ng, i - B.lo[0], j - B.lo[1], k - B.lo[2])];
  }
  s = block_sum(s, red, phase);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[blockIdx.x] = s;
}

// Per-tile partial of sum a*b over valid cells (a, b: layouts with ng 0 or 1),
// reduced in a fixed order; k_sum_final adds the partials in order.
__global__ void __launch_bounds__(256)
    k_dot_partial(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                  const double* __restrict__ a, int ang, const double* __restrict__ b, int bng,
                  double* __restrict__ partials, int tz) {
  __shared__ double red[32];
  int phase = 0;
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  double s = 0.0;
  if (i <= B.hi[0] && j <= B.hi[1]) {
    const int kend = min(t.z0 + tz - 1, B.hi[2]);
    const double* A = a + (ang ? B.off_g1 : B.off_g0);
    const double* Bv = b + (bng ? B.off_g1 : B.off_g0);
    const int il = i - B.lo[0], jl = j - B.lo[1];
    for (int k = t.z0; k <= kend; ++k) {
      const int kl = k - B.lo[2];
      s += A[cidx(d, ang, il, jl, kl)] * Bv[cidx(d, bng, il, jl, kl)];
    }
  }
  s = block_sum(s, red, phase);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[blockIdx.x] = s;
}

// Conjugate-gradient updates with the scalars kept on the device.
// x += alpha p, r -= alpha q with alpha = *num / *den; max |r| -> normbits.
// Products and sums are rounded separately (no fused multiply-add), as in
// the plain formulation.
__global__ void __launch_bounds__(256)
    k_cg_xr(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes, double* __restrict__ x,
            const double* __restrict__ p, double* __restrict__ r, const double* __restrict__ q,
            const double* __restrict__ num, const double* __restrict__ den,
            unsigned long long* normbits, float* __restrict__ r32, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  unsigned long long mx = 0;
  if (i <= B.hi[0] && j <= B.hi[1]) {
    const double alpha = *num / *den;
    const int kend = min(t.z0 + tz - 1, B.hi[2]);
    const int il = i - B.lo[0], jl = j - B.lo[1];
    for (int k = t.z0; k <= kend; ++k) {
      const int kl = k - B.lo[2];
      const long long c1 = B.off_g1 + cidx(d, 1, il, jl, kl);
      const long long c0 = B.off_g0 + cidx(d, 0, il, jl, kl);
      x[c1] = __dadd_rn(x[c1], __dmul_rn(alpha, p[c1]));
      const double rv = __dsub_rn(r[c0], __dmul_rn(alpha, q[c0]));
      r[c0] = rv;
      if (r32) r32[c0] = (float)rv;
      const unsigned long long bits = absbits(rv);
      mx = bits > mx ? bits : mx;
    }
  }
  block_max_u64(mx, normbits);
}

// z (ng 1, FP64) = e (ng 1, FP32) on valid cells, and per tile the partial
// of sum r*z (r ghost-free), for k_sum_final.
__global__ void __launch_bounds__(256)
    k_widen_dot(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                const float* __restrict__ e, double* __restrict__ z, const double* __restrict__ r,
                double* __restrict__ partials, int tz) {
  __shared__ double red[32];
  int phase = 0;
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  double s = 0.0;
  if (i <= B.hi[0] && j <= B.hi[1]) {
    const int kend = min(t.z0 + tz - 1, B.hi[2]);
    const int il = i - B.lo[0], jl = j - B.lo[1];
    for (int k = t.z0; k <= kend; ++k) {
      const int kl = k - B.lo[2];
      const long long c1 = B.off_g1 + cidx(d, 1, il, jl, kl);
      const double zv = (double)e[c1];
      z[c1] = zv;
      s += r[B.off_g0 + cidx(d, 0, il, jl, kl)] * zv;
    }
  }
  s = block_sum(s, red, phase);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[blockIdx.x] = s;
}

// Krylov-basis kernels over one level's valid cells (vectors ghost-free,
// basis vector i at V + i*vstride).  Partials of every product go to
// partials[i*pstride + poff + tile], so a level's tiles can follow another
// level's in the same row and one ordered sum per i covers both.
__global__ void __launch_bounds__(256)
    k_mdot(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
           const double* __restrict__ w, const double* __restrict__ V, long long vstride, int n,
           double* __restrict__ partials, int pstride, int poff, int tz) {
  __shared__ double red[32];
  int phase = 0;
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  const bool act = i <= B.hi[0] && j <= B.hi[1];
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  for (int q = 0; q < n; ++q) {
    double s = 0.0;
    if (act)
      for (int k = t.z0; k <= kend; ++k) {
        const long long c = B.off_g0 + cidx(d, 0, i - B.lo[0], j - B.lo[1], k - B.lo[2]);
        s += w[c] * V[q * vstride + c];
      }
    s = block_sum(s, red, phase);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[q * pstride + poff + blockIdx.x] = s;
  }
}

// out = sign*w - sum_q h_q V_q with h_q = sign * dots[q] (subtractions in q
// order, products rounded separately), and the partial of sum out^2.
__global__ void __launch_bounds__(256)
    k_maxpy(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
            const double* __restrict__ w, const double* __restrict__ V, long long vstride, int n,
            const double* __restrict__ dots, double sign, double* __restrict__ out,
            double* __restrict__ partials, int poff, int tz) {
  __shared__ double red[32];
  int phase = 0;
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  double s = 0.0;
  if (i <= B.hi[0] && j <= B.hi[1]) {
    const int kend = min(t.z0 + tz - 1, B.hi[2]);
    for (int k = t.z0; k <= kend; ++k) {
      const long long c = B.off_g0 + cidx(d, 0, i - B.lo[0], j - B.lo[1], k - B.lo[2]);
      double v = sign * w[c];
      for (int q = 0; q < n; ++q) v = __dsub_rn(v, __dmul_rn(sign * dots[q], V[q * vstride + c]));
      out[c] = v;
      s += v * v;
    }
  }
  s = block_sum(s, red, phase);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[poff + blockIdx.x] = s;
}

// v = w / sqrt(*ss) on valid cells (ghost-free).
__global__ void __launch_bounds__(256)
    k_vnormalise(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                 const double* __restrict__ w, double* __restrict__ v, const double* __restrict__ ss,
                 int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const double hn = sqrt(*ss);
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  for (int k = t.z0; k <= kend; ++k) {
    const long long c = B.off_g0 + cidx(d, 0, i - B.lo[0], j - B.lo[1], k - B.lo[2]);
    v[c] = w[c] / hn;
  }
}

// phi (ng 1) += sum_q y[q] Z_q (ng 1, Z_q at Z + q*zstride), in q order.
__global__ void __launch_bounds__(256)
    k_zaxpy(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
            double* __restrict__ phi, const double* __restrict__ Z, long long zstride, int n,
            const double* __restrict__ y, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  for (int k = t.z0; k <= kend; ++k) {
    const long long c = B.off_g1 + cidx(d, 1, i - B.lo[0], j - B.lo[1], k - B.lo[2]);
    double v = phi[c];
    for (int q = 0; q < n; ++q) v = __dadd_rn(v, __dmul_rn(y[q], Z[q * zstride + c]));
    phi[c] = v;
  }
}

// p = z (first) or p = z + (*num / *den) p, both with one ghost layer.
__global__ void __launch_bounds__(256)
    k_cg_p(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes, double* __restrict__ p,
           const double* __restrict__ z, const double* __restrict__ num,
           const double* __restrict__ den, int first, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const double beta = first ? 0.0 : *num / *den;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  const int il = i - B.lo[0], jl = j - B.lo[1];
  for (int k = t.z0; k <= kend; ++k) {
    const long long c = B.off_g1 + cidx(d, 1, il, jl, k - B.lo[2]);
    p[c] = first ? z[c] : __dadd_rn(z[c], __dmul_rn(beta, p[c]));
  }
}

// One work-group of kSumLanes lanes; lane l adds partials l, l + kSumLanes,
// ... into four accumulators in turn (four independent loads in flight per
// lane: tens of thousands of partials take a few round trips, not hundreds),
// then the accumulators and the lanes in a fixed tree: the same order on
// every call.
constexpr int kSumLanes = 1024;
__global__ void __launch_bounds__(kSumLanes) k_sum_final(const double* __restrict__ partials, int n,
                                                        double* __restrict__ out) {
  __shared__ double red[32];
  int phase = 0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * kSumLanes < n; i += 4 * kSumLanes) {
    a0 += partials[i];
    a1 += partials[i + kSumLanes];
    a2 += partials[i + 2 * kSumLanes];
    a3 += partials[i + 3 * kSumLanes];
  }
  for (; i < n; i += kSumLanes) a0 += partials[i];
  double s = (a0 + a1) + (a2 + a3);
  s = block_sum(s, red, phase);
  if (threadIdx.x == 0) *out = s;
}

__global__ void __launch_bounds__(256)
    k_shift_valid(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                  double* __restrict__ v, int ng, const double* __restrict__ sum, double inv_n,
                  int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const double m = *sum * inv_n;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  double* V = v + (ng ? B.off_g1 : B.off_g0);
  for (int k = t.z0; k <= kend; ++k) V[cidx(d, ng, i - B.lo[0], j - B.lo[1], k - B.lo[2])] -= m;
}

template <typename T>
__global__ void __launch_bounds__(FB_CHUNK)
    k_fill_boundary(const FbTag* __restrict__ tags, const FbChunk* __restrict__ chunks,
                    T* __restrict__ data, int ncomp) {
  const FbChunk c = chunks[blockIdx.x];
  const FbTag g = tags[c.tag];
  const int l = c.start + threadIdx.x;
  if (l >= g.ncell) return;
  const int i = l % g.nx;
  const int r = l / g.nx;
  const int j = r % g.ny;
  const int k = r / g.ny;
  const long long dsti = g.dst_base + i + (long long)j * g.dsy + (long long)k * g.dsz;
  const long long srci = g.src_base + i + (long long)j * g.ssy + (long long)k * g.ssz;
  for (int comp = 0; comp < ncomp; ++comp)
    data[dsti + comp * g.dst_cstride] = data[srci + comp * g.src_cstride];
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Plain device copy, one 16-byte element per lane (the achievable streaming
// rate and the reference for the HBM traffic counters).
__global__ void __launch_bounds__(256)
    k_stream_copy(const uint4* __restrict__ in, uint4* __restrict__ out, long long n) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < n) out[i] = in[i];
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (TO)in[i];
}

__global__ void k_scale_faces(const double* __restrict__ in, double* __restrict__ out,
                              long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = in ? in[i] : v;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_coarsen_cell(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ fine,
                   const BoxInfo* __restrict__ coarse, const T* __restrict__ af,
                   T* __restrict__ ac, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo F = fine[t.box];
  const BoxInfo C = coarse[F.parent];
  const BoxDims df = dims(F), dc = dims(C);
  const int I = t.x0 + threadIdx.x, J = t.y0 + threadIdx.y;
  if (I > fdiv2(F.hi[0]) || J > fdiv2(F.hi[1])) return;
  const int kend = min(t.z0 + tz - 1, fdiv2(F.hi[2]));
  const T* A = af + F.off_g0;
  const long long sy = df.nx, sz = (long long)df.nx * df.ny;
  for (int K = t.z0; K <= kend; ++K) {
    const long long b = cidx(df, 0, 2 * I - F.lo[0], 2 * J - F.lo[1], 2 * K - F.lo[2]);
    const T z0 = (A[b] + A[b + 1]) + (A[b + sy] + A[b + sy + 1]);
    const T z1 = (A[b + sz] + A[b + sz + 1]) + (A[b + sz + sy] + A[b + sz + sy + 1]);
    ac[C.off_g0 + cidx(dc, 0, I - C.lo[0], J - C.lo[1], K - C.lo[2])] = (z0 + z1) * T(0.125);
  }
}

// Face extents of box B along direction d: (nx + (d==0), ny + (d==1), nz + (d==2)).
__device__ __forceinline__ void face_dims(const BoxDims& bd, int d, int& fx, int& fy, int& fz) {
  fx = bd.nx + (d == 0);
  fy = bd.ny + (d == 1);
  fz = bd.nz + (d == 2);
}

// grid.y = fine box; coarse face value = mean of the 4 fine faces on it.
__global__ void __launch_bounds__(256)
    k_coarsen_face(const BoxInfo* __restrict__ fine, const BoxInfo* __restrict__ coarse, int d,
                   const double* __restrict__ bf, double* __restrict__ bc) {
  const BoxInfo F = fine[blockIdx.y];
  const BoxInfo C = coarse[F.parent];
  const BoxDims df = dims(F), dc = dims(C);
  int ffx, ffy, ffz, cfx, cfy, cfz;
  face_dims(df, d, ffx, ffy, ffz);
  face_dims(dc, d, cfx, cfy, cfz);
  // coarse faces lying on coarsen(F): lo/2 .. hi/2 (+1 along d)
  const int clo[3] = {fdiv2(F.lo[0]), fdiv2(F.lo[1]), fdiv2(F.lo[2])};
  const int nxc = df.nx / 2 + (d == 0), nyc = df.ny / 2 + (d == 1), nzc = df.nz / 2 + (d == 2);
  const long long total = (long long)nxc * nyc * nzc;
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const long long fst[3] = {1, ffx, (long long)ffx * ffy};
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int a = e % nxc;
    const int b = (e / nxc) % nyc;
    const int c = e / ((long long)nxc * nyc);
    const int cl[3] = {a, b, c};  // relative to clo
    int fl[3];
    for (int q = 0; q < 3; ++q) fl[q] = 2 * (clo[q] + cl[q]) - F.lo[q];
    const long long base = F.off_f[d] + fl[0] + fl[1] * fst[1] + fl[2] * fst[2];
    const double p0 = bf[base], p1 = bf[base + fst[t2]];
    const double p2 = bf[base + fst[t1]], p3 = bf[base + fst[t1] + fst[t2]];
    const int gl[3] = {clo[0] + a - C.lo[0], clo[1] + b - C.lo[1], clo[2] + c - C.lo[2]};
    bc[C.off_f[d] + gl[0] + (long long)gl[1] * cfx + (long long)gl[2] * cfx * cfy] =
        ((p0 + p1) + (p2 + p3)) * 0.25;
  }
}

__global__ void __launch_bounds__(256)
    k_scatter_faces(const BoxInfo* __restrict__ boxes, int d, int3 dlo, int3 dn,
                    const double* __restrict__ g, double* __restrict__ out, int is_log) {
  const BoxInfo B = boxes[blockIdx.y];
  const BoxDims bd = dims(B);
  int fx, fy, fz;
  face_dims(bd, d, fx, fy, fz);
  const long long gx = dn.x + (d == 0), gy = dn.y + (d == 1);
  const long long total = (long long)fx * fy * fz;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = e % fx, j = (e / fx) % fy, k = e / ((long long)fx * fy);
    const long long gi = (B.lo[0] - dlo.x + i) + gx * ((B.lo[1] - dlo.y + j) + gy * (B.lo[2] - dlo.z + k));
    const double v = g[gi];
    out[B.off_f[d] + e] = is_log ? exp(v) : v;
  }
}

__global__ void __launch_bounds__(256)
    k_scatter_cells(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes, int3 dlo,
                    int3 dn, const double* __restrict__ g, double* __restrict__ out, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  for (int k = t.z0; k <= kend; ++k)
    out[B.off_g0 + cidx(d, 0, i - B.lo[0], j - B.lo[1], k - B.lo[2])] =
        g[(i - dlo.x) + (long long)dn.x * ((j - dlo.y) + (long long)dn.y * (k - dlo.z))];
}

// Adjoint gradient on every face of one box in one pass (grid.y = box).  A
// 64 x 4 block takes 64 x 4 cells of a column of tz planes; a lane computes
// the low x, y and z faces of its cell, and the box's high face along d
// where its cell is the last along d.  The cell below (z) stays in
// registers from the previous plane, the x and y neighbours come through
// the caches; offsets are 32-bit inside a box (face arrays of a box < 2^31
// elements, checked on the host).  MODE 0: per-box face arrays (every face of the box); MODE 1:
// global face arrays: a box writes its low faces, its high faces on the
// domain's high side, and along a periodic direction the face at index 0
// also at index n (the same face).
template <int MODE>
__global__ void __launch_bounds__(256)
    k_face_grad3(StencilArgs<double> op, const double* __restrict__ phi,
                 const double* __restrict__ lam, double* __restrict__ g0,
                 double* __restrict__ g1, double* __restrict__ g2, int3 dlo, int3 dn,
                 int perbits, int ntx, int nty, int tz) {
  const BoxInfo B = op.boxes[blockIdx.y];
  const int nx = B.hi[0] - B.lo[0] + 1, ny = B.hi[1] - B.lo[1] + 1, nz = B.hi[2] - B.lo[2] + 1;
  int t = blockIdx.x;
  const int tx = t % ntx;
  t /= ntx;
  const int ty = t % nty;
  const int tzb = t / nty;
  const int i = tx * 64 + threadIdx.x, j = ty * 4 + threadIdx.y, k0 = tzb * tz;
  if (i >= nx || j >= ny || k0 >= nz) return;
  const int k1 = min(k0 + tz, nz);
  const int sy = nx + 2, sz = sy * (ny + 2);
  const double* __restrict__ P = phi + B.off_g1;
  const double* __restrict__ L = lam + B.off_g1;
  const double* __restrict__ bx = op.b0 + B.off_f[0];
  const double* __restrict__ by = op.b1 + B.off_f[1];
  const double* __restrict__ bz = op.b2 + B.off_f[2];
  const int m = B.bcmask;
  const bool xlo = i == 0, xhi = i == nx - 1, ylo = j == 0, yhi = j == ny - 1;
  // high faces of the box: written in mode 0, or on the domain's high side
  const bool dhx = MODE == 0 || B.hi[0] + 1 - dlo.x == dn.x;
  const bool dhy = MODE == 0 || B.hi[1] + 1 - dlo.y == dn.y;
  const bool dhz = MODE == 0 || B.hi[2] + 1 - dlo.z == dn.z;
  const double beta = op.beta, ih0 = op.ih0, ih1 = op.ih1, ih2 = op.ih2;
  // face-array offsets of face (i, j, k0) in the box's x, y and z face arrays
  int fxo = i + (nx + 1) * (j + ny * k0);
  int fyo = i + nx * (j + (ny + 1) * k0);
  int fzo = i + nx * (j + ny * k0);
  const int fxs = (nx + 1) * ny, fys = nx * (ny + 1), fzs = nx * ny;
  // output offsets of the same faces (box arrays, or the global arrays)
  long long ox, oy, oz, oxs, oys, ozs;
  long long gx0 = 0, gy0 = 0, gz0 = 0;  // global index along d of this lane's low face
  if (MODE == 0) {
    ox = B.off_f[0] + fxo;
    oy = B.off_f[1] + fyo;
    oz = B.off_f[2] + fzo;
    oxs = fxs;
    oys = fys;
    ozs = fzs;
  } else {
    const long long I = B.lo[0] - dlo.x + i, J = B.lo[1] - dlo.y + j, K = B.lo[2] - dlo.z + k0;
    ox = I + (dn.x + 1ll) * (J + (long long)dn.y * K);
    oy = I + (long long)dn.x * (J + (dn.y + 1ll) * K);
    oz = I + (long long)dn.x * (J + (long long)dn.y * K);
    oxs = (dn.x + 1ll) * dn.y;
    oys = (long long)dn.x * (dn.y + 1);
    ozs = (long long)dn.x * dn.y;
    gx0 = I;
    gy0 = J;
    gz0 = K;
  }
  int p = (i + 1) + sy * (j + 1) + sz * (k0 + 1);
  double pb = P[p - sz], lb = L[p - sz];
  for (int k = k0; k < k1; ++k, p += sz, fxo += fxs, fyo += fys, fzo += fzs, ox += oxs,
           oy += oys, oz += ozs) {
    const double pc = P[p], lc = L[p];
    const double pw = P[p - 1], lw = L[p - 1];
    const double ps = P[p - sy], ls = L[p - sy];
    // x faces
    {
      const double c = (beta * bx[fxo]) * ih0;
      const double g = (xlo && (m & 1)) ? -2.0 * c * pc * lc : -c * (pc - pw) * (lc - lw);
      if (MODE == 0) {
        g0[ox] = g;
      } else {
        g0[ox] = g;
        if ((perbits & 1) && gx0 == 0) g0[ox + dn.x] = g;
      }
      if (xhi && dhx) {
        const double ch = (beta * bx[fxo + 1]) * ih0;
        double gh;
        if (m & 2) {
          gh = -2.0 * ch * pc * lc;
        } else {
          const double pe = P[p + 1], le = L[p + 1];
          gh = -ch * (pe - pc) * (le - lc);
        }
        g0[ox + 1] = gh;
      }
    }
    // y faces
    {
      const double c = (beta * by[fyo]) * ih1;
      const double g = (ylo && (m & 4)) ? -2.0 * c * pc * lc : -c * (pc - ps) * (lc - ls);
      g1[oy] = g;
      if (MODE == 1 && (perbits & 2) && gy0 == 0) g1[oy + (long long)dn.x * dn.y] = g;
      if (yhi && dhy) {
        const double ch = (beta * by[fyo + nx]) * ih1;
        double gh;
        if (m & 8) {
          gh = -2.0 * ch * pc * lc;
        } else {
          const double pn = P[p + sy], ln = L[p + sy];
          gh = -ch * (pn - pc) * (ln - lc);
        }
        g1[oy + (MODE == 0 ? nx : dn.x)] = gh;
      }
    }
    // z faces
    {
      const double c = (beta * bz[fzo]) * ih2;
      const bool zlo = k == 0;
      const double g = (zlo && (m & 16)) ? -2.0 * c * pc * lc : -c * (pc - pb) * (lc - lb);
      g2[oz] = g;
      if (MODE == 1 && (perbits & 4) && gz0 + (k - k0) == 0)
        g2[oz + (long long)dn.x * dn.y * dn.z] = g;
      if (k == nz - 1 && dhz) {
        const double ch = (beta * bz[fzo + fzs]) * ih2;
        double gh;
        if (m & 32) {
          gh = -2.0 * ch * pc * lc;
        } else {
          const double pu = P[p + sz], lu = L[p + sz];
          gh = -ch * (pu - pc) * (lu - lc);
        }
        g2[oz + ozs] = gh;
      }
    }
    pb = pc;
    lb = lc;
  }
}

template <typename T>
__global__ void k_bottom_setup(BottomTables bt, StencilArgs<T> op, T* __restrict__ diag,
                               T* __restrict__ coef) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= bt.n) return;
  const T* bs[3] = {op.b0, op.b1, op.b2};
  const T ih[3] = {op.ih0, op.ih1, op.ih2};
  T dg = op.a ? op.alpha * op.a[bt.aidx[c]] : op.alpha;
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const T cf = (op.beta * bs[d][bt.fidx[f * bt.n + c]]) * ih[d];
    const bool wall = bt.nbr[f * bt.n + c] < 0;
    dg = dg + (wall ? T(2) * cf : cf);
    coef[f * bt.n + c] = wall ? T(0) : cf;
  }
  diag[c] = dg;
}

// One work-group of 1024 lanes runs the whole CG; lane l owns cells
// l, l+1024, ...  Vectors x, r, q and the search direction p live in the
// workspace (L2-resident at bottom sizes); every phase that reads another
// lane's p is separated by a barrier.  Dot products accumulate in double.
template <typename T>
__global__ void __launch_bounds__(1024)
    k_bottom_cg(BottomTables bt, const T* __restrict__ diag, const T* __restrict__ coef,
                const T* __restrict__ rhs, T* __restrict__ out, int accumulate, T* work,
                double tol, int maxiter, int singular, int* iters_out) {
  __shared__ double red[32];
  int phase = 0;
  const int n = bt.n;
  T* x = work;
  T* r = work + n;
  T* p = work + 2 * (long long)n;
  T* q = work + 3 * (long long)n;
  const int tid = threadIdx.x, nt = blockDim.x;
  double s = 0.0;
  for (int c = tid; c < n; c += nt) {
    const T v = rhs[bt.map_rhs[c]];
    r[c] = v;
    x[c] = T(0);
    s += (double)v;
  }
  if (singular) {
    s = block_sum(s, red, phase);
    const T m = (T)(s / n);
    for (int c = tid; c < n; c += nt) r[c] = r[c] - m;
  }
  s = 0.0;
  for (int c = tid; c < n; c += nt) s += (double)r[c] * (double)r[c];
  double rho = block_sum(s, red, phase);
  const double bnorm = sqrt(rho);
  int it = 0;
  if (bnorm > 0.0) {
    for (int c = tid; c < n; c += nt) p[c] = r[c];
    while (it < maxiter) {
      __syncthreads();
      s = 0.0;
      for (int c = tid; c < n; c += nt) {
        T off = T(0);
        for (int f = 0; f < 6; ++f) {
          const int nb = bt.nbr[f * n + c];
          off = off + (nb < 0 ? T(0) : coef[f * n + c] * p[nb]);
        }
        const T qv = diag[c] * p[c] - off;
        q[c] = qv;
        s += (double)p[c] * (double)qv;
      }
      const double pq = block_sum(s, red, phase);
      const double al = rho / pq;
      const T alT = (T)al;
      s = 0.0;
      for (int c = tid; c < n; c += nt) {
        x[c] = x[c] + alT * p[c];
        const T rv = r[c] - alT * q[c];
        r[c] = rv;
        s += (double)rv * (double)rv;
      }
      ++it;
      const double rho_new = block_sum(s, red, phase);
      if (!(sqrt(rho_new) > tol * bnorm)) break;
      const T btT = (T)(rho_new / rho);
      // p is read by other lanes in the next product: barrier before rewriting
      __syncthreads();
      for (int c = tid; c < n; c += nt) p[c] = r[c] + btT * p[c];
      rho = rho_new;
    }
  }
  if (singular) {
    s = 0.0;
    for (int c = tid; c < n; c += nt) s += (double)x[c];
    s = block_sum(s, red, phase);
    const T m = (T)(s / n);
    for (int c = tid; c < n; c += nt) x[c] = x[c] - m;
  }
  for (int c = tid; c < n; c += nt) {
    const long long o = bt.map_out[c];
    out[o] = accumulate ? out[o] + x[c] : x[c];
  }
  if (tid == 0) *iters_out = it;
}

// One work-group (whole wavefronts, up to 1024 lanes) runs the whole
// BiCGStab (stabilised bi-conjugate gradients, shadow residual r^ = r_0,
// from x = 0); lane l owns cells l, l+nt, ...  Iteration:
// p = r + beta (p - omega v), v = A p, alpha = rho / (r^, v), s = r - alpha v,
// t = A s, omega = (t, s) / (t, t), x = (x + alpha p) + omega s,
// r = s - omega t, rho = (r^, r).  Stops on
// ||r||_2 <= tol ||r_0||_2, on ||s||_2 there (x += alpha p), or on a
// breakdown (rho or (r^, v) zero; (t, t) zero takes x += alpha p).  The
// seven vectors live in the workspace (L2-resident at bottom sizes); p and
// s, which other lanes read in the products, are separated from their
// writes by barriers.  Dots accumulate in double.
template <typename T>
__global__ void __launch_bounds__(1024)
    k_bottom_bicgstab(BottomTables bt, const T* __restrict__ diag, const T* __restrict__ coef,
                      const T* __restrict__ rhs, T* __restrict__ out, int accumulate, T* work,
                      double tol, int maxiter, int singular, int* iters_out) {
  __shared__ double red[32];
  int phase = 0;
  const int n = bt.n;
  T* x = work;
  T* r = work + n;
  T* rh = work + 2 * (long long)n;
  T* p = work + 3 * (long long)n;
  T* v = work + 4 * (long long)n;
  T* sv = work + 5 * (long long)n;
  T* tv = work + 6 * (long long)n;
  const int tid = threadIdx.x, nt = blockDim.x;
  auto apply = [&](const T* u, int c) {
    T off = T(0);
    for (int f = 0; f < 6; ++f) {
      const int nb = bt.nbr[f * n + c];
      off = off + (nb < 0 ? T(0) : coef[f * n + c] * u[nb]);
    }
    return diag[c] * u[c] - off;
  };
  double s = 0.0;
  for (int c = tid; c < n; c += nt) {
    const T val = rhs[bt.map_rhs[c]];
    r[c] = val;
    x[c] = T(0);
    s += (double)val;
  }
  if (singular) {
    s = block_sum(s, red, phase);
    const T m = (T)(s / n);
    for (int c = tid; c < n; c += nt) r[c] = r[c] - m;
  }
  s = 0.0;
  for (int c = tid; c < n; c += nt) {
    rh[c] = r[c];
    p[c] = T(0);
    v[c] = T(0);
    s += (double)r[c] * (double)r[c];
  }
  double rho = block_sum(s, red, phase);
  const double bnorm = sqrt(rho);
  int it = 0;
  if (bnorm > 0.0) {
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    while (it < maxiter) {
      if (rho == 0.0) break;
      const T btT = (T)((rho / rho_prev) * (alpha / omega));
      const T omT = (T)omega;
      for (int c = tid; c < n; c += nt) p[c] = r[c] + btT * (p[c] - omT * v[c]);
      __syncthreads();
      s = 0.0;
      for (int c = tid; c < n; c += nt) {
        const T q = apply(p, c);
        v[c] = q;
        s += (double)rh[c] * (double)q;
      }
      const double rv = block_sum(s, red, phase);
      if (rv == 0.0) break;
      alpha = rho / rv;
      const T alT = (T)alpha;
      s = 0.0;
      for (int c = tid; c < n; c += nt) {
        const T q = r[c] - alT * v[c];
        sv[c] = q;
        s += (double)q * (double)q;
      }
      ++it;
      const double ss = block_sum(s, red, phase);
      if (!(sqrt(ss) > tol * bnorm)) {
        for (int c = tid; c < n; c += nt) x[c] = x[c] + alT * p[c];
        break;
      }
      double ts = 0.0;
      s = 0.0;
      for (int c = tid; c < n; c += nt) {
        const T q = apply(sv, c);
        tv[c] = q;
        ts += (double)q * (double)sv[c];
        s += (double)q * (double)q;
      }
      const double tt = block_sum(s, red, phase);
      ts = block_sum(ts, red, phase);
      if (tt == 0.0) {
        for (int c = tid; c < n; c += nt) x[c] = x[c] + alT * p[c];
        break;
      }
      omega = ts / tt;
      const T om2 = (T)omega;
      double rr = 0.0, rhr = 0.0;
      for (int c = tid; c < n; c += nt) {
        x[c] = (x[c] + alT * p[c]) + om2 * sv[c];
        const T q = sv[c] - om2 * tv[c];
        r[c] = q;
        rr += (double)q * (double)q;
        rhr += (double)rh[c] * (double)q;
      }
      rr = block_sum(rr, red, phase);
      rhr = block_sum(rhr, red, phase);
      if (!(sqrt(rr) > tol * bnorm)) break;
      if (omega == 0.0) break;
      rho_prev = rho;
      rho = rhr;
    }
  }
  if (singular) {
    s = 0.0;
    for (int c = tid; c < n; c += nt) s += (double)x[c];
    s = block_sum(s, red, phase);
    const T m = (T)(s / n);
    for (int c = tid; c < n; c += nt) x[c] = x[c] - m;
  }
  for (int c = tid; c < n; c += nt) {
    const long long o = bt.map_out[c];
    out[o] = accumulate ? out[o] + x[c] : x[c];
  }
  if (tid == 0) *iters_out = it;
}

// Coarse cells of coarsen(fine box): mean of the 8 children or zero.
template <typename T>
__global__ void __launch_bounds__(256)
    k_avgdown(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ fine,
              const BoxInfo* __restrict__ coarse, const T* __restrict__ f, int fng,
              T* __restrict__ c, int cng, int zero_only, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo F = fine[t.box];
  const BoxInfo C = coarse[F.parent];
  const BoxDims df = dims(F), dc = dims(C);
  const int I = t.x0 + threadIdx.x, J = t.y0 + threadIdx.y;
  if (I > fdiv2(F.hi[0]) || J > fdiv2(F.hi[1])) return;
  const int kend = min(t.z0 + tz - 1, fdiv2(F.hi[2]));
  const T* R = zero_only ? nullptr : f + (fng ? F.off_g1 : F.off_g0);
  T* Q = c + (cng ? C.off_g1 : C.off_g0);
  const long long sy = df.nx + 2 * fng, sz = sy * (df.ny + 2 * fng);
  for (int K = t.z0; K <= kend; ++K) {
    const long long q = cidx(dc, cng, I - C.lo[0], J - C.lo[1], K - C.lo[2]);
    if (zero_only) {
      Q[q] = T(0);
      continue;
    }
    const long long b = cidx(df, fng, 2 * I - F.lo[0], 2 * J - F.lo[1], 2 * K - F.lo[2]);
    const T z0 = (R[b] + R[b + 1]) + (R[b + sy] + R[b + sy + 1]);
    const T z1 = (R[b + sz] + R[b + sz + 1]) + (R[b + sz + sy] + R[b + sz + sy + 1]);
    Q[q] = (z0 + z1) * T(0.125);
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_cf_ghost(const CfGhost* __restrict__ g, int n, const T* __restrict__ coarse,
               T* __restrict__ fine) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CfGhost e = g[i];
  const T vc = coarse[e.c];
  T acc = T(0);
  for (int d = 0; d < 3; ++d) {
    const T lo = e.nb[2 * d] >= 0 ? coarse[e.nb[2 * d]] : -vc;
    const T hi = e.nb[2 * d + 1] >= 0 ? coarse[e.nb[2 * d + 1]] : -vc;
    const T s = T(0.5) * (hi - lo);
    acc = acc + (((e.sign >> d) & 1) ? s : -s);
  }
  fine[e.dst] = vc + T(0.25) * acc;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_cf_reflux(const CfCell* __restrict__ cells, int ncell, const CfFace* __restrict__ faces,
                const T* __restrict__ phic, const T* __restrict__ phif, const T* __restrict__ bc0,
                const T* __restrict__ bc1, const T* __restrict__ bc2, const T* __restrict__ bf0,
                const T* __restrict__ bf1, const T* __restrict__ bf2, T beta, T ihc0, T ihc1,
                T ihc2, T ihf0, T ihf1, T ihf2, T* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const CfCell cc = cells[i];
  const T pI = phic[cc.phi_idx];
  T acc = r[cc.r_idx];
  for (int k = 0; k < cc.count; ++k) {
    const CfFace f = faces[cc.first + k];
    const T* bc = f.d == 0 ? bc0 : (f.d == 1 ? bc1 : bc2);
    const T* bf = f.d == 0 ? bf0 : (f.d == 1 ? bf1 : bf2);
    const T ic = f.d == 0 ? ihc0 : (f.d == 1 ? ihc1 : ihc2);
    const T ifn = f.d == 0 ? ihf0 : (f.d == 1 ? ihf1 : ihf2);
    const T c = (beta * bc[f.cb_idx]) * ic;
    const T term_c = c * (pI - phic[f.j_idx]);
    T fl[4];
    for (int q = 0; q < 4; ++q) fl[q] = beta * bf[f.fb[q]] * (phif[f.fg[q]] - phif[f.fv[q]]);
    // mean fine flux / h_c, ifn = 1 / (h_f h_c)
    const T term_f = (((fl[0] + fl[1]) + (fl[2] + fl[3])) * T(0.25)) * ifn;
    acc = acc + (term_c - term_f);
  }
  r[cc.r_idx] = acc;
}

__global__ void __launch_bounds__(256)
    k_axpy_valid(const Tile* __restrict__ tiles, const BoxInfo* __restrict__ boxes,
                 double* __restrict__ v, const double* __restrict__ w, int tz) {
  const Tile t = tiles[blockIdx.x];
  const BoxInfo B = boxes[t.box];
  const BoxDims d = dims(B);
  const int i = t.x0 + threadIdx.x, j = t.y0 + threadIdx.y;
  if (i > B.hi[0] || j > B.hi[1]) return;
  const int kend = min(t.z0 + tz - 1, B.hi[2]);
  for (int k = t.z0; k <= kend; ++k) {
    const long long p = B.off_g1 + cidx(d, 1, i - B.lo[0], j - B.lo[1], k - B.lo[2]);
    v[p] += w[p];
  }
}

// The same CG with the search direction p held in LDS and each lane's x, r, q
// in registers (CPT cells per lane, lane l owns l, l+nt, ...), and for up to
// two cells per lane also their stencil (diagonal, six coefficients and
// neighbours): an iteration then reads nothing but LDS.  The work-group is
// sized to the bottom level (one wavefront for 64 cells), so its reductions
// cross few wavefronts.  Same arithmetic per cell as k_bottom_cg.
// The body runs on any work-group: lanes stride the cells by nt (lane l owns
// l, l+nt, ...), the dot products add the first nw waves' sums, and every
// wave takes part in the barriers (lanes past the cells hold zeros).  p:
// n values of LDS.
// The CG's sums and barriers.  ONE_WAVE: the CG runs in wavefront 0 alone
// (n <= 64, lanes 0..63): the butterfly leaves the sum in every lane (the
// value the work-group form reads back for one wave) and LDS needs only
// wave-level ordering.
template <bool ONE_WAVE>
__device__ __forceinline__ double cg_sum(double v, double* red, int& phase, int nw) {
  if (ONE_WAVE) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  }
  return block_sum_w(v, red, phase, nw);
}

template <bool ONE_WAVE>
__device__ __forceinline__ void cg_sync() {
  if (ONE_WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename T, int CPT, bool ONE_WAVE = false>
__device__ __forceinline__ void cg_lds_run(const BottomTables& bt, const T* __restrict__ diag,
                                           const T* __restrict__ coef, const T* __restrict__ rhs,
                                           T* __restrict__ out, int accumulate, double tol,
                                           int maxiter, int singular, int* iters_out, T* p,
                                           double* red, int nt, int nw) {
  // no multiply-add fusion: whether the compiler fuses a product into an
  // addition depends on the code around it, and the work-group and the
  // one-wavefront forms (and every kernel that runs this body) must round
  // the same way
#pragma clang fp contract(off)
  int phase = 0;
  const int n = bt.n;
  const int tid = threadIdx.x;
  // stencil in registers up to two cells per lane (more would spill)
  constexpr bool REG = CPT <= 2;
  constexpr int RC = REG ? CPT : 1;
  T x[CPT], r[CPT], q[CPT], dg[RC], cf[RC][6];
  int nb[RC][6];
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
    const int c = tid + m * nt;
    x[m] = T(0);
    r[m] = T(0);
    if (c < n) {
      r[m] = rhs[bt.map_rhs[c]];
      s += (double)r[m];
    }
    if (REG) {
      dg[m % RC] = c < n ? diag[c] : T(1);
      for (int f = 0; f < 6; ++f) {
        nb[m % RC][f] = c < n ? bt.nbr[f * n + c] : -1;
        cf[m % RC][f] = c < n ? coef[f * n + c] : T(0);
      }
    }
  }
  if (singular) {
    s = cg_sum<ONE_WAVE>(s, red, phase, nw);
    const T mean = (T)(s / n);
#pragma unroll
    for (int m = 0; m < CPT; ++m)
      if (tid + m * nt < n) r[m] = r[m] - mean;
  }
  s = 0.0;
#pragma unroll
  for (int m = 0; m < CPT; ++m) s += (double)r[m] * (double)r[m];
  double rho = cg_sum<ONE_WAVE>(s, red, phase, nw);
  const double bnorm = sqrt(rho);
  int it = 0;
  if (bnorm > 0.0) {
#pragma unroll
    for (int m = 0; m < CPT; ++m)
      if (tid + m * nt < n) p[tid + m * nt] = r[m];
    while (it < maxiter) {
      cg_sync<ONE_WAVE>();
      s = 0.0;
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * nt;
        q[m] = T(0);
        if (c < n) {
          T off = T(0);
          if (REG) {
#pragma unroll
            for (int f = 0; f < 6; ++f)
              off = off + (nb[m % RC][f] < 0 ? T(0) : cf[m % RC][f] * p[nb[m % RC][f]]);
            q[m] = dg[m % RC] * p[c] - off;
          } else {
            for (int f = 0; f < 6; ++f) {
              const int k = bt.nbr[f * n + c];
              off = off + (k < 0 ? T(0) : coef[f * n + c] * p[k]);
            }
            q[m] = diag[c] * p[c] - off;
          }
          s += (double)p[c] * (double)q[m];
        }
      }
      const double pq = cg_sum<ONE_WAVE>(s, red, phase, nw);
      const T alT = (T)(rho / pq);
      s = 0.0;
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * nt;
        if (c < n) {
          x[m] = x[m] + alT * p[c];
          r[m] = r[m] - alT * q[m];
          s += (double)r[m] * (double)r[m];
        }
      }
      ++it;
      const double rho_new = cg_sum<ONE_WAVE>(s, red, phase, nw);
      if (!(sqrt(rho_new) > tol * bnorm)) break;
      const T btT = (T)(rho_new / rho);
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * nt;
        if (c < n) p[c] = r[m] + btT * p[c];
      }
      rho = rho_new;
    }
  }
  if (singular) {
    s = 0.0;
#pragma unroll
    for (int m = 0; m < CPT; ++m)
      if (tid + m * nt < n) s += (double)x[m];
    s = cg_sum<ONE_WAVE>(s, red, phase, nw);
    const T mean = (T)(s / n);
#pragma unroll
    for (int m = 0; m < CPT; ++m) x[m] = x[m] - mean;
  }
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
    const int c = tid + m * nt;
    if (c < n) {
      const long long o = bt.map_out[c];
      out[o] = accumulate ? out[o] + x[m] : x[m];
    }
  }
  if (tid == 0) *iters_out = it;
}

template <typename T, int CPT>
__global__ void __launch_bounds__(1024)
    k_bottom_cg_lds(BottomTables bt, const T* __restrict__ diag, const T* __restrict__ coef,
                    const T* __restrict__ rhs, T* __restrict__ out, int accumulate, double tol,
                    int maxiter, int singular, int* iters_out) {
  extern __shared__ unsigned char lds_raw[];
  __shared__ double red[32];
  cg_lds_run<T, CPT>(bt, diag, coef, rhs, out, accumulate, tol, maxiter, singular, iters_out,
                     reinterpret_cast<T*>(lds_raw), red, blockDim.x, (blockDim.x + 63) / 64);
}

// ---------------------------------------------------------------------------
// The coarse tail (launch_tail): one work-group, a barrier between passes.
// Every pass evaluates the operator with eval and stores each result once,
// with the update, residual, restriction and interpolation expressions of
// the per-level kernels, so it stores the bits those launches store.
// Box tables (BoxInfo, WtBox) are staged in LDS at the start; cell entries,
// data and write-through entries stay in global memory (the L2 cache, at
// these sizes).  Pointers read from the plan are cast to the global address
// space so that their accesses compile to global loads and stores, which a
// lane can have in flight while it reads LDS.

#define TAIL_G __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ TAIL_G T* g1(T* p) {
  return (TAIL_G T*)p;
}

__device__ __forceinline__ void tail_unpack(unsigned c, int& b, int& il, int& jl, int& kl) {
  kl = (int)(c & 63u);
  jl = (int)((c >> 6) & 63u);
  il = (int)((c >> 12) & 63u);
  b = (int)(c >> 18);
}

// The arrays of one tail level, global address space.
template <typename T>
struct TailPtrs {
  TAIL_G T* e;
  TAIL_G const T* rhs;
  TAIL_G T* r;
  TAIL_G const T* b0;
  TAIL_G const T* b1;
  TAIL_G const T* b2;
  TAIL_G const T* a;
  TAIL_G const WtEntry* wte;
  TAIL_G const unsigned* cells;
};

template <typename T>
__device__ __forceinline__ TailPtrs<T> tail_ptrs(const TailLevel<T>& L) {
  TailPtrs<T> q;
  q.e = g1(L.e);
  q.rhs = g1((const T*)L.rhs);
  q.r = g1(L.r);
  q.b0 = g1(L.op.b0);
  q.b1 = g1(L.op.b1);
  q.b2 = g1(L.op.b2);
  q.a = L.op.a ? g1(L.op.a) : nullptr;
  q.wte = g1(L.wte);
  q.cells = g1(L.cells);
  return q;
}

// gather's loads (same indices, rhs without ghosts) through global pointers
template <typename T, bool READ_PHI, bool READ_CENTRE>
__device__ __forceinline__ void tail_gather(Nbr<T>& v, const Strides& s, const TailPtrs<T>& q,
                                            const BoxInfo& B, bool read_f, int il, int jl,
                                            int kl, int pc) {
  TAIL_G const T* P = q.e + B.off_g1;
  if (read_f) v.f = q.rhs[B.off_g0 + il + s.rsy * jl + s.rsz * kl];
  const int fx = il + (s.nx + 1) * (jl + s.ny * kl);
  const int fy = il + s.nx * (jl + (s.ny + 1) * kl);
  const int fz = il + s.nx * (jl + s.ny * kl);
  TAIL_G const T* BX = q.b0 + B.off_f[0];
  TAIL_G const T* BY = q.b1 + B.off_f[1];
  TAIL_G const T* BZ = q.b2 + B.off_f[2];
  v.bxl = BX[fx];
  v.bxh = BX[fx + 1];
  v.byl = BY[fy];
  v.byh = BY[fy + s.nx];
  v.bzl = BZ[fz];
  v.bzh = BZ[fz + s.nx * s.ny];
  if (q.a) v.a = q.a[B.off_g0 + fz];
  if (READ_CENTRE) v.pc = P[pc];
  if (READ_PHI) {
    v.pxl = P[pc - 1];
    v.pxh = P[pc + 1];
    v.pyl = P[pc - s.sy];
    v.pyh = P[pc + s.sy];
    v.pzl = P[pc - s.sz];
    v.pzh = P[pc + s.sz];
  }
}

// a new value of a cell on its box's boundary layer into the face ghosts
// that mirror it (every entry of each face it lies on; wt_store's test)
template <typename T>
__device__ __forceinline__ void tail_wt(const WtBox& wb, TAIL_G const WtEntry* wte,
                                        TAIL_G T* phi, const Strides& s, int il, int jl, int kl,
                                        T v) {
  const bool on[6] = {il == 0, il == s.nx - 1, jl == 0, jl == s.ny - 1, kl == 0, kl == s.nz - 1};
  for (int f = 0; f < 6; ++f) {
    if (!on[f]) continue;
    for (int e = wb.first[f]; e < wb.first[f] + wb.count[f]; ++e) {
      TAIL_G const WtEntry* w = wte + e;
      if (il >= w->lo[0] && il <= w->hi[0] && jl >= w->lo[1] && jl <= w->hi[1] &&
          kl >= w->lo[2] && kl <= w->hi[2])
        phi[w->base + il + (long long)jl * w->sy + (long long)kl * w->sz] = v;
    }
  }
}

__device__ __forceinline__ bool on_rim(const Strides& s, int il, int jl, int kl) {
  return il == 0 || il == s.nx - 1 || jl == 0 || jl == s.ny - 1 || kl == 0 || kl == s.nz - 1;
}

// Half-sweep of one colour (red = 0): two cells per lane and step; each
// phase (cell entries, then the stencil's loads) is issued for both cells
// before either waits.  ZG: from zero (only rhs is read).  bi, wb: the
// level's box tables in LDS.
template <typename T, bool ZG>
__device__ __forceinline__ void tail_half(const TailLevel<T>& L, const TailPtrs<T>& q,
                                          const BoxInfo* bi, const WtBox* wb, int colour) {
  const int beg = colour ? L.nred : 0, end = colour ? L.ncell : L.nred;
  const int nt = blockDim.x;
  for (int q0 = beg + (int)threadIdx.x; q0 < end; q0 += 2 * nt) {
    const bool ok1 = q0 + nt < end;
    const unsigned c0 = q.cells[q0];
    const unsigned c1 = ok1 ? q.cells[q0 + nt] : 0u;
    Nbr<T> v[2];
    int b[2], il[2], jl[2], kl[2], pc[2];
    Strides s[2];
    tail_unpack(c0, b[0], il[0], jl[0], kl[0]);
    tail_unpack(c1, b[1], il[1], jl[1], kl[1]);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !ok1) continue;
      const BoxInfo& B = bi[b[u]];
      s[u] = strides_of(B, 0);
      pc[u] = (il[u] + 1) + s[u].sy * (jl[u] + 1) + s[u].sz * (kl[u] + 1);
      tail_gather<T, !ZG, false>(v[u], s[u], q, B, true, il[u], jl[u], kl[u], pc[u]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !ok1) continue;
      const BoxInfo& B = bi[b[u]];
      const Cell<T> c = eval<T, !ZG>(L.op, v[u], q.a != nullptr, B.bcmask, s[u], il[u], jl[u],
                                     kl[u]);
      const T nv = ZG ? v[u].f / c.diag : (v[u].f + c.off) / c.diag;
      q.e[B.off_g1 + pc[u]] = nv;
      if (on_rim(s[u], il[u], jl[u], kl[u]))
        tail_wt<T>(wb[b[u]], q.wte, q.e, s[u], il[u], jl[u], kl[u], nv);
    }
  }
}

// r = rhs - A e on every cell (k_residual's expression)
template <typename T>
__device__ __forceinline__ void tail_resid(const TailLevel<T>& L, const TailPtrs<T>& q,
                                           const BoxInfo* bi) {
  const int nt = blockDim.x;
  for (int q0 = (int)threadIdx.x; q0 < L.ncell; q0 += 2 * nt) {
    const bool ok1 = q0 + nt < L.ncell;
    const unsigned c0 = q.cells[q0];
    const unsigned c1 = ok1 ? q.cells[q0 + nt] : 0u;
    Nbr<T> v[2];
    int b[2], il[2], jl[2], kl[2];
    Strides s[2];
    tail_unpack(c0, b[0], il[0], jl[0], kl[0]);
    tail_unpack(c1, b[1], il[1], jl[1], kl[1]);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !ok1) continue;
      const BoxInfo& B = bi[b[u]];
      s[u] = strides_of(B, 0);
      const int pc = (il[u] + 1) + s[u].sy * (jl[u] + 1) + s[u].sz * (kl[u] + 1);
      tail_gather<T, true, true>(v[u], s[u], q, B, true, il[u], jl[u], kl[u], pc);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !ok1) continue;
      const BoxInfo& B = bi[b[u]];
      const Cell<T> c = eval<T, true>(L.op, v[u], q.a != nullptr, B.bcmask, s[u], il[u], jl[u],
                                      kl[u]);
      const T Aphi = c.diag * v[u].pc - c.off;
      q.r[B.off_g0 + il[u] + s[u].nx * (jl[u] + s[u].ny * kl[u])] = v[u].f - Aphi;
    }
  }
}

// rc (no ghosts, boxes ci) = mean of the 8 children in rf (no ghosts,
// boxes fi), k_restrict's summation order
template <typename T>
__device__ __forceinline__ void tail_restrict(TAIL_G const T* rf, const BoxInfo* fi,
                                              TAIL_G const unsigned* rcells, int n,
                                              const BoxInfo* ci, TAIL_G T* rc) {
  for (int q = (int)threadIdx.x; q < n; q += blockDim.x) {
    int fb, oi, oj, ok;
    tail_unpack(rcells[q], fb, oi, oj, ok);
    const BoxInfo& F = fi[fb];
    const BoxInfo& C = ci[F.parent];
    const BoxDims df = dims(F), dc = dims(C);
    const int I = fdiv2(F.lo[0]) + oi, J = fdiv2(F.lo[1]) + oj, K = fdiv2(F.lo[2]) + ok;
    TAIL_G const T* R = rf + F.off_g0;
    const long long sy = df.nx, sz = (long long)df.nx * df.ny;
    const long long b = cidx(df, 0, 2 * I - F.lo[0], 2 * J - F.lo[1], 2 * K - F.lo[2]);
    const T z0 = (R[b] + R[b + 1]) + (R[b + sy] + R[b + sy + 1]);
    const T z1 = (R[b + sz] + R[b + sz + 1]) + (R[b + sz + sy] + R[b + sz + sy + 1]);
    rc[C.off_g0 + cidx(dc, 0, I - C.lo[0], J - C.lo[1], K - C.lo[2])] = (z0 + z1) * T(0.125);
  }
}

// e += parent value of ec (k_prolong_add's addition), written through to
// the face ghosts, so the first post-smoothing half-sweep needs no exchange
template <typename T>
__device__ __forceinline__ void tail_prolong(const TailLevel<T>& L, const TailPtrs<T>& q,
                                             const BoxInfo* bi, const WtBox* wb,
                                             const BoxInfo* ci, TAIL_G const T* ec) {
  for (int i0 = (int)threadIdx.x; i0 < L.ncell; i0 += blockDim.x) {
    int b, il, jl, kl;
    tail_unpack(q.cells[i0], b, il, jl, kl);
    const BoxInfo& F = bi[b];
    const BoxInfo& C = ci[F.parent];
    const BoxDims df = dims(F), dc = dims(C);
    const long long p = F.off_g1 + cidx(df, 1, il, jl, kl);
    const int i = il + F.lo[0], j = jl + F.lo[1], k = kl + F.lo[2];
    const T nv = q.e[p] + ec[C.off_g1 + cidx(dc, 1, fdiv2(i) - C.lo[0], fdiv2(j) - C.lo[1],
                                              fdiv2(k) - C.lo[2])];
    q.e[p] = nv;
    const Strides s = strides_of(F, 0);
    if (on_rim(s, il, jl, kl)) tail_wt<T>(wb[b], q.wte, q.e, s, il, jl, kl, nv);
  }
}

__device__ __forceinline__ void lds_copy(void* dst, const void* src, int bytes) {
  int* d = static_cast<int*>(dst);
  TAIL_G const int* s = g1(static_cast<const int*>(src));
  for (int i = (int)threadIdx.x; i < bytes / 4; i += blockDim.x) d[i] = s[i];
}

template <typename T>
__global__ void __launch_bounds__(kTailLanes) k_tail(const TailPlan<T>* __restrict__ tp) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  __shared__ double red[32];
  const int nlev = tp->nlev, nu1 = tp->nu1, nu2 = tp->nu2;
  // stage the box tables
  lds_copy(tail_lds + tp->lds_fi, tp->finfo, (int)sizeof(BoxInfo) * tp->fnbox);
  for (int l = 0; l < nlev; ++l) {
    lds_copy(tail_lds + tp->lds_bi[l], tp->lev[l].op.boxes, (int)sizeof(BoxInfo) * tp->lev[l].nbox);
    lds_copy(tail_lds + tp->lds_wb[l], tp->lev[l].wtb, (int)sizeof(WtBox) * tp->lev[l].nbox);
  }
  lds_copy(tail_lds + tp->lds_bi[nlev], tp->binfo, (int)sizeof(BoxInfo) * tp->bnbox);
  __syncthreads();
  auto BI = [&](int l) { return reinterpret_cast<const BoxInfo*>(tail_lds + tp->lds_bi[l]); };
  auto WB = [&](int l) { return reinterpret_cast<const WtBox*>(tail_lds + tp->lds_wb[l]); };
  tail_restrict<T>(g1(tp->rf), reinterpret_cast<const BoxInfo*>(tail_lds + tp->lds_fi),
                   g1(tp->rcells), tp->nrc, BI(0), g1(tp->lev[0].rhs));
  __syncthreads();
  for (int l = 0; l < nlev; ++l) {
    const TailLevel<T>& L = tp->lev[l];
    const TailPtrs<T> q = tail_ptrs(L);
    for (int k = 0; k < nu1; ++k) {
      if (k == 0)
        tail_half<T, true>(L, q, BI(l), WB(l), 0);
      else
        tail_half<T, false>(L, q, BI(l), WB(l), 0);
      __syncthreads();
      tail_half<T, false>(L, q, BI(l), WB(l), 1);
      __syncthreads();
    }
    tail_resid<T>(L, q, BI(l));
    __syncthreads();
    tail_restrict<T>(q.r, BI(l), g1(L.rcells), L.nrc, BI(l + 1),
                     g1(l + 1 < nlev ? tp->lev[l + 1].rhs : tp->brhs));
    __syncthreads();
  }
  {
    BottomTables bt = tp->bt;
    T* p = reinterpret_cast<T*>(tail_lds);
    if (bt.n <= 64) {
      if (threadIdx.x < 64)
        cg_lds_run<T, 1, true>(bt, tp->bdiag, tp->bcoef, tp->brhs, tp->be, 0, tp->tol,
                               tp->maxiter, tp->singular, tp->iters, p, red, 64, 1);
    } else {
      cg_lds_run<T, 1>(bt, tp->bdiag, tp->bcoef, tp->brhs, tp->be, 0, tp->tol, tp->maxiter,
                       tp->singular, tp->iters, p, red, blockDim.x, (bt.n + 63) / 64);
    }
  }
  __syncthreads();
  const int c0 = tp->reverse ? 1 : 0;
  for (int l = nlev - 1; l >= 0; --l) {
    const TailLevel<T>& L = tp->lev[l];
    const TailPtrs<T> q = tail_ptrs(L);
    tail_prolong<T>(L, q, BI(l), WB(l), BI(l + 1), g1(l + 1 < nlev ? tp->lev[l + 1].e : tp->be));
    __syncthreads();
    for (int k = 0; k < nu2; ++k) {
      tail_half<T, false>(L, q, BI(l), WB(l), c0);
      __syncthreads();
      tail_half<T, false>(L, q, BI(l), WB(l), 1 - c0);
      __syncthreads();
    }
  }
}

#undef TAIL_G

inline dim3 block_of(Shape sh) { return dim3(sh.lx, sh.ly, 1); }

}  // namespace

template <typename T>
hipError_t launch_gsrb(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                       const StencilArgs<T>& op, T* phi, const T* rhs, int rhs_ng, int colour,
                       int zero_guess, const WtBox* wtb, const WtEntry* wte,
                       const BoxInfo* cinfo, const T* ec, const BoxInfo* finfo, const T* rf,
                       T* rout) {
  if (ntiles <= 0) return hipSuccess;
  if (ec && (!wtb || zero_guess || !cinfo)) return hipErrorInvalidValue;
  if (rf && (!zero_guess || ec || !finfo || !rout || rhs_ng != 0)) return hipErrorInvalidValue;
  const dim3 g(ntiles), b = block_of(sh);
  const size_t lds = wtb ? 2 * (size_t)sh.ly * sh.tz * sizeof(T) : 0;
#define GS(U, Z, W, X, E, F, RS)                                                                 \
  hipLaunchKernelGGL((k_gsrb<T, U, Z, W, X, E, F, RS>), g, b, lds, st, tiles, op, phi, rhs,      \
                     rhs_ng, colour, sh.tz, wtb, wte, cinfo, ec, finfo, rf, rout)
#define GSU(Z, W, X, E, F)                       \
  if (sh.u >= 4) GS(4, Z, W, X, E, F, false);    \
  else if (sh.u == 2) GS(2, Z, W, X, E, F, false); \
  else GS(1, Z, W, X, E, F, false);
#define GSR(X)                                  \
  if (sh.u >= 4) GS(4, true, false, X, false, false, true); \
  else if (sh.u == 2) GS(2, true, false, X, false, false, true); \
  else GS(1, true, false, X, false, false, true);
  // buffer loads on the write-through paths the solve runs most, where the
  // level streams (op.buf)
  const bool buf = op.buf != 0;
  if (sh.wp == 2) {
    // two cells of the colour per lane (FP32, buffer loads, write-through)
    if constexpr (!std::is_same<T, float>::value) {
      return hipErrorInvalidValue;
    } else {
      if (!buf || !wtb || rf || sh.u > 2) return hipErrorInvalidValue;
#define GQ(Z, E)                                                                              \
  if (sh.u == 2)                                                                              \
    hipLaunchKernelGGL((k_gsrb_quad<2, Z, E>), g, b, lds, st, tiles, op, phi, rhs, rhs_ng,    \
                       colour, sh.tz, wtb, wte, cinfo, ec);                                   \
  else                                                                                        \
    hipLaunchKernelGGL((k_gsrb_quad<1, Z, E>), g, b, lds, st, tiles, op, phi, rhs, rhs_ng,    \
                       colour, sh.tz, wtb, wte, cinfo, ec);
      if (ec) { GQ(false, true) }
      else if (zero_guess) { GQ(true, false) }
      else { GQ(false, false) }
#undef GQ
      return hipGetLastError();
    }
  }
  if (rf) {
    // the restriction into this level's rhs folded into its zero-guess
    // first half-sweep (global loads, as on every cached level)
    if (wtb) { GSR(true) }
    else { GSR(false) }
  } else if (ec) {
    // never whole pairs: the other cell of a pair would be stored with its
    // correction while other lanes still read it and add the correction.
    // Buffer loads (the correction's included) where the level streams: at
    // 256^3 with single-plane tiles 164 against 171 us (FP64), and faster in
    // FP32 as well
    if (buf) { GSU(false, false, true, true, true) }
    else { GSU(false, false, true, true, false) }
  } else if (wtb) {
    // a zero-guess half-sweep reads f and the faces once each: streaming
    // levels take them through buffer descriptors with the non-temporal hint
    if (zero_guess && buf) { GSU(true, false, true, false, true) }
    else if (zero_guess) { GSU(true, false, true, false, false) }
    else if (sh.wp) { GSU(false, true, true, false, false) }
    else if (buf) { GSU(false, false, true, false, true) }
    else { GSU(false, false, true, false, false) }
  } else {
    if (zero_guess) { GSU(true, false, false, false, false) }
    else if (sh.wp) { GSU(false, true, false, false, false) }
    else { GSU(false, false, false, false, false) }
  }
#undef GSR
#undef GSU
#undef GS
  return hipGetLastError();
}

// Tile shapes the fused sweep is instantiated for: (lx, ly) cells.
bool sweep_shape_ok(Shape sh) {
  return ((sh.lx == 64 && (sh.ly == 4 || sh.ly == 8)) || (sh.lx == 32 && (sh.ly == 8 || sh.ly == 16))) &&
         sh.tz >= 1;
}

size_t sweep_lds_bytes(Shape sh, size_t elem) {
  if (!sweep_shape_ok(sh)) return 0;
  const size_t n = 5 * (size_t)(sh.lx + 4) * (sh.ly + 4) + 3 * (size_t)(sh.lx + 2) * (sh.ly + 2);
  return n * elem;
}

template <typename T>
hipError_t launch_sweep(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const StencilArgs<T>& op, const T* pin, T* pout, const T* rhs,
                        int rhs_ng, int zero_guess, unsigned long long* normbits) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = sweep_lds_bytes(sh, sizeof(T));
  if (!lds) return hipErrorInvalidValue;
  const dim3 g(ntiles), b((sh.lx / 2) * sh.ly);
#define SW(X, Y, Z, N)                                                                        \
  hipLaunchKernelGGL((k_sweep<T, X, Y, Z, N>), g, b, lds, st, tiles, op, pin, pout, rhs,       \
                     rhs_ng, sh.tz, normbits)
#define SWS(X, Y)                                 \
  if (zero_guess) SW(X, Y, true, false);          \
  else if (normbits) SW(X, Y, false, true);       \
  else SW(X, Y, false, false);
  if (sh.lx == 64 && sh.ly == 4) { SWS(64, 4) }
  else if (sh.lx == 64) { SWS(64, 8) }
  else if (sh.ly == 8) { SWS(32, 8) }
  else { SWS(32, 16) }
#undef SWS
#undef SW
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rim(hipStream_t st, const RimTile* tiles, int ntiles, const StencilArgs<T>& op,
                      T* phi, const T* rhs, int rhs_ng) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rim<T>, dim3(ntiles), dim3(256), 0, st, tiles, op, phi, rhs, rhs_ng);
  return hipGetLastError();
}

template <typename T, typename TO>
hipError_t launch_residual(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                           const StencilArgs<T>& op, const T* phi, const T* rhs, int rhs_ng,
                           TO* out, unsigned long long* normbits, int mode,
                           double* dot_partials, T* pnext, const WtBox* wtb, const WtEntry* wte) {
  if (ntiles <= 0) return hipSuccess;
  if (pnext && (mode != 0 || !rhs || pnext == phi)) return hipErrorInvalidValue;
  if ((wtb || wte) && (!pnext || !wtb || !wte)) return hipErrorInvalidValue;
  const dim3 g(ntiles), b = block_of(sh);
#define RS(U, F, N)                                                                           \
  hipLaunchKernelGGL((k_residual<T, TO, U, F, N>), g, b, 0, st, tiles, op, phi, rhs, rhs_ng,    \
                     out, normbits, sh.tz, mode, dot_partials, pnext, wtb, wte)
#define RSU(F, N) \
  if (sh.u >= 4) RS(4, F, N); else if (sh.u == 2) RS(2, F, N); else RS(1, F, N);
  // buffer loads where the level streams (op.buf)
  if (pnext) {
    if constexpr (std::is_same<T, TO>::value) {
      if (op.buf) { RSU(true, true) } else { RSU(false, true) }
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    if (op.buf) { RSU(true, false) } else { RSU(false, false) }
  }
#undef RSU
#undef RS
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resid_restrict(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                                 const StencilArgs<T>& op, const T* phi, const T* rhs, int rhs_ng,
                                 const BoxInfo* cinfo, T* rc) {
  if (ntiles <= 0) return hipSuccess;
  if (sh.lx < 2 || (sh.lx & 1) || (sh.ly & 1) || (sh.tz & 1) || sh.lx * sh.ly > 256)
    return hipErrorInvalidValue;
  const dim3 g(ntiles), b = block_of(sh);
  if (op.buf)
    hipLaunchKernelGGL((k_resid_restrict<T, true>), g, b, 0, st, tiles, op, phi, rhs, rhs_ng,
                       sh.tz, cinfo, rc);
  else
    hipLaunchKernelGGL((k_resid_restrict<T, false>), g, b, 0, st, tiles, op, phi, rhs, rhs_ng,
                       sh.tz, cinfo, rc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_maxabs(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                         const BoxInfo* boxes, const T* v, int ng, unsigned long long* normbits) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_maxabs<T>, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, v, ng,
                     normbits, sh.tz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                           const BoxInfo* fine, const BoxInfo* coarse, const T* rf, T* rc) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict<T>, dim3(ntiles), block_of(sh), 0, st, tiles, fine, coarse, rf,
                     rc, sh.tz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                              const BoxInfo* fine, const BoxInfo* coarse, T* ef, const T* ec) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prolong_add<T>, dim3(ntiles), block_of(sh), 0, st, tiles, fine, coarse, ef,
                     ec, sh.tz);
  return hipGetLastError();
}

hipError_t launch_update(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                         const BoxInfo* boxes, double* phi, const float* e) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, phi, e, sh.tz);
  return hipGetLastError();
}

hipError_t launch_copy_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, const double* src, int src_ng, double* dst,
                             int dst_ng) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_valid, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, src, src_ng,
                     dst, dst_ng, sh.tz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zero_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, T* v, int ng) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_valid<T>, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, v, ng,
                     sh.tz);
  return hipGetLastError();
}

hipError_t launch_sum_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                            const BoxInfo* boxes, const double* v, int ng, double* partials,
                            double* sum) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_partial, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, v, ng,
                     partials, sh.tz);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kSumLanes), 0, st, partials, ntiles, sum);
  return hipGetLastError();
}

hipError_t launch_shift_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                              const BoxInfo* boxes, double* v, int ng, const double* sum,
                              long long ncell) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shift_valid, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, v, ng, sum,
                     1.0 / (double)ncell, sh.tz);
  return hipGetLastError();
}

hipError_t launch_dot(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                      const BoxInfo* boxes, const double* a, int ang, const double* b, int bng,
                      double* partials, double* out) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dot_partial, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, a, ang, b,
                     bng, partials, sh.tz);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kSumLanes), 0, st, partials, ntiles, out);
  return hipGetLastError();
}

hipError_t launch_cg_xr(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const BoxInfo* boxes, double* x, const double* p, double* r,
                        const double* q, const double* num, const double* den,
                        unsigned long long* normbits, float* r32) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_xr, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, x, p, r, q, num,
                     den, normbits, r32, sh.tz);
  return hipGetLastError();
}

hipError_t launch_sum_final(hipStream_t st, const double* partials, int n, double* out) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kSumLanes), 0, st, partials, n, out);
  return hipGetLastError();
}

// One ordered sum per row: out[q] = sum of partials[q*n .. q*n + n - 1].
__global__ void __launch_bounds__(256) k_sum_rows(const double* __restrict__ partials, int n,
                                                  double* __restrict__ out) {
  __shared__ double red[32];
  int phase = 0;
  double s = 0.0;
  const double* row = partials + (long long)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += row[i];
  s = block_sum(s, red, phase);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

hipError_t launch_mdot(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                       const BoxInfo* boxes, const double* w, const double* V, long long vstride,
                       int n, double* partials, int pstride, int poff) {
  if (ntiles <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mdot, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, w, V, vstride, n,
                     partials, pstride, poff, sh.tz);
  return hipGetLastError();
}

hipError_t launch_sum_rows(hipStream_t st, const double* partials, int rows, int n, double* out) {
  if (rows <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_rows, dim3(rows), dim3(256), 0, st, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_maxpy(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const BoxInfo* boxes, const double* w, const double* V, long long vstride,
                        int n, const double* dots, double sign, double* out, double* partials,
                        int poff) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_maxpy, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, w, V, vstride, n,
                     dots, sign, out, partials, poff, sh.tz);
  return hipGetLastError();
}

hipError_t launch_vnormalise(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, const double* w, double* v, const double* ss) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vnormalise, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, w, v, ss,
                     sh.tz);
  return hipGetLastError();
}

hipError_t launch_zaxpy(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                        const BoxInfo* boxes, double* phi, const double* Z, long long zstride,
                        int n, const double* y) {
  if (ntiles <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zaxpy, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, phi, Z, zstride, n,
                     y, sh.tz);
  return hipGetLastError();
}

hipError_t launch_widen_dot(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                            const BoxInfo* boxes, const float* e, double* z, const double* r,
                            double* partials, double* out) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_widen_dot, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, e, z, r,
                     partials, sh.tz);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kSumLanes), 0, st, partials, ntiles, out);
  return hipGetLastError();
}

hipError_t launch_cg_p(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                       const BoxInfo* boxes, double* p, const double* z, const double* num,
                       const double* den, int first) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_p, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, p, z, num, den,
                     first, sh.tz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_boundary(hipStream_t st, const FbTag* tags, const FbChunk* chunks,
                                int nchunks, T* data, int ncomp) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_boundary<T>, dim3(nchunks), dim3(FB_CHUNK), 0, st, tags, chunks, data,
                     ncomp);
  return hipGetLastError();
}

// Fixed device scratch of the allocation-free ghost exchange: the copy plan
// (tags, then chunks) of the last such call on this device.  In host code the
// array's name is not a device address; fb_scratch_address() returns the
// address the runtime resolved for the current device.
static __device__ __align__(256) unsigned char scratch[kFbScratchBytes];

hipError_t fb_scratch_address(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mtx;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mtx);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_fill_u64(hipStream_t st, unsigned long long* p, int n, unsigned long long v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, st, p, n, v);
  return hipGetLastError();
}

static inline int grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename TI, typename TO>
hipError_t launch_convert(hipStream_t st, const TI* in, TO* out, long long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_stream_copy(hipStream_t st, const void* in, void* out, long long n16) {
  if (n16 <= 0) return hipSuccess;
  const long long blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const uint4*>(in), static_cast<uint4*>(out), n16);
  return hipGetLastError();
}

hipError_t launch_scale_faces(hipStream_t st, const double* in, double* out, long long n,
                              double v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_faces, dim3(grid_for(n)), dim3(256), 0, st, in, out, n, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarsen_cell(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                               const BoxInfo* fine, const BoxInfo* coarse, const T* af, T* ac) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarsen_cell<T>, dim3(ntiles), block_of(sh), 0, st, tiles, fine, coarse,
                     af, ac, sh.tz);
  return hipGetLastError();
}

hipError_t launch_coarsen_face(hipStream_t st, const BoxInfo* fine, int nbox_fine,
                               const BoxInfo* coarse, int d, const double* bf, double* bc,
                               int max_faces_per_box) {
  if (nbox_fine <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarsen_face, dim3(grid_for(max_faces_per_box), nbox_fine), dim3(256), 0,
                     st, fine, coarse, d, bf, bc);
  return hipGetLastError();
}

hipError_t launch_scatter_faces(hipStream_t st, const BoxInfo* boxes, int nbox, int d,
                                const int dom_lo[3], const int dom_n[3], const double* g,
                                double* out, int is_log, int max_faces_per_box) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_faces, dim3(grid_for(max_faces_per_box), nbox), dim3(256), 0, st,
                     boxes, d, make_int3(dom_lo[0], dom_lo[1], dom_lo[2]),
                     make_int3(dom_n[0], dom_n[1], dom_n[2]), g, out, is_log);
  return hipGetLastError();
}

hipError_t launch_scatter_cells(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                                const BoxInfo* boxes, const int dom_lo[3], const int dom_n[3],
                                const double* g, double* out) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_cells, dim3(ntiles), block_of(sh), 0, st, tiles, boxes,
                     make_int3(dom_lo[0], dom_lo[1], dom_lo[2]),
                     make_int3(dom_n[0], dom_n[1], dom_n[2]), g, out, sh.tz);
  return hipGetLastError();
}

hipError_t launch_face_grad(hipStream_t st, int nbox, const StencilArgs<double>& op,
                            const double* phi, const double* lam, double* const out[3], int mode,
                            const int dom_lo[3], const int dom_n[3], int perbits,
                            const int max_n[3]) {
  if (nbox <= 0) return hipSuccess;
  const int tz = 8;
  const int ntx = (max_n[0] + 63) / 64, nty = (max_n[1] + 3) / 4, ntz = (max_n[2] + tz - 1) / tz;
  const long long nblk = (long long)ntx * nty * ntz;
  if (nblk > 0x7fffffffll || nbox > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblk, nbox), block(64, 4);
  const int3 lo = make_int3(dom_lo[0], dom_lo[1], dom_lo[2]);
  const int3 n = make_int3(dom_n[0], dom_n[1], dom_n[2]);
  if (mode == 0)
    hipLaunchKernelGGL(k_face_grad3<0>, grid, block, 0, st, op, phi, lam, out[0], out[1], out[2],
                       lo, n, perbits, ntx, nty, tz);
  else
    hipLaunchKernelGGL(k_face_grad3<1>, grid, block, 0, st, op, phi, lam, out[0], out[1], out[2],
                       lo, n, perbits, ntx, nty, tz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_avgdown(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                          const BoxInfo* fine, const BoxInfo* coarse, const T* f, int fng, T* c,
                          int cng, int zero_only) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_avgdown<T>, dim3(ntiles), block_of(sh), 0, st, tiles, fine, coarse, f, fng,
                     c, cng, zero_only, sh.tz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cf_ghost(hipStream_t st, const CfGhost* g, int n, const T* coarse, T* fine) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cf_ghost<T>, dim3((n + 255) / 256), dim3(256), 0, st, g, n, coarse, fine);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cf_reflux(hipStream_t st, const CfCell* cells, int ncell, const CfFace* faces,
                            const T* phic, const T* phif, const T* bc0, const T* bc1,
                            const T* bc2, const T* bf0, const T* bf1, const T* bf2, double beta,
                            const double ihc[3], const double ihf[3], T* r) {
  if (ncell <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cf_reflux<T>, dim3((ncell + 255) / 256), dim3(256), 0, st, cells, ncell,
                     faces, phic, phif, bc0, bc1, bc2, bf0, bf1, bf2, (T)beta, (T)ihc[0],
                     (T)ihc[1], (T)ihc[2], (T)ihf[0], (T)ihf[1], (T)ihf[2], r);
  return hipGetLastError();
}

hipError_t launch_axpy_valid(hipStream_t st, const Tile* tiles, int ntiles, Shape sh,
                             const BoxInfo* boxes, double* v, const double* w) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_valid, dim3(ntiles), block_of(sh), 0, st, tiles, boxes, v, w, sh.tz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bottom_setup(hipStream_t st, const BottomTables& bt, const StencilArgs<T>& op,
                               T* diag, T* coef) {
  if (bt.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bottom_setup<T>, dim3((bt.n + 255) / 256), dim3(256), 0, st, bt, op, diag,
                     coef);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bottom_cg(hipStream_t st, const BottomTables& bt, const T* diag, const T* coef,
                            const T* rhs, T* out, int accumulate, T* work, double tol,
                            int maxiter, int singular, int* iters_out) {
  if (bt.n <= 0) return hipSuccess;
  const size_t lds = sizeof(T) * (size_t)bt.n;
  if (lds <= 61440 && bt.n <= 8 * 1024) {  // stays under 64 KiB with the reduction scratch
    // up to 1024 cells one per lane in whole wavefronts, then 1024 lanes
    const int nt = bt.n <= 1024 ? (bt.n + 63) / 64 * 64 : 1024;
#define CGL(C) \
  hipLaunchKernelGGL((k_bottom_cg_lds<T, C>), dim3(1), dim3(nt), lds, st, bt, diag, coef, rhs, \
                     out, accumulate, tol, maxiter, singular, iters_out)
    if (bt.n <= 1024) CGL(1); else if (bt.n <= 2048) CGL(2); else if (bt.n <= 4096) CGL(4);
    else CGL(8);
#undef CGL
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_bottom_cg<T>, dim3(1), dim3(1024), 0, st, bt, diag, coef, rhs, out,
                     accumulate, work, tol, maxiter, singular, iters_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail(hipStream_t st, const TailPlan<T>* plan, int nbottom, size_t lds) {
  if (!plan || nbottom <= 0 || nbottom > kTailMaxBottom || lds > kTailMaxLds)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(kTailLanes), lds, st, plan);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bottom_bicgstab(hipStream_t st, const BottomTables& bt, const T* diag,
                                  const T* coef, const T* rhs, T* out, int accumulate, T* work,
                                  double tol, int maxiter, int singular, int* iters_out) {
  if (bt.n <= 0) return hipSuccess;
  const int nt = bt.n <= 1024 ? (bt.n + 63) / 64 * 64 : 1024;  // whole wavefronts
  hipLaunchKernelGGL(k_bottom_bicgstab<T>, dim3(1), dim3(nt), 0, st, bt, diag, coef, rhs, out,
                     accumulate, work, tol, maxiter, singular, iters_out);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_gsrb<T>(hipStream_t, const Tile*, int, Shape, const StencilArgs<T>&, \
                                     T*, const T*, int, int, int, const WtBox*,                  \
                                     const WtEntry*, const BoxInfo*, const T*, const BoxInfo*,   \
                                     const T*, T*);                                              \
  template hipError_t launch_sweep<T>(hipStream_t, const Tile*, int, Shape,                      \
                                      const StencilArgs<T>&, const T*, T*, const T*, int, int,   \
                                      unsigned long long*);                                      \
  template hipError_t launch_rim<T>(hipStream_t, const RimTile*, int, const StencilArgs<T>&, T*, \
                                    const T*, int);                                              \
  template hipError_t launch_avgdown<T>(hipStream_t, const Tile*, int, Shape, const BoxInfo*,    \
                                        const BoxInfo*, const T*, int, T*, int, int);            \
  template hipError_t launch_cf_ghost<T>(hipStream_t, const CfGhost*, int, const T*, T*);        \
  template hipError_t launch_cf_reflux<T>(hipStream_t, const CfCell*, int, const CfFace*,        \
                                          const T*, const T*, const T*, const T*, const T*,      \
                                          const T*, const T*, const T*, double, const double*,   \
                                          const double*, T*);                                    \
  template hipError_t launch_maxabs<T>(hipStream_t, const Tile*, int, Shape, const BoxInfo*,     \
                                       const T*, int, unsigned long long*);                      \
  template hipError_t launch_restrict<T>(hipStream_t, const Tile*, int, Shape, const BoxInfo*,   \
                                         const BoxInfo*, const T*, T*);                          \
  template hipError_t launch_resid_restrict<T>(hipStream_t, const Tile*, int, Shape,             \
                                               const StencilArgs<T>&, const T*, const T*, int,   \
                                               const BoxInfo*, T*);                              \
  template hipError_t launch_prolong_add<T>(hipStream_t, const Tile*, int, Shape,                \
                                            const BoxInfo*, const BoxInfo*, T*, const T*);       \
  template hipError_t launch_zero_valid<T>(hipStream_t, const Tile*, int, Shape, const BoxInfo*, \
                                           T*, int);                                             \
  template hipError_t launch_fill_boundary<T>(hipStream_t, const FbTag*, const FbChunk*, int, T*, \
                                              int);                                              \
  template hipError_t launch_coarsen_cell<T>(hipStream_t, const Tile*, int, Shape,               \
                                             const BoxInfo*, const BoxInfo*, const T*, T*);      \
  template hipError_t launch_bottom_setup<T>(hipStream_t, const BottomTables&,                   \
                                             const StencilArgs<T>&, T*, T*);                     \
  template hipError_t launch_bottom_cg<T>(hipStream_t, const BottomTables&, const T*, const T*,  \
                                          const T*, T*, int, T*, double, int, int, int*);      \
  template hipError_t launch_bottom_bicgstab<T>(hipStream_t, const BottomTables&, const T*,      \
                                                const T*, const T*, T*, int, T*, double, int,    \
                                                int, int*);                                      \
  template hipError_t launch_tail<T>(hipStream_t, const TailPlan<T>*, int, size_t);

INST(double)
INST(float)
#undef INST

template hipError_t launch_residual<double, double>(hipStream_t, const Tile*, int, Shape,
                                                    const StencilArgs<double>&, const double*,
                                                    const double*, int, double*,
                                                    unsigned long long*, int, double*, double*,
                                                    const WtBox*, const WtEntry*);
template hipError_t launch_residual<double, float>(hipStream_t, const Tile*, int, Shape,
                                                   const StencilArgs<double>&, const double*,
                                                   const double*, int, float*,
                                                   unsigned long long*, int, double*, double*,
                                                   const WtBox*, const WtEntry*);
template hipError_t launch_residual<float, float>(hipStream_t, const Tile*, int, Shape,
                                                  const StencilArgs<float>&, const float*,
                                                  const float*, int, float*,
                                                  unsigned long long*, int, double*, float*,
                                                  const WtBox*, const WtEntry*);
template hipError_t launch_convert<double, float>(hipStream_t, const double*, float*, long long);
template hipError_t launch_convert<float, double>(hipStream_t, const float*, double*, long long);

}  // namespace amrmg
