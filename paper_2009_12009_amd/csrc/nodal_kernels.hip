// gfx950 kernels of the node-centred finite-element solve (the nodal solver
// of the paper's "Linear Solvers" section).
//
// Finest level: (A phi)_u = sum over the 8 cells s at node u of sigma_s times
// the cell's stiffness row, (1/V) sum_{corners b} K_{1-s, b} phi(u + b + s - 1);
// K depends only on which coordinates of the two corners differ, so the
// kernel takes the 8 values kappa[pattern] (K / V).  Coarse levels: 27
// couplings per node, 14 stored (offsets >= 0 in (z, y, x) order, the centre
// first), the other 13 read from the neighbour they couple to.
//
// Work-groups are 64 x 4 lanes (x contiguous across a wavefront) marching
// tz planes along z.  On the finest level the 3 x 3 x 3 block of phi and the
// 2 x 2 x 2 block of sigma a node needs are kept in registers from plane to
// plane, so a step loads one new plane of each.
#include <hip/hip_runtime.h>

#include "nodal.hpp"

namespace amrmg {

namespace {

__device__ __forceinline__ int pidx(const NdGeo& g, int x, int y, int z) {
  // padded element of unknown (x, y, z); x, y, z in [-1, m]
  return (x + 1) + g.px * ((y + 1) + g.py * (z + 1));
}

// Work-groups go to the 8 XCDs round robin (block b to XCD b % 8), and each
// XCD has its own L2.  The tiled kernels take their tile from a 1-D grid of
// 8 * ceil(n / 8) blocks so that every XCD runs one contiguous run of the
// tile order (x fastest, then y, then z): tiles that share halo rows and
// planes then share an L2.  A block past the last tile has no work.
constexpr int kNdXcds = 8;

__device__ __forceinline__ bool nd_tile(int ntx, int nty, int ntz, int& tx, int& ty, int& tz) {
  const int n = ntx * nty * ntz;
  const int per = (n + kNdXcds - 1) / kNdXcds;
  const int b = (int)blockIdx.x;
  const int t = (b % kNdXcds) * per + b / kNdXcds;
  if (t >= n) return false;
  tx = t % ntx;
  const int r = t / ntx;
  ty = r % nty;
  tz = r / nty;
  return true;
}

__device__ __forceinline__ int nd_ntx(const NdGeo& g) { return (g.mx + 63) / 64; }
__device__ __forceinline__ int nd_nty(const NdGeo& g) { return (g.my + 3) / 4; }
__device__ __forceinline__ int nd_ntz(const NdGeo& g) { return (g.mz + g.tz - 1) / g.tz; }

__device__ __forceinline__ unsigned long long absbits(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}

// Unsigned max of a per-lane value over the work-group, folded into way
// (blockIdx % kNdNormWays) of the slot at dst (skipped when the way already
// holds at least that value).
__device__ void nd_block_max(unsigned long long v, unsigned long long* dst) {
  const int nb = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  dst += kNdNormStride * (nb % kNdNormWays);
  __shared__ unsigned long long red[16];
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = (unsigned long long)__shfl_xor((long long)v, o);
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

// The 14 stored offsets, centre first, then (z, y, x) lexicographic.
__constant__ int kUp[kNdStored][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 1, 0}, {0, 1, 0},  {1, 1, 0}, {-1, -1, 1}, {0, -1, 1},
    {1, -1, 1}, {-1, 0, 1}, {0, 0, 1},  {1, 0, 1},  {-1, 1, 1}, {0, 1, 1},  {1, 1, 1}};

// Finest-level sweep, see nd_launch_sweep0.
template <int MODE, bool NORM>
__global__ void __launch_bounds__(256)
    k_nd_sweep0(NdGeo g, NdKappa kap, const double* __restrict__ sig,
                const double* __restrict__ phi, const double* __restrict__ f,
                double* __restrict__ out, double omega, unsigned long long* norm) {
  int tx, ty, tz;
  if (!nd_tile(nd_ntx(g), nd_nty(g), nd_ntz(g), tx, ty, tz)) return;  // whole block
  const int ux = tx * 64 + threadIdx.x;
  const int uy = ty * 4 + threadIdx.y;
  const int z0 = tz * g.tz;
  const bool act = ux < g.mx && uy < g.my && z0 < g.mz;
  unsigned long long mx = 0;
  if (act) {
    const int z1 = min(z0 + g.tz, g.mz);
    const int sx = g.mx + 1, sy = g.my + 1;  // sigma pitches
    double P[3][3][3];  // [z - uz + 1][y - uy + 1][x - ux + 1]
    double S[2][2][2];  // sigma of cells [z][y][x] = u + s
    if (MODE != ND_ZERO) {
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx)
            P[dz + 1][dy][dx] = phi[pidx(g, ux + dx - 1, uy + dy - 1, z0 + dz - 1)];
    }
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx)
        S[1][cy][cx] = sig[(ux + cx) + sx * ((uy + cy) + sy * z0)];
    for (int uz = z0; uz < z1; ++uz) {
      // shift the register blocks one plane down and load the new plane
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          S[0][cy][cx] = S[1][cy][cx];
          S[1][cy][cx] = sig[(ux + cx) + sx * ((uy + cy) + sy * (uz + 1))];
        }
      if (MODE != ND_ZERO) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            P[0][dy][dx] = P[1][dy][dx];
            P[1][dy][dx] = P[2][dy][dx];
            P[2][dy][dx] = phi[pidx(g, ux + dx - 1, uy + dy - 1, uz + 1)];
          }
      }
      const int c = pidx(g, ux, uy, uz);
      const double fv = f[c];
      double ssum = 0.0;
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) ssum += S[cz][cy][cx];
      const double diag = kap.k[0] * ssum;
      double v;
      if (MODE == ND_ZERO) {
        v = omega * fv / diag;
      } else {
        // cell s spans offsets s-1 .. s along each direction
        double ap = 0.0;
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
          for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
              double t = 0.0;
#pragma unroll
              for (int bz = 0; bz < 2; ++bz)
#pragma unroll
                for (int by = 0; by < 2; ++by)
#pragma unroll
                  for (int bx = 0; bx < 2; ++bx) {
                    const int ox = cx - 1 + bx, oy = cy - 1 + by, oz = cz - 1 + bz;
                    const int pat = (ox != 0 ? 1 : 0) | (oy != 0 ? 2 : 0) | (oz != 0 ? 4 : 0);
                    t += kap.k[pat] * P[oz + 1][oy + 1][ox + 1];
                  }
              ap += S[cz][cy][cx] * t;
            }
        const double r = fv - ap;
        if (NORM) {
          const unsigned long long b = absbits(r);
          mx = b > mx ? b : mx;
        }
        v = MODE == ND_RESID ? r : (MODE == ND_APPLY ? ap : P[1][1][1] + omega * r / diag);
      }
      out[c] = v;
    }
  }
  if (NORM) nd_block_max(mx, norm);
}

// Coarse-level sweep (stored couplings), see nd_launch_sweep_st.
template <int MODE, bool NORM>
__global__ void __launch_bounds__(256)
    k_nd_sweep_st(NdGeo g, NdStencilC s, const double* __restrict__ phi,
                  const double* __restrict__ f, double* __restrict__ out, double omega,
                  unsigned long long* norm) {
  int tx, ty, tz;
  if (!nd_tile(nd_ntx(g), nd_nty(g), nd_ntz(g), tx, ty, tz)) return;  // whole block
  const int ux = tx * 64 + threadIdx.x;
  const int uy = ty * 4 + threadIdx.y;
  const int z0 = tz * g.tz;
  const bool act = ux < g.mx && uy < g.my && z0 < g.mz;
  unsigned long long mx = 0;
  if (act) {
    const int z1 = min(z0 + g.tz, g.mz);
    for (int uz = z0; uz < z1; ++uz) {
      const int c = pidx(g, ux, uy, uz);
      const double fv = f[c];
      const double diag = s.w[0][c];
      double v;
      if (MODE == ND_ZERO) {
        v = omega * fv / diag;
      } else {
        double ap = diag * phi[c];
#pragma unroll
        for (int q = 1; q < kNdStored; ++q) {
          const int d = kUp[q][0] + g.px * (kUp[q][1] + g.py * kUp[q][2]);
          ap += s.w[q][c] * phi[c + d];
          ap += s.w[q][c - d] * phi[c - d];
        }
        const double r = fv - ap;
        if (NORM) {
          const unsigned long long b = absbits(r);
          mx = b > mx ? b : mx;
        }
        v = MODE == ND_RESID ? r : (MODE == ND_APPLY ? ap : phi[c] + omega * r / diag);
      }
      out[c] = v;
    }
  }
  if (NORM) nd_block_max(mx, norm);
}

// Index along one direction of fine unknown 2 G + u for coarse unknown I
// (G = I + off, off = 1 on a Dirichlet direction), wrapped when periodic.
__device__ __forceinline__ int fine_of(int I, int u, bool per, int mf) {
  int q = 2 * I + (per ? 0 : 1) + u;
  if (per) q = q < 0 ? q + mf : (q >= mf ? q - mf : q);
  return q;
}

__device__ __forceinline__ double pw1(int t) { return t == 0 ? 1.0 : ((t == 1 || t == -1) ? 0.5 : 0.0); }

__global__ void __launch_bounds__(256)
    k_nd_restrict(NdGeo gf, NdGeo gc, const double* __restrict__ rf, double* __restrict__ rc) {
  int tx, ty, K;
  if (!nd_tile(nd_ntx(gc), nd_nty(gc), gc.mz, tx, ty, K)) return;
  const int I = tx * 64 + threadIdx.x;
  const int J = ty * 4 + threadIdx.y;
  if (I >= gc.mx || J >= gc.my) return;
  double acc = 0.0;
#pragma unroll
  for (int uz = -1; uz <= 1; ++uz) {
    const int z = fine_of(K, uz, gf.per & 4, gf.mz);
#pragma unroll
    for (int uy = -1; uy <= 1; ++uy) {
      const int y = fine_of(J, uy, gf.per & 2, gf.my);
#pragma unroll
      for (int ux = -1; ux <= 1; ++ux) {
        const int x = fine_of(I, ux, gf.per & 1, gf.mx);
        acc += (pw1(ux) * pw1(uy) * pw1(uz)) * rf[pidx(gf, x, y, z)];
      }
    }
  }
  rc[pidx(gc, I, J, K)] = acc * 0.125;
}

// One direction of the trilinear interpolation at fine unknown q: the coarse
// unknowns (ia, ib) and weights (wa, wb); a wall node gets weight 0.
__device__ __forceinline__ void interp1(int q, bool per, int mc, int& ia, int& ib, double& wa,
                                        double& wb) {
  const int G = q + (per ? 0 : 1);  // global fine node
  const int off = per ? 0 : 1;
  if ((G & 1) == 0) {
    ia = G / 2 - off;
    ib = ia;
    wa = 1.0;
    wb = 0.0;
  } else {
    ia = (G - 1) / 2 - off;
    ib = (G + 1) / 2 - off;
    wa = 0.5;
    wb = 0.5;
  }
  if (per) {
    ia = ia < 0 ? ia + mc : (ia >= mc ? ia - mc : ia);
    ib = ib < 0 ? ib + mc : (ib >= mc ? ib - mc : ib);
  } else {
    if (ia < 0 || ia >= mc) { wa = 0.0; ia = 0; }
    if (ib < 0 || ib >= mc) { wb = 0.0; ib = 0; }
  }
}

__global__ void __launch_bounds__(256)
    k_nd_interp_add(NdGeo gf, NdGeo gc, const double* __restrict__ ec, double* __restrict__ pf) {
  // lanes along x, gf.tz planes per work-group; every lane loads its 8
  // coarse values (a term of weight 0 reads a valid node and adds 0 exactly,
  // so neighbouring lanes of both parities take the same path)
  int tx, ty, tz;
  if (!nd_tile(nd_ntx(gf), nd_nty(gf), nd_ntz(gf), tx, ty, tz)) return;
  const int x = tx * 64 + threadIdx.x;
  const int y = ty * 4 + threadIdx.y;
  const int z0 = tz * gf.tz;
  if (x >= gf.mx || y >= gf.my) return;
  int ix[2], iy[2];
  double wx[2], wy[2];
  interp1(x, gf.per & 1, gc.mx, ix[0], ix[1], wx[0], wx[1]);
  interp1(y, gf.per & 2, gc.my, iy[0], iy[1], wy[0], wy[1]);
  const int z1 = min(z0 + gf.tz, gf.mz);
  for (int z = z0; z < z1; ++z) {
    int iz[2];
    double wz[2];
    interp1(z, gf.per & 4, gc.mz, iz[0], iz[1], wz[0], wz[1]);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a)
          acc += (wx[a] * wy[b] * wz[c]) * ec[pidx(gc, ix[a], iy[b], iz[c])];
    pf[pidx(gf, x, y, z)] += acc;
  }
}

// Ghosts of direction d from the opposite valid layer; grid covers the
// padded extent of the other two directions.
__global__ void __launch_bounds__(256) k_nd_fill_ghosts(NdGeo g, double* a, int d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int pz = g.mz + 2;
  int n1, n2;
  if (d == 0) { n1 = g.py; n2 = pz; }
  else if (d == 1) { n1 = g.px; n2 = pz; }
  else { n1 = g.px; n2 = g.py; }
  if (i >= n1 * n2) return;
  const int p = i % n1, q = i / n1;
  const int m = d == 0 ? g.mx : (d == 1 ? g.my : g.mz);
  auto at = [&](int t) -> int {
    // padded coordinates: t along d, (p, q) along the others
    if (d == 0) return t + g.px * (p + g.py * q);
    if (d == 1) return p + g.px * (t + g.py * q);
    return p + g.px * (q + g.py * t);
  };
  a[at(0)] = a[at(m)];
  a[at(m + 1)] = a[at(1)];
}

// Galerkin product: for coarse node (I, J, K) and each stored offset o,
// 1/8 sum_u r(u) sum_v W_f(2I + u, v) P(u + v - 2o).  FROM_SIGMA: W_f from
// the finest level's cells; else from the finer level's stored couplings.
template <bool FROM_SIGMA>
__global__ void __launch_bounds__(256)
    k_nd_rap(NdGeo gf, NdGeo gc, NdKappa kap, const double* __restrict__ sig, NdStencilC in,
             NdStencil out) {
  const int I = blockIdx.x * 64 + threadIdx.x;
  const int J = blockIdx.y * 4 + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= gc.mx || J >= gc.my || K >= gc.mz) return;
  double acc[kNdStored];
#pragma unroll
  for (int q = 0; q < kNdStored; ++q) acc[q] = 0.0;
  const int sx = gf.mx + 1, sy = gf.my + 1;
  for (int u = 0; u < 27; ++u) {
    const int ux = u % 3 - 1, uy = (u / 3) % 3 - 1, uz = u / 9 - 1;
    const int x = fine_of(I, ux, gf.per & 1, gf.mx);
    const int y = fine_of(J, uy, gf.per & 2, gf.my);
    const int z = fine_of(K, uz, gf.per & 4, gf.mz);
    const double ru = pw1(ux) * pw1(uy) * pw1(uz);
    // the fine node's 27 couplings W[v], v = (vx, vy, vz) + 1 indexed vz*9 + vy*3 + vx
    double W[27];
    if (FROM_SIGMA) {
      double S[2][2][2];
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx)
            S[cz][cy][cx] = sig[(x + cx) + sx * ((y + cy) + sy * (z + cz))];
#pragma unroll
      for (int v = 0; v < 27; ++v) {
        const int vx = v % 3 - 1, vy = (v / 3) % 3 - 1, vz = v / 9 - 1;
        // cells holding both the node and node + v: s_d = 0 for v_d = -1,
        // 1 for v_d = 1, either for v_d = 0
        double ss = 0.0;
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
          for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
              const bool ok = (vx == 0 || vx == 2 * cx - 1) && (vy == 0 || vy == 2 * cy - 1) &&
                              (vz == 0 || vz == 2 * cz - 1);
              if (ok) ss += S[cz][cy][cx];
            }
        const int pat = (vx != 0 ? 1 : 0) | (vy != 0 ? 2 : 0) | (vz != 0 ? 4 : 0);
        W[v] = kap.k[pat] * ss;
      }
    } else {
      const int c = pidx(gf, x, y, z);
#pragma unroll
      for (int q = 0; q < kNdStored; ++q) {
        const int vx = kUp[q][0], vy = kUp[q][1], vz = kUp[q][2];
        const int d = vx + gf.px * (vy + gf.py * vz);
        W[(vz + 1) * 9 + (vy + 1) * 3 + (vx + 1)] = in.w[q][c];
        if (q > 0) W[(1 - vz) * 9 + (1 - vy) * 3 + (1 - vx)] = in.w[q][c - d];
      }
    }
#pragma unroll
    for (int q = 0; q < kNdStored; ++q) {
      const int ox = kUp[q][0], oy = kUp[q][1], oz = kUp[q][2];
      double t = 0.0;
#pragma unroll
      for (int v = 0; v < 27; ++v) {
        const int vx = v % 3 - 1, vy = (v / 3) % 3 - 1, vz = v / 9 - 1;
        const double p = pw1(ux + vx - 2 * ox) * pw1(uy + vy - 2 * oy) * pw1(uz + vz - 2 * oz);
        t += p * W[v];
      }
      acc[q] += ru * t;
    }
  }
  const int c = pidx(gc, I, J, K);
#pragma unroll
  for (int q = 0; q < kNdStored; ++q) out.w[q][c] = acc[q] * 0.125;
}

// Block-wide sum in FP64 (all threads get the result).
__device__ double nd_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// q = A p on the bottom level (wrapped neighbours; walls skipped).
__device__ double nd_apply_at(const NdGeo& g, const NdStencilC& s, const double* p, int ux, int uy,
                              int uz) {
  const int c = pidx(g, ux, uy, uz);
  double ap = s.w[0][c] * p[c];
  for (int q = 1; q < kNdStored; ++q) {
    const int d = kUp[q][0] + g.px * (kUp[q][1] + g.py * kUp[q][2]);
    ap += s.w[q][c] * p[c + d];
    ap += s.w[q][c - d] * p[c - d];
  }
  return ap;
}

// Whole CG in one work-group of 1024 lanes.  x, r, p, q live in padded
// arrays whose ghosts the work-group keeps wrapped (periodic) or 0 (walls).
__global__ void __launch_bounds__(1024)
    k_nd_bottom_cg(NdGeo g, NdStencilC s, const double* __restrict__ rhs, double* x, double* r,
                   double* p, double* q, double tol, int maxit, int singular, int* iters) {
  __shared__ double red[16];
  const int n = g.mx * g.my * g.mz;
  const int tid = threadIdx.x, nt = blockDim.x;
  auto node = [&](int i, int& ux, int& uy, int& uz) {
    ux = i % g.mx;
    uy = (i / g.mx) % g.my;
    uz = i / (g.mx * g.my);
  };
  auto wrap_fill = [&](double* a) {
    // ghosts along periodic directions, one direction after the other
    for (int d = 0; d < 3; ++d) {
      if (!(g.per & (1 << d))) continue;
      __syncthreads();
      const int pz = g.mz + 2;
      const int n1 = d == 0 ? g.py : g.px;
      const int n2 = d == 2 ? g.py : pz;
      const int m = d == 0 ? g.mx : (d == 1 ? g.my : g.mz);
      for (int i = tid; i < n1 * n2; i += nt) {
        const int pp = i % n1, qq = i / n1;
        int lo, hi, slo, shi;
        if (d == 0) {
          lo = 0 + g.px * (pp + g.py * qq);
          hi = (m + 1) + g.px * (pp + g.py * qq);
          slo = m + g.px * (pp + g.py * qq);
          shi = 1 + g.px * (pp + g.py * qq);
        } else if (d == 1) {
          lo = pp + g.px * (0 + g.py * qq);
          hi = pp + g.px * ((m + 1) + g.py * qq);
          slo = pp + g.px * (m + g.py * qq);
          shi = pp + g.px * (1 + g.py * qq);
        } else {
          lo = pp + g.px * (qq + g.py * 0);
          hi = pp + g.px * (qq + g.py * (m + 1));
          slo = pp + g.px * (qq + g.py * m);
          shi = pp + g.px * (qq + g.py * 1);
        }
        a[lo] = a[slo];
        a[hi] = a[shi];
      }
    }
    __syncthreads();
  };
  // b = rhs (mean removed when singular); x = 0; r = p = b
  double mean = 0.0;
  if (singular) {
    double sm = 0.0;
    for (int i = tid; i < n; i += nt) {
      int ux, uy, uz;
      node(i, ux, uy, uz);
      sm += rhs[pidx(g, ux, uy, uz)];
    }
    mean = nd_block_sum(sm, red) / n;
  }
  double bb = 0.0;
  for (int i = tid; i < n; i += nt) {
    int ux, uy, uz;
    node(i, ux, uy, uz);
    const int c = pidx(g, ux, uy, uz);
    const double b = rhs[c] - mean;
    x[c] = 0.0;
    r[c] = b;
    p[c] = b;
    bb += b * b;
  }
  double rr = nd_block_sum(bb, red);
  const double nb = sqrt(rr);
  wrap_fill(p);
  int it = 0;
  while (nb > 0.0 && it < maxit && sqrt(rr) > tol * nb) {
    double pq = 0.0;
    for (int i = tid; i < n; i += nt) {
      int ux, uy, uz;
      node(i, ux, uy, uz);
      const int c = pidx(g, ux, uy, uz);
      const double v = nd_apply_at(g, s, p, ux, uy, uz);
      q[c] = v;
      pq += p[c] * v;
    }
    pq = nd_block_sum(pq, red);
    const double alpha = rr / pq;
    double rn = 0.0;
    for (int i = tid; i < n; i += nt) {
      int ux, uy, uz;
      node(i, ux, uy, uz);
      const int c = pidx(g, ux, uy, uz);
      x[c] += alpha * p[c];
      r[c] -= alpha * q[c];
      rn += r[c] * r[c];
    }
    rn = nd_block_sum(rn, red);
    const double beta = rn / rr;
    rr = rn;
    for (int i = tid; i < n; i += nt) {
      int ux, uy, uz;
      node(i, ux, uy, uz);
      const int c = pidx(g, ux, uy, uz);
      p[c] = r[c] + beta * p[c];
    }
    wrap_fill(p);
    ++it;
  }
  if (singular) {
    double sm = 0.0;
    for (int i = tid; i < n; i += nt) {
      int ux, uy, uz;
      node(i, ux, uy, uz);
      sm += x[pidx(g, ux, uy, uz)];
    }
    const double mx = nd_block_sum(sm, red) / n;
    for (int i = tid; i < n; i += nt) {
      int ux, uy, uz;
      node(i, ux, uy, uz);
      x[pidx(g, ux, uy, uz)] -= mx;
    }
  }
  if (tid == 0) *iters = it;
}

__global__ void __launch_bounds__(256)
    k_nd_maxabs(NdGeo g, const double* __restrict__ v, unsigned long long* norm) {
  const int ux = blockIdx.x * 64 + threadIdx.x;
  const int uy = blockIdx.y * 4 + threadIdx.y;
  const int z0 = blockIdx.z * g.tz;
  unsigned long long mx = 0;
  if (ux < g.mx && uy < g.my) {
    const int z1 = min(z0 + g.tz, g.mz);
    for (int uz = z0; uz < z1; ++uz) {
      const unsigned long long b = absbits(v[pidx(g, ux, uy, uz)]);
      mx = b > mx ? b : mx;
    }
  }
  nd_block_max(mx, norm);
}

// Unknown index along d of global node G (relative to the domain), or -1 on
// a wall node; periodic directions wrap.
__device__ __forceinline__ int unknown_of(int G, int n, bool per) {
  if (per) return ((G % n) + n) % n;
  return (G <= 0 || G >= n) ? -1 : G - 1;
}

// grid.y = box; x covers the box's nodes (lo..hi+1 grown by ng)
__global__ void __launch_bounds__(256)
    k_nd_gather(NdGeo g, const NdBox* __restrict__ boxes, int ng, int3 dlo,
                const double* __restrict__ src, double* __restrict__ dst) {
  const NdBox B = boxes[blockIdx.y];
  const int nx = B.hi[0] - B.lo[0] + 2 + 2 * ng, ny = B.hi[1] - B.lo[1] + 2 + 2 * ng;
  const int nz = B.hi[2] - B.lo[2] + 2 + 2 * ng;
  const long long total = (long long)nx * ny * nz;
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += 256ll * gridDim.x) {
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((long long)nx * ny));
    // global node of this element; the box owns the nodes of its own cells
    const int G[3] = {B.lo[0] - ng + i, B.lo[1] - ng + j, B.lo[2] - ng + k};
    if (G[0] < B.lo[0] || G[0] > B.hi[0] || G[1] < B.lo[1] || G[1] > B.hi[1] || G[2] < B.lo[2] ||
        G[2] > B.hi[2])
      continue;
    const int u[3] = {G[0] - dlo.x - ((g.per & 1) ? 0 : 1), G[1] - dlo.y - ((g.per & 2) ? 0 : 1),
                      G[2] - dlo.z - ((g.per & 4) ? 0 : 1)};
    if (u[0] < 0 || u[1] < 0 || u[2] < 0) continue;  // wall node
    dst[pidx(g, u[0], u[1], u[2])] = src[B.off + e];
  }
}

__global__ void __launch_bounds__(256)
    k_nd_scatter(NdGeo g, const NdBox* __restrict__ boxes, int ng, int3 dlo, int3 dn,
                 const double* __restrict__ src, double* __restrict__ dst) {
  const NdBox B = boxes[blockIdx.y];
  const int nx = B.hi[0] - B.lo[0] + 2 + 2 * ng, ny = B.hi[1] - B.lo[1] + 2 + 2 * ng;
  const int nz = B.hi[2] - B.lo[2] + 2 + 2 * ng;
  const long long total = (long long)nx * ny * nz;
  const int n[3] = {dn.x, dn.y, dn.z};
  const int lo[3] = {dlo.x, dlo.y, dlo.z};
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += 256ll * gridDim.x) {
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((long long)nx * ny));
    const int G[3] = {B.lo[0] - ng + i - lo[0], B.lo[1] - ng + j - lo[1], B.lo[2] - ng + k - lo[2]};
    bool inside = true, wall = false;
    int u[3];
    for (int d = 0; d < 3; ++d) {
      const bool per = g.per & (1 << d);
      if (!per && (G[d] < 0 || G[d] > n[d])) inside = false;
      u[d] = unknown_of(G[d], n[d], per);
      if (u[d] < 0) wall = true;
    }
    if (!inside) continue;  // a ghost node beyond a wall keeps its value
    dst[B.off + e] = wall ? 0.0 : src[pidx(g, u[0], u[1], u[2])];
  }
}

// grid.y = box of the cell MultiFab (ng 0): sigma entry of each cell (and,
// along a periodic direction, the wrapped entry 0 from the last cell).
__global__ void __launch_bounds__(256)
    k_nd_sigma(NdGeo g, const NdBox* __restrict__ boxes, int3 dlo, int3 dn,
               const double* __restrict__ cells, double* __restrict__ sig) {
  const NdBox B = boxes[blockIdx.y];
  const int nx = B.hi[0] - B.lo[0] + 1, ny = B.hi[1] - B.lo[1] + 1, nz = B.hi[2] - B.lo[2] + 1;
  const long long total = (long long)nx * ny * nz;
  const int sx = g.mx + 1, sy = g.my + 1;
  const int n[3] = {dn.x, dn.y, dn.z};
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += 256ll * gridDim.x) {
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((long long)nx * ny));
    const int c[3] = {B.lo[0] + i - dlo.x, B.lo[1] + j - dlo.y, B.lo[2] + k - dlo.z};
    const double v = cells[B.off + e];
    // entry index: the cell itself on a Dirichlet direction, cell + 1 on a
    // periodic one (entry 0 holds the last cell)
    int a[3], nw = 1;
    int alt[3] = {-1, -1, -1};
    for (int d = 0; d < 3; ++d) {
      const bool per = g.per & (1 << d);
      a[d] = per ? c[d] + 1 : c[d];
      if (per && c[d] == n[d] - 1) alt[d] = 0;
    }
    // write every combination of the entry and its wrapped copy
    for (int m = 0; m < 8; ++m) {
      int q[3];
      bool ok = true;
      for (int d = 0; d < 3; ++d) {
        if (m & (1 << d)) {
          if (alt[d] < 0) ok = false;
          q[d] = alt[d];
        } else {
          q[d] = a[d];
        }
      }
      if (!ok) continue;
      sig[q[0] + sx * (q[1] + sy * q[2])] = v;
    }
    (void)nw;
  }
}

// Partial sums of the valid nodes, one per work-group (FP64, fixed order).
__global__ void __launch_bounds__(256)
    k_nd_sum_partials(NdGeo g, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double red[4];
  const int ux = blockIdx.x * 64 + threadIdx.x;
  const int uy = blockIdx.y * 4 + threadIdx.y;
  const int z0 = blockIdx.z * g.tz;
  double sm = 0.0;
  if (ux < g.mx && uy < g.my) {
    const int z1 = min(z0 + g.tz, g.mz);
    for (int uz = z0; uz < z1; ++uz) sm += v[pidx(g, ux, uy, uz)];
  }
  for (int o = 32; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
  if (threadIdx.x == 0) red[threadIdx.y] = sm;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0)
    part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] =
        (red[0] + red[1]) + (red[2] + red[3]);
}

// v -= (sum of the partials) / (number of unknowns) on every valid node; the
// partials are summed by every work-group in the same order.
__global__ void __launch_bounds__(256)
    k_nd_shift(NdGeo g, double* __restrict__ v, const double* __restrict__ part, int npart) {
  __shared__ double mean;
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    double s = 0.0;
    for (int i = 0; i < npart; ++i) s += part[i];
    mean = s / ((double)g.mx * g.my * g.mz);
  }
  __syncthreads();
  const int ux = blockIdx.x * 64 + threadIdx.x;
  const int uy = blockIdx.y * 4 + threadIdx.y;
  const int z0 = blockIdx.z * g.tz;
  if (ux < g.mx && uy < g.my) {
    const int z1 = min(z0 + g.tz, g.mz);
    for (int uz = z0; uz < z1; ++uz) v[pidx(g, ux, uy, uz)] -= mean;
  }
}

// Partial sums of a.b over the valid nodes, one per work-group.
__global__ void __launch_bounds__(256)
    k_nd_dot_partials(NdGeo g, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ part) {
  __shared__ double red[4];
  const int ux = blockIdx.x * 64 + threadIdx.x;
  const int uy = blockIdx.y * 4 + threadIdx.y;
  const int z0 = blockIdx.z * g.tz;
  double sm = 0.0;
  if (ux < g.mx && uy < g.my) {
    const int z1 = min(z0 + g.tz, g.mz);
    for (int uz = z0; uz < z1; ++uz) {
      const int c = pidx(g, ux, uy, uz);
      sm += a[c] * b[c];
    }
  }
  for (int o = 32; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
  if (threadIdx.x == 0) red[threadIdx.y] = sm;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0)
    part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] =
        (red[0] + red[1]) + (red[2] + red[3]);
}

// out = sum of n partials (one work-group, fixed order).
__global__ void __launch_bounds__(256)
    k_nd_sum_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[4];
  double sm = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) sm += part[i];
  for (int o = 32; o > 0; o >>= 1) sm += __shfl_xor(sm, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sm;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// p = z (restart) or z + (rho / rho_old) p.
__global__ void __launch_bounds__(256)
    k_nd_cg_p(NdGeo g, double* __restrict__ p, const double* __restrict__ z,
              const double* __restrict__ rho, const double* __restrict__ rho_old, int restart) {
  const int ux = blockIdx.x * 64 + threadIdx.x;
  const int uy = blockIdx.y * 4 + threadIdx.y;
  const int z0 = blockIdx.z * g.tz;
  if (ux >= g.mx || uy >= g.my) return;
  const double beta = restart ? 0.0 : *rho / *rho_old;
  const int z1 = min(z0 + g.tz, g.mz);
  for (int uz = z0; uz < z1; ++uz) {
    const int c = pidx(g, ux, uy, uz);
    p[c] = restart ? z[c] : z[c] + beta * p[c];
  }
}

// alpha = rho / pq; x += alpha p; r -= alpha q; max |r| into norm.
__global__ void __launch_bounds__(256)
    k_nd_cg_xr(NdGeo g, double* __restrict__ x, const double* __restrict__ p,
               double* __restrict__ r, const double* __restrict__ q,
               const double* __restrict__ rho, const double* __restrict__ pq,
               unsigned long long* norm) {
  const int ux = blockIdx.x * 64 + threadIdx.x;
  const int uy = blockIdx.y * 4 + threadIdx.y;
  const int z0 = blockIdx.z * g.tz;
  unsigned long long mx = 0;
  if (ux < g.mx && uy < g.my) {
    const double alpha = *rho / *pq;
    const int z1 = min(z0 + g.tz, g.mz);
    for (int uz = z0; uz < z1; ++uz) {
      const int c = pidx(g, ux, uy, uz);
      x[c] += alpha * p[c];
      const double rv = r[c] - alpha * q[c];
      r[c] = rv;
      const unsigned long long b = absbits(rv);
      mx = b > mx ? b : mx;
    }
  }
  nd_block_max(mx, norm);
}

__global__ void k_nd_fill(double* a, long long n, double v) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_nd_fill_u64(unsigned long long* a, int n, unsigned long long v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) a[i] = v;
}

dim3 sweep_grid(const NdGeo& g) {
  return dim3((g.mx + 63) / 64, (g.my + 3) / 4, (g.mz + g.tz - 1) / g.tz);
}
dim3 plane_grid(const NdGeo& g) { return dim3((g.mx + 63) / 64, (g.my + 3) / 4, g.mz); }
// 1-D grids of the XCD-grouped tile order (nd_tile)
dim3 xcd_grid(long long ntiles) {
  return dim3((unsigned)(kNdXcds * ((ntiles + kNdXcds - 1) / kNdXcds)));
}
dim3 sweep_grid_xcd(const NdGeo& g) {
  const dim3 t = sweep_grid(g);
  return xcd_grid((long long)t.x * t.y * t.z);
}
dim3 plane_grid_xcd(const NdGeo& g) {
  const dim3 t = plane_grid(g);
  return xcd_grid((long long)t.x * t.y * t.z);
}

}  // namespace

hipError_t nd_launch_sweep0(hipStream_t st, const NdGeo& g, const NdKappa& k, const double* sig,
                            const double* phi, const double* f, double* out, double omega,
                            int mode, unsigned long long* norm) {
  const dim3 b(64, 4);
#define L0(M, N) \
  hipLaunchKernelGGL((k_nd_sweep0<M, N>), sweep_grid_xcd(g), b, 0, st, g, k, sig, phi, f, out, omega, norm)
  if (mode == ND_ZERO) L0(ND_ZERO, false);
  else if (mode == ND_APPLY) L0(ND_APPLY, false);
  else if (mode == ND_RESID) { if (norm) L0(ND_RESID, true); else L0(ND_RESID, false); }
  else { if (norm) L0(ND_JACOBI, true); else L0(ND_JACOBI, false); }
#undef L0
  return hipGetLastError();
}

hipError_t nd_launch_sweep_st(hipStream_t st, const NdGeo& g, const NdStencilC& s,
                              const double* phi, const double* f, double* out, double omega,
                              int mode, unsigned long long* norm) {
  const dim3 b(64, 4);
#define LS(M, N) \
  hipLaunchKernelGGL((k_nd_sweep_st<M, N>), sweep_grid_xcd(g), b, 0, st, g, s, phi, f, out, omega, norm)
  if (mode == ND_ZERO) LS(ND_ZERO, false);
  else if (mode == ND_APPLY) LS(ND_APPLY, false);
  else if (mode == ND_RESID) { if (norm) LS(ND_RESID, true); else LS(ND_RESID, false); }
  else { if (norm) LS(ND_JACOBI, true); else LS(ND_JACOBI, false); }
#undef LS
  return hipGetLastError();
}

hipError_t nd_launch_restrict(hipStream_t st, const NdGeo& gf, const NdGeo& gc, const double* rf,
                              double* rc) {
  hipLaunchKernelGGL(k_nd_restrict, plane_grid_xcd(gc), dim3(64, 4), 0, st, gf, gc, rf, rc);
  return hipGetLastError();
}

hipError_t nd_launch_interp_add(hipStream_t st, const NdGeo& gf, const NdGeo& gc,
                                const double* ec, double* phif) {
  hipLaunchKernelGGL(k_nd_interp_add, sweep_grid_xcd(gf), dim3(64, 4), 0, st, gf, gc, ec, phif);
  return hipGetLastError();
}

hipError_t nd_launch_fill_ghosts(hipStream_t st, const NdGeo& g, double* a) {
  for (int d = 0; d < 3; ++d) {
    if (!(g.per & (1 << d))) continue;
    const int pz = g.mz + 2;
    const int n = d == 0 ? g.py * pz : (d == 1 ? g.px * pz : g.px * g.py);
    hipLaunchKernelGGL(k_nd_fill_ghosts, dim3((n + 255) / 256), dim3(256), 0, st, g, a, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t nd_launch_rap0(hipStream_t st, const NdGeo& gf, const NdGeo& gc, const NdKappa& k,
                          const double* sig, const NdStencil& out) {
  NdStencilC none{};
  hipLaunchKernelGGL(k_nd_rap<true>, plane_grid(gc), dim3(64, 4), 0, st, gf, gc, k, sig, none,
                     out);
  return hipGetLastError();
}

hipError_t nd_launch_rap(hipStream_t st, const NdGeo& gf, const NdGeo& gc, const NdStencilC& in,
                         const NdStencil& out) {
  NdKappa k{};
  hipLaunchKernelGGL(k_nd_rap<false>, plane_grid(gc), dim3(64, 4), 0, st, gf, gc, k, nullptr, in,
                     out);
  return hipGetLastError();
}

hipError_t nd_launch_bottom_cg(hipStream_t st, const NdGeo& g, const NdStencilC& s,
                               const double* rhs, double* x, double* work, double tol, int maxit,
                               int singular, int* iters) {
  const long long sz = (long long)g.px * g.py * (g.mz + 2);
  hipLaunchKernelGGL(k_nd_bottom_cg, dim3(1), dim3(1024), 0, st, g, s, rhs, x, work,
                     work + sz, work + 2 * sz, tol, maxit, singular, iters);
  return hipGetLastError();
}

hipError_t nd_launch_maxabs(hipStream_t st, const NdGeo& g, const double* v,
                            unsigned long long* norm) {
  hipLaunchKernelGGL(k_nd_maxabs, sweep_grid(g), dim3(64, 4), 0, st, g, v, norm);
  return hipGetLastError();
}

hipError_t nd_launch_gather(hipStream_t st, const NdGeo& g, const NdBox* boxes, int nbox,
                            int maxnodes, int ng, const int dom_lo[3], const double* src,
                            double* dst) {
  if (nbox <= 0) return hipSuccess;
  int gx = (maxnodes + 255) / 256;
  gx = gx < 1 ? 1 : (gx > 4096 ? 4096 : gx);
  hipLaunchKernelGGL(k_nd_gather, dim3(gx, nbox), dim3(256), 0, st, g, boxes, ng,
                     make_int3(dom_lo[0], dom_lo[1], dom_lo[2]), src, dst);
  return hipGetLastError();
}

hipError_t nd_launch_scatter(hipStream_t st, const NdGeo& g, const NdBox* boxes, int nbox,
                             int maxnodes, int ng, const int dom_lo[3], const int dom_n[3],
                             const double* src, double* dst) {
  if (nbox <= 0) return hipSuccess;
  int gx = (maxnodes + 255) / 256;
  gx = gx < 1 ? 1 : (gx > 4096 ? 4096 : gx);
  hipLaunchKernelGGL(k_nd_scatter, dim3(gx, nbox), dim3(256), 0, st, g, boxes, ng,
                     make_int3(dom_lo[0], dom_lo[1], dom_lo[2]),
                     make_int3(dom_n[0], dom_n[1], dom_n[2]), src, dst);
  return hipGetLastError();
}

hipError_t nd_launch_sigma(hipStream_t st, const NdGeo& g, const NdBox* boxes, int nbox,
                           int maxcells, const int dom_lo[3], const int dom_n[3],
                           const double* cells, double* sig) {
  if (nbox <= 0) return hipSuccess;
  int gx = (maxcells + 255) / 256;
  gx = gx < 1 ? 1 : (gx > 4096 ? 4096 : gx);
  hipLaunchKernelGGL(k_nd_sigma, dim3(gx, nbox), dim3(256), 0, st, g, boxes,
                     make_int3(dom_lo[0], dom_lo[1], dom_lo[2]),
                     make_int3(dom_n[0], dom_n[1], dom_n[2]), cells, sig);
  return hipGetLastError();
}

int nd_sum_partials_count(const NdGeo& g) {
  const dim3 gr = sweep_grid(g);
  return (int)(gr.x * gr.y * gr.z);
}

hipError_t nd_launch_remove_mean(hipStream_t st, const NdGeo& g, double* v, double* part) {
  hipLaunchKernelGGL(k_nd_sum_partials, sweep_grid(g), dim3(64, 4), 0, st, g, v, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nd_shift, sweep_grid(g), dim3(64, 4), 0, st, g, v, part,
                     nd_sum_partials_count(g));
  return hipGetLastError();
}

hipError_t nd_launch_dot(hipStream_t st, const NdGeo& g, const double* a, const double* b,
                         double* part, double* out) {
  hipLaunchKernelGGL(k_nd_dot_partials, sweep_grid(g), dim3(64, 4), 0, st, g, a, b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nd_sum_final, dim3(1), dim3(256), 0, st, part, nd_sum_partials_count(g),
                     out);
  return hipGetLastError();
}

hipError_t nd_launch_cg_p(hipStream_t st, const NdGeo& g, double* p, const double* z,
                          const double* rho, const double* rho_old, int restart) {
  hipLaunchKernelGGL(k_nd_cg_p, sweep_grid(g), dim3(64, 4), 0, st, g, p, z, rho, rho_old,
                     restart);
  return hipGetLastError();
}

hipError_t nd_launch_cg_xr(hipStream_t st, const NdGeo& g, double* x, const double* p, double* r,
                           const double* q, const double* rho, const double* pq,
                           unsigned long long* norm) {
  hipLaunchKernelGGL(k_nd_cg_xr, sweep_grid(g), dim3(64, 4), 0, st, g, x, p, r, q, rho, pq, norm);
  return hipGetLastError();
}

hipError_t nd_launch_fill(hipStream_t st, double* a, long long n, double v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nd_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, v);
  return hipGetLastError();
}

hipError_t nd_launch_fill_u64(hipStream_t st, unsigned long long* a, int n,
                              unsigned long long v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nd_fill_u64, dim3((n + 255) / 256), dim3(256), 0, st, a, n, v);
  return hipGetLastError();
}

}  // namespace amrmg
