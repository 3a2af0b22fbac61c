// Grid transfer steps of Sec. II.B and the final assembly:
//   anterpolation   q^1[mu] = sum_j phi^1_mu(x_j) xi_j            (eq:anterpolation)
//   restriction     q^k[M]  = sum_nu q^{k-1}[nu] phi^k_M(x^{k-1}_nu),  k = 2..l
//   prolongation    E^k[nu] = e^k[nu] + sum_M phi^{k+1}_M(x^k_nu) E^{k+1}[M]
//   interpolation   u_i = e^0_i + sum_mu phi^1_mu(x_i) E^1[mu]    (eq:interpolation)
// with the tensor-product basis phi of eq:def-phi on periodic grids whose
// level-k spacing is 2^(k-1) h_1, and the energy
//   E = -1/2 [ sum_i xi_i u_i - gamma(0) a^-6 sum_i xi_i^2 ]
// (eq:interpolation-pot with the self-interaction energy of
// eq:self-interaction-energy removed; E = -V in the paper's notation).
// Forces are the exact gradient: F_i = F^loc_i + xi_i sum_mu grad phi^1_mu(x_i) E^1[mu].
#include <algorithm>

#include "device_math.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

struct GridGeom {
  int n[3];
  double invh[3];
};

// ------------------------------------------------------------ anterpolation
template <int P>
__global__ void __launch_bounds__(kBlock) k_anterp_f64(const double4* __restrict__ xs, int n, GridGeom gg,
                                                       double* __restrict__ q) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double4 p = xs[s];
  const double pc[3] = {p.x, p.y, p.z};
  double w[3][P];
  int idx[3][P];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double t = pc[d] * gg.invh[d];
    const double m0 = floor(t);
    basis_weights<P, double>(t - m0, w[d]);
    const int base = (int)m0 - (P / 2 - 1);
#pragma unroll
    for (int j = 0; j < P; ++j) idx[d][j] = wrapi(base + j, gg.n[d]);
  }
#pragma unroll
  for (int jz = 0; jz < P; ++jz)
#pragma unroll
    for (int jy = 0; jy < P; ++jy) {
      const double wzy = p.w * w[2][jz] * w[1][jy];
      double* row = q + ((size_t)idx[2][jz] * gg.n[1] + idx[1][jy]) * gg.n[0];
#pragma unroll
      for (int jx = 0; jx < P; ++jx) unsafeAtomicAdd(row + idx[0][jx], wzy * w[0][jx]);
    }
}

// Owner-computes anterpolation: a block owns the finest-grid points whose
// positions fall inside a box of CBx x CBy x CBz linked cells (point m of
// dimension d belongs to cell-block b when ceil(c0 n/nc) <= m < ceil(c1 n/nc)).
// It gathers the atoms of those cells and of an nh-cell halo (with their
// periodic image shifts), adds each atom's p^3 contributions that land on
// owned points into an LDS tile, and stores the tile without global atomics.
constexpr int kAntTile = 16;     // max owned points per dimension
constexpr int kAntThreads = 256;
constexpr int kMaxSeg = 1024;

struct AntGeom {
  int cb[3];   // cells per block and dimension
  int nb[3];   // blocks per dimension
  int nh[3];   // halo cells
};

template <int P, class W>
__global__ void __launch_bounds__(kAntThreads) k_anterp_owned(const double4* __restrict__ xs,
                                                              const int* __restrict__ cstart, CellGeom cg,
                                                              GridGeom gg, AntGeom ag, double* __restrict__ q) {
  __shared__ double tile[kAntTile * kAntTile * kAntTile];
  __shared__ int seg_begin[kMaxSeg];
  __shared__ int seg_off[kMaxSeg + 1];
  __shared__ int seg_shift[kMaxSeg][3];
  __shared__ int nseg_s;
  const int b = blockIdx.x;
  const int bi[3] = {b % ag.nb[0], (b / ag.nb[0]) % ag.nb[1], b / (ag.nb[0] * ag.nb[1])};
  int c0[3], c1[3], lo[3], wd[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c0[d] = bi[d] * ag.cb[d];
    c1[d] = min(c0[d] + ag.cb[d], cg.nc[d]);
    lo[d] = (c0[d] * gg.n[d] + cg.nc[d] - 1) / cg.nc[d];
    wd[d] = (c1[d] * gg.n[d] + cg.nc[d] - 1) / cg.nc[d] - lo[d];
  }
  for (int i = threadIdx.x; i < kAntTile * kAntTile * kAntTile; i += kAntThreads) tile[i] = 0.0;
  if (threadIdx.x == 0) {
    // contiguous runs of sorted atoms: rows of cells along x, split where the
    // periodic image changes
    int ns = 0, tot = 0;
    for (int cz = c0[2] - ag.nh[2]; cz < c1[2] + ag.nh[2]; ++cz) {
      const int iz = floordiv(cz, cg.nc[2]);
      const int wz = cz - iz * cg.nc[2];
      for (int cy = c0[1] - ag.nh[1]; cy < c1[1] + ag.nh[1]; ++cy) {
        const int iy = floordiv(cy, cg.nc[1]);
        const int wy = cy - iy * cg.nc[1];
        const int rowc = (wz * cg.nc[1] + wy) * cg.nc[0];
        int cx = c0[0] - ag.nh[0];
        const int cxe = c1[0] + ag.nh[0];
        while (cx < cxe) {
          const int ix = floordiv(cx, cg.nc[0]);
          const int wx = cx - ix * cg.nc[0];
          const int run = min(cxe - cx, cg.nc[0] - wx);
          const int a0 = cstart[rowc + wx], a1 = cstart[rowc + wx + run];
          if (a1 > a0 && ns < kMaxSeg) {
            seg_begin[ns] = a0;
            seg_off[ns] = tot;
            seg_shift[ns][0] = ix;
            seg_shift[ns][1] = iy;
            seg_shift[ns][2] = iz;
            tot += a1 - a0;
            ++ns;
          }
          cx += run;
        }
      }
    }
    seg_off[ns] = tot;
    nseg_s = ns;
  }
  __syncthreads();
  const int ns = nseg_s;
  const int tot = seg_off[ns];
  int sg = 0;
  for (int i = threadIdx.x; i < tot; i += kAntThreads) {
    while (seg_off[sg + 1] <= i) ++sg;
    const double4 p = xs[seg_begin[sg] + (i - seg_off[sg])];
    const double pc[3] = {p.x, p.y, p.z};
    W w[3][P];
    int l0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double t = pc[d] * gg.invh[d];
      const double m0 = floor(t);
      basis_weights<P, W>((W)(t - m0), w[d]);
      l0[d] = (int)m0 - (P / 2 - 1) + seg_shift[sg][d] * gg.n[d] - lo[d];
    }
    const W xiw = (W)p.w;
#pragma unroll
    for (int jz = 0; jz < P; ++jz) {
      const int lz = l0[2] + jz;
      if (lz < 0 || lz >= wd[2]) continue;
#pragma unroll
      for (int jy = 0; jy < P; ++jy) {
        const int ly = l0[1] + jy;
        if (ly < 0 || ly >= wd[1]) continue;
        const W wzy = xiw * w[2][jz] * w[1][jy];
        double* row = tile + (lz * kAntTile + ly) * kAntTile;
#pragma unroll
        for (int jx = 0; jx < P; ++jx) {
          const int lx = l0[0] + jx;
          // charges accumulate in FP64 whatever the weight precision
          if (lx >= 0 && lx < wd[0]) atomicAdd(row + lx, (double)(wzy * w[0][jx]));
        }
      }
    }
  }
  __syncthreads();
  const int cnt = wd[0] * wd[1] * wd[2];
  for (int i = threadIdx.x; i < cnt; i += kAntThreads) {
    const int lx = i % wd[0], ly = (i / wd[0]) % wd[1], lz = i / (wd[0] * wd[1]);
    q[((size_t)(lo[2] + lz) * gg.n[1] + (lo[1] + ly)) * gg.n[0] + lo[0] + lx] =
        tile[(lz * kAntTile + ly) * kAntTile + lx];
  }
}

// ------------------------------------------------------------ restriction
// Per-dimension taps around fine index 2M: offsets 0, +-1, +-3 (, +-5).
template <int P>
__global__ void __launch_bounds__(kBlock) k_restrict_f64(const double* __restrict__ qf, GridDims f,
                                                         double* __restrict__ qc, GridDims c) {
  const int M = blockIdx.x * blockDim.x + threadIdx.x;
  if (M >= c.size) return;
  const int X = M % c.n[0], Y = (M / c.n[0]) % c.n[1], Z = M / (c.n[0] * c.n[1]);
  constexpr int K = P + 1;  // 0, +-1, +-3, (+-5)
  int ix[K], iy[K], iz[K];
  double w[K];
  w[0] = 1.0;
  ix[0] = wrapi(2 * X, f.n[0]);
  iy[0] = wrapi(2 * Y, f.n[1]);
  iz[0] = wrapi(2 * Z, f.n[2]);
#pragma unroll
  for (int k = 0; k < P / 2; ++k) {
    const int o = 2 * k + 1;
    w[1 + 2 * k] = w[2 + 2 * k] = rp_weight_odd<P>(k);
    ix[1 + 2 * k] = wrapi(2 * X - o, f.n[0]);
    ix[2 + 2 * k] = wrapi(2 * X + o, f.n[0]);
    iy[1 + 2 * k] = wrapi(2 * Y - o, f.n[1]);
    iy[2 + 2 * k] = wrapi(2 * Y + o, f.n[1]);
    iz[1 + 2 * k] = wrapi(2 * Z - o, f.n[2]);
    iz[2 + 2 * k] = wrapi(2 * Z + o, f.n[2]);
  }
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < K; ++a) {
    double sy = 0.0;
#pragma unroll
    for (int b = 0; b < K; ++b) {
      const double* row = qf + ((size_t)iz[a] * f.n[1] + iy[b]) * f.n[0];
      double sx = 0.0;
#pragma unroll
      for (int cc = 0; cc < K; ++cc) sx += w[cc] * row[ix[cc]];
      sy += w[b] * sx;
    }
    acc += w[a] * sy;
  }
  qc[M] = acc;
}

// ------------------------------------------------------------ prolongation
// Fine index j receives coarse M with j - 2M in {0} (j even) or the odd
// offsets +-1, +-3 (, +-5) (j odd).
template <int P>
__device__ __forceinline__ int prolong_taps(int j, int nc, int* idx, double* w) {
  if ((j & 1) == 0) {
    idx[0] = wrapi(j >> 1, nc);
    w[0] = 1.0;
    return 1;
  }
#pragma unroll
  for (int k = 0; k < P / 2; ++k) {
    const int o = 2 * k + 1;
    idx[2 * k] = wrapi((j - o) >> 1, nc);
    idx[2 * k + 1] = wrapi((j + o) >> 1, nc);
    w[2 * k] = w[2 * k + 1] = rp_weight_odd<P>(k);
  }
  return P;
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_prolong_f64(const double* __restrict__ Ec, GridDims c,
                                                        const double* __restrict__ ef, double* __restrict__ Ef,
                                                        GridDims f) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= f.size) return;
  const int x = J % f.n[0], y = (J / f.n[0]) % f.n[1], z = J / (f.n[0] * f.n[1]);
  int ix[P], iy[P], iz[P];
  double wx[P], wy[P], wz[P];
  const int nx = prolong_taps<P>(x, c.n[0], ix, wx);
  const int ny = prolong_taps<P>(y, c.n[1], iy, wy);
  const int nz = prolong_taps<P>(z, c.n[2], iz, wz);
  double acc = 0.0;
  for (int a = 0; a < nz; ++a) {
    double sy = 0.0;
    for (int b = 0; b < ny; ++b) {
      const double* row = Ec + ((size_t)iz[a] * c.n[1] + iy[b]) * c.n[0];
      double sx = 0.0;
      for (int cc = 0; cc < nx; ++cc) sx += wx[cc] * row[ix[cc]];
      sy += wy[b] * sx;
    }
    acc += wz[a] * sy;
  }
  Ef[J] = ef[J] + acc;
}

// ------------------------------------------------------------ interpolation + assembly
struct OutPtrs {
  double* forces;
  double* potential;
  double* dE_dc6;
};

template <int P, class W>
__global__ void __launch_bounds__(kBlock) k_interp_f64(const double4* __restrict__ xs, const int* __restrict__ perm,
                                                       int n, GridGeom gg, const double* __restrict__ E1,
                                                       const double* __restrict__ e0, const double* __restrict__ floc,
                                                       double cself, OutPtrs out, double* __restrict__ partial) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double su = 0.0, sxx = 0.0;
  if (s < n) {
    const double4 p = xs[s];
    const double pc[3] = {p.x, p.y, p.z};
    W w[3][P], dw[3][P];
    int idx[3][P];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double t = pc[d] * gg.invh[d];
      const double m0 = floor(t);
      basis_weights_d<P, W>((W)(t - m0), w[d], dw[d]);
      const int base = (int)m0 - (P / 2 - 1);
#pragma unroll
      for (int j = 0; j < P; ++j) idx[d][j] = wrapi(base + j, gg.n[d]);
    }
    double u = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int jz = 0; jz < P; ++jz) {
      double ru = 0.0, rgx = 0.0, rgy = 0.0;
#pragma unroll
      for (int jy = 0; jy < P; ++jy) {
        const double* row = E1 + ((size_t)idx[2][jz] * gg.n[1] + idx[1][jy]) * gg.n[0];
        double v = 0.0, vd = 0.0;
#pragma unroll
        for (int jx = 0; jx < P; ++jx) {
          const double e = row[idx[0][jx]];
          v += (double)w[0][jx] * e;
          vd += (double)dw[0][jx] * e;
        }
        ru += (double)w[1][jy] * v;
        rgx += (double)w[1][jy] * vd;
        rgy += (double)dw[1][jy] * v;
      }
      u += (double)w[2][jz] * ru;
      gx += (double)w[2][jz] * rgx;
      gy += (double)w[2][jz] * rgy;
      gz += (double)dw[2][jz] * ru;
    }
    const int i = perm[s];
    const double xi = p.w;
    const double utot = e0[s] + u;
    if (out.forces) {
      out.forces[3 * (size_t)i + 0] = floc[3 * (size_t)s + 0] + xi * gx * gg.invh[0];
      out.forces[3 * (size_t)i + 1] = floc[3 * (size_t)s + 1] + xi * gy * gg.invh[1];
      out.forces[3 * (size_t)i + 2] = floc[3 * (size_t)s + 2] + xi * gz * gg.invh[2];
    }
    if (out.potential) out.potential[i] = utot;
    if (out.dE_dc6) out.dE_dc6[i] = -(utot - cself * xi) / (2.0 * xi);
    su = xi * utot;
    sxx = xi * xi;
  }
  // block reduction of sum xi u and sum xi^2 (fixed order: deterministic)
  __shared__ double r1[kBlock], r2[kBlock];
  r1[threadIdx.x] = su;
  r2[threadIdx.x] = sxx;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      r1[threadIdx.x] += r1[threadIdx.x + off];
      r2[threadIdx.x] += r2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = r1[0];
    partial[2 * blockIdx.x + 1] = r2[0];
  }
}

__global__ void __launch_bounds__(kBlock) k_energy_final(const double* __restrict__ partial, int nb, double cself,
                                                         double* __restrict__ energy) {
  __shared__ double r1[kBlock], r2[kBlock];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      r1[threadIdx.x] += r1[threadIdx.x + off];
      r2[threadIdx.x] += r2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *energy = -0.5 * (r1[0] - cself * r2[0]);
}

// ------------------------------------------------------------ stage copies
__global__ void k_scatter_atoms(const int* __restrict__ perm, int n, const double* __restrict__ src, int width,
                                double* __restrict__ dst) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
  for (int c = 0; c < width; ++c) dst[(size_t)i * width + c] = src[(size_t)s * width + c];
}

inline int nblocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

GridGeom finest_geom(const mls_plan_s* P) {
  GridGeom gg;
  for (int d = 0; d < 3; ++d) {
    gg.n[d] = P->lv[0].g.n[d];
    gg.invh[d] = P->invh1[d];
  }
  return gg;
}

}  // namespace

// Owner-computes geometry: cells per block so that a block owns at most
// kAntTile points per dimension, halo cells covering the basis support.
bool anterp_owned_geom(const mls_plan_s* P, AntGeom& ag) {
  const int half = P->order / 2;
  int segs = 1;
  for (int d = 0; d < 3; ++d) {
    const int n = P->lv[0].g.n[d], nc = P->cg.nc[d];
    // owned width of cb cells <= ceil(cb n / nc) <= kAntTile
    int cb = 0;
    while (cb < nc && ((cb + 1) * (int64_t)n + nc - 1) / nc <= kAntTile) ++cb;
    if (cb == 0) return false;
    ag.cb[d] = cb;
    ag.nb[d] = (nc + cb - 1) / cb;
    // atoms within (half + 1) grid spacings of the owned range
    ag.nh[d] = (int)(((int64_t)(half + 1) * nc + n - 1) / n);
    const int span = cb + 2 * ag.nh[d];
    // rows along x split at every periodic wrap
    segs *= (d == 0 ? std::min(span, (span + nc - 1) / nc + 1) : span);
  }
  return segs <= kMaxSeg;
}

hipError_t launch_anterpolate(mls_plan_s* P, int n, hipStream_t s) {
  Level& L1 = P->lv[0];
  GridGeom gg = finest_geom(P);
  AntGeom ag;
  if (anterp_owned_geom(P, ag)) {
    // every owned point is written, so no zero fill is needed
    const int nb = ag.nb[0] * ag.nb[1] * ag.nb[2];
    const bool mixed = P->precision == MLS_MIXED;
    if (P->order == 4 && !mixed)
      k_anterp_owned<4, double><<<nb, kAntThreads, 0, s>>>(P->d_xs, P->d_cell_start, P->cg, gg, ag, L1.q);
    else if (P->order == 4)
      k_anterp_owned<4, float><<<nb, kAntThreads, 0, s>>>(P->d_xs, P->d_cell_start, P->cg, gg, ag, L1.q);
    else if (!mixed)
      k_anterp_owned<6, double><<<nb, kAntThreads, 0, s>>>(P->d_xs, P->d_cell_start, P->cg, gg, ag, L1.q);
    else
      k_anterp_owned<6, float><<<nb, kAntThreads, 0, s>>>(P->d_xs, P->d_cell_start, P->cg, gg, ag, L1.q);
    return hipGetLastError();
  }
  hipError_t e = launch_zero(L1.q, L1.g.size, s);
  if (e != hipSuccess || n == 0) return e;
  if (P->order == 4)
    k_anterp_f64<4><<<nblocks(n, kBlock), kBlock, 0, s>>>(P->d_xs, n, gg, L1.q);
  else
    k_anterp_f64<6><<<nblocks(n, kBlock), kBlock, 0, s>>>(P->d_xs, n, gg, L1.q);
  return hipGetLastError();
}

hipError_t launch_restrict(mls_plan_s* P, int k_fine, hipStream_t s) {
  Level& F = P->lv[k_fine - 1];
  Level& C = P->lv[k_fine];
  if (P->order == 4)
    k_restrict_f64<4><<<nblocks(C.g.size, kBlock), kBlock, 0, s>>>(F.q, F.g, C.q, C.g);
  else
    k_restrict_f64<6><<<nblocks(C.g.size, kBlock), kBlock, 0, s>>>(F.q, F.g, C.q, C.g);
  return hipGetLastError();
}

hipError_t launch_prolong(mls_plan_s* P, int k_fine, hipStream_t s) {
  Level& F = P->lv[k_fine - 1];
  Level& C = P->lv[k_fine];
  if (P->order == 4)
    k_prolong_f64<4><<<nblocks(F.g.size, kBlock), kBlock, 0, s>>>(C.E, C.g, F.e, F.E, F.g);
  else
    k_prolong_f64<6><<<nblocks(F.g.size, kBlock), kBlock, 0, s>>>(C.E, C.g, F.e, F.E, F.g);
  return hipGetLastError();
}

hipError_t launch_interpolate(mls_plan_s* P, int n, double* energy, double* forces, double* potential,
                              double* dE_dc6, hipStream_t s) {
  const int nb = std::max(1, nblocks(n, kBlock));
  if (n > 0) {
    GridGeom gg = finest_geom(P);
    OutPtrs out{forces, potential, dE_dc6};
    const bool mixed = P->precision == MLS_MIXED;
    if (P->order == 4 && !mixed)
      k_interp_f64<4, double><<<nb, kBlock, 0, s>>>(P->d_xs, P->d_perm, n, gg, P->lv[0].E, P->d_e0, P->d_floc,
                                                    P->cself, out, P->d_partial);
    else if (P->order == 4)
      k_interp_f64<4, float><<<nb, kBlock, 0, s>>>(P->d_xs, P->d_perm, n, gg, P->lv[0].E, P->d_e0, P->d_floc,
                                                   P->cself, out, P->d_partial);
    else if (!mixed)
      k_interp_f64<6, double><<<nb, kBlock, 0, s>>>(P->d_xs, P->d_perm, n, gg, P->lv[0].E, P->d_e0, P->d_floc,
                                                    P->cself, out, P->d_partial);
    else
      k_interp_f64<6, float><<<nb, kBlock, 0, s>>>(P->d_xs, P->d_perm, n, gg, P->lv[0].E, P->d_e0, P->d_floc,
                                                   P->cself, out, P->d_partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    hipError_t e = launch_zero(P->d_partial, 2, s);
    if (e != hipSuccess) return e;
  }
  k_energy_final<<<1, kBlock, 0, s>>>(P->d_partial, n > 0 ? nb : 1, P->cself, energy);
  return hipGetLastError();
}

hipError_t launch_copy_stage(mls_plan_s* P, int what, int level, void* dst, hipStream_t s) {
  const int n = (int)std::max<int64_t>(P->last_n, 0);
  switch (what) {
    case MLS_STAGE_PERM:
      return hipMemcpyAsync(dst, P->d_perm, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s);
    case MLS_STAGE_CELL_START:
      return hipMemcpyAsync(dst, P->d_cell_start, sizeof(int) * ((size_t)P->cg.ncell + 1), hipMemcpyDeviceToDevice,
                            s);
    case MLS_STAGE_E0:
    case MLS_STAGE_FLOC:
      if (n == 0) return hipSuccess;
      k_scatter_atoms<<<nblocks(n, kBlock), kBlock, 0, s>>>(P->d_perm, n, what == MLS_STAGE_E0 ? P->d_e0 : P->d_floc,
                                                            what == MLS_STAGE_E0 ? 1 : 3, (double*)dst);
      return hipGetLastError();
    default: {
      Level& L = P->lv[level - 1];
      const double* src = what == MLS_STAGE_Q ? L.q : (what == MLS_STAGE_E_LEVEL ? L.e : L.E);
      return hipMemcpyAsync(dst, src, sizeof(double) * (size_t)L.g.size, hipMemcpyDeviceToDevice, s);
    }
  }
}

}  // namespace mls
