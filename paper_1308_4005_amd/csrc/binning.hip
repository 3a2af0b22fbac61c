// Linked-cell binning (Sec. III.D): wrap positions into the box, assign each
// atom to the cell of width L/nc (the smallest width >= a dividing the box),
// and counting-sort the atoms by cell, stable in the original index.  The
// result is integer and bit-exact: per-cell counts by atomics, an exclusive
// scan, an unordered scatter, then a rank sort inside every cell by original
// index.
#include <algorithm>

#include "device_math.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_bin_count(const double* __restrict__ pos,
                                                      const double* __restrict__ c6, int n, CellGeom g,
                                                      int* __restrict__ cid, int* __restrict__ count,
                                                      double4* __restrict__ xw, int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = pos[3 * (size_t)i], y = pos[3 * (size_t)i + 1], z = pos[3 * (size_t)i + 2];
  double c = c6[i];
  int bad = 0;
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
    bad |= 1;
    x = y = z = 0.0;
  }
  if (!isfinite(c) || !(c >= 0.0)) {
    bad |= 2;
    c = 0.0;
  }
  if (bad) atomicOr(flags, bad);
  double X = wrap_coord(x, g.L[0], g.invL[0]);
  double Y = wrap_coord(y, g.L[1], g.invL[1]);
  double Z = wrap_coord(z, g.L[2], g.invL[2]);
  // coordinates so large that the wrap loses them are reported, not binned
  if (!(X >= 0.0 && X < g.L[0] && Y >= 0.0 && Y < g.L[1] && Z >= 0.0 && Z < g.L[2])) {
    atomicOr(flags, 1);
    X = Y = Z = 0.0;
  }
  int cx = max(0, min((int)(X * g.inv_w[0]), g.nc[0] - 1));
  int cy = max(0, min((int)(Y * g.inv_w[1]), g.nc[1] - 1));
  int cz = max(0, min((int)(Z * g.inv_w[2]), g.nc[2] - 1));
  int id = (cz * g.nc[1] + cy) * g.nc[0] + cx;
  cid[i] = id;
  xw[i] = make_double4(X, Y, Z, sqrt(c));
  atomicAdd(&count[id], 1);
}

// Exclusive scan of `count` (m entries) into start[0..m]; one block.
constexpr int kScan = 1024;
__global__ void __launch_bounds__(kScan) k_scan(const int* __restrict__ count, int* __restrict__ start, int m,
                                                int* __restrict__ max_count) {
  __shared__ int s[kScan];
  __shared__ int smax[kScan];
  const int t = threadIdx.x;
  const int per = (m + kScan - 1) / kScan;
  const int b = min(m, t * per), e = min(m, b + per);
  int sum = 0, mx = 0;
  for (int i = b; i < e; ++i) {
    int c = count[i];
    sum += c;
    mx = max(mx, c);
  }
  s[t] = sum;
  smax[t] = mx;
  __syncthreads();
  for (int off = 1; off < kScan; off <<= 1) {
    int v = t >= off ? s[t - off] : 0;
    int w = t >= off ? smax[t - off] : 0;
    __syncthreads();
    s[t] += v;
    smax[t] = max(smax[t], w);
    __syncthreads();
  }
  int run = s[t] - sum;
  for (int i = b; i < e; ++i) {
    start[i] = run;
    run += count[i];
  }
  if (t == kScan - 1) {
    start[m] = s[kScan - 1];
    *max_count = smax[kScan - 1];
  }
}

__global__ void __launch_bounds__(kBlock) k_bin_scatter(const int* __restrict__ cid, int n,
                                                        const int* __restrict__ start, int* __restrict__ fill,
                                                        int* __restrict__ perm_tmp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cid[i];
  int slot = start[c] + atomicAdd(&fill[c], 1);
  perm_tmp[slot] = i;
}

// One wave per cell: each atom's rank among the cell's atoms by original
// index gives its stable position.
constexpr int kWave = 64;
__global__ void __launch_bounds__(kBlock) k_cell_rank(const int* __restrict__ start, int ncell,
                                                      const int* __restrict__ perm_tmp, int* __restrict__ perm) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  if (wave >= ncell) return;
  const int b = start[wave], e = start[wave + 1];
  const int cnt = e - b;
  for (int k = lane; k < cnt; k += kWave) {
    const int v = perm_tmp[b + k];
    int rank = 0;
    for (int j = 0; j < cnt; ++j) rank += perm_tmp[b + j] < v;
    perm[b + rank] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_gather_sorted(const int* __restrict__ perm, int n,
                                                          const double4* __restrict__ xw,
                                                          const int* __restrict__ cid,
                                                          double4* __restrict__ xs, int* __restrict__ cell_s,
                                                          float4* __restrict__ xr, CellGeom g) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int i = perm[s];
  double4 p = xw[i];
  int c = cid[i];
  xs[s] = p;
  cell_s[s] = c;
  if (xr) {
    // cell-relative FP32 coordinates for the mixed-precision pair kernel
    int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    xr[s] = make_float4((float)(p.x - cx * g.w[0]), (float)(p.y - cy * g.w[1]), (float)(p.z - cz * g.w[2]),
                        (float)p.w);
  }
}

__global__ void k_zero(double* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void k_zero_i(int* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

inline int nblocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_zero(double* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>(nblocks(count, kBlock), 4096);
  k_zero<<<blocks, kBlock, 0, s>>>(p, count);
  return hipGetLastError();
}

hipError_t launch_zero_i(int* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>(nblocks(count, kBlock), 4096);
  k_zero_i<<<blocks, kBlock, 0, s>>>(p, count);
  return hipGetLastError();
}

hipError_t launch_binning(mls_plan_s* P, int n, const double* pos, const double* c6, hipStream_t s) {
  const CellGeom& g = P->cg;
  hipError_t e;
  if ((e = launch_zero_i(P->d_count, g.ncell, s)) != hipSuccess) return e;
  if ((e = launch_zero_i(P->d_fill, g.ncell, s)) != hipSuccess) return e;
  if (n > 0) {
    k_bin_count<<<nblocks(n, kBlock), kBlock, 0, s>>>(pos, c6, n, g, P->d_cid, P->d_count, P->d_xw, P->d_flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  k_scan<<<1, kScan, 0, s>>>(P->d_count, P->d_cell_start, g.ncell, P->d_ncell_max);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  k_bin_scatter<<<nblocks(n, kBlock), kBlock, 0, s>>>(P->d_cid, n, P->d_cell_start, P->d_fill, P->d_perm_tmp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_cell_rank<<<nblocks((int64_t)g.ncell * kWave, kBlock), kBlock, 0, s>>>(P->d_cell_start, g.ncell,
                                                                           P->d_perm_tmp, P->d_perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_gather_sorted<<<nblocks(n, kBlock), kBlock, 0, s>>>(P->d_perm, n, P->d_xw, P->d_cid, P->d_xs, P->d_cell_s,
                                                        P->d_xr, g);
  return hipGetLastError();
}

}  // namespace mls
