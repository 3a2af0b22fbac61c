// Linked-cell binning (Sec. III.D): wrap positions into the box, assign each
// atom to its cell, and counting-sort the atoms by cell, stable in the
// original index.  The result is integer and bit-exact:
//   1. per atom: wrapped position, cell id, arrival slot in its cell (atomic)
//   2. exclusive scan of the cell counts (block scan, scan of block sums, add)
//   3. scatter to start[cell] + slot (arrival order)
//   4. per cell: reorder by original index (rank among the cell's atoms)
//   5. gather the sorted position/xi array and cell ids
#include <algorithm>

#include "device_math.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_bin_count(const double* __restrict__ pos,
                                                      const double* __restrict__ c6, int n, CellGeom g,
                                                      int* __restrict__ cid, int* __restrict__ slot,
                                                      int* __restrict__ count, double4* __restrict__ xw,
                                                      int* __restrict__ flags) {
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
  double X = wrap_coord(x, g.L[0], g.invL[0]);
  double Y = wrap_coord(y, g.L[1], g.invL[1]);
  double Z = wrap_coord(z, g.L[2], g.invL[2]);
  // coordinates so large that the wrap loses them are reported, not binned
  if (!(X >= 0.0 && X < g.L[0] && Y >= 0.0 && Y < g.L[1] && Z >= 0.0 && Z < g.L[2])) {
    bad |= 1;
    X = Y = Z = 0.0;
  }
  if (bad) atomicOr(flags, bad);
  int cx = max(0, min((int)(X * g.inv_w[0]), g.nc[0] - 1));
  int cy = max(0, min((int)(Y * g.inv_w[1]), g.nc[1] - 1));
  int cz = max(0, min((int)(Z * g.inv_w[2]), g.nc[2] - 1));
  int id = (cz * g.nc[1] + cy) * g.nc[0] + cx;
  cid[i] = id;
  xw[i] = make_double4(X, Y, Z, sqrt(c));
  slot[i] = atomicAdd(&count[id], 1);
}

// Scan phase 1: each block scans kScanItems consecutive counts (exclusive,
// written to start) and records its total and maximum.
constexpr int kScanPer = 8;
constexpr int kScanItems = kBlock * kScanPer;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    int u = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += u;
    __syncthreads();
  }
  total = sh[kBlock - 1];
  const int excl = sh[t] - v;
  __syncthreads();
  return excl;
}

__device__ __forceinline__ int block_max(int v, int* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  const int r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kBlock) k_scan_blocks(const int* __restrict__ count, int m,
                                                        int* __restrict__ start, int* __restrict__ bsum,
                                                        int* __restrict__ bmax) {
  __shared__ int sh[kBlock];
  const int base = blockIdx.x * kScanItems + threadIdx.x * kScanPer;
  int v[kScanPer];
  int sum = 0, mx = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < m ? count[base + k] : 0;
    sum += v[k];
    mx = max(mx, v[k]);
  }
  int total;
  int run = block_exclusive_scan(sum, sh, total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < m) start[base + k] = run;
    run += v[k];
  }
  const int bm = block_max(mx, sh);
  if (threadIdx.x == 0) {
    bsum[blockIdx.x] = total;
    bmax[blockIdx.x] = bm;
  }
}

// Scan phase 2: one block turns the block totals into exclusive offsets and
// writes the grand total start[m] and the largest cell count.
__global__ void __launch_bounds__(kBlock) k_scan_sums(int* __restrict__ bsum, const int* __restrict__ bmax, int nb,
                                                      int* __restrict__ start, int m, int* __restrict__ max_count) {
  __shared__ int sh[kBlock];
  int carry = 0, mx = 0;
  for (int b0 = 0; b0 < nb; b0 += kBlock) {
    const int b = b0 + threadIdx.x;
    const int v = b < nb ? bsum[b] : 0;
    if (b < nb) mx = max(mx, bmax[b]);
    int total;
    const int ex = block_exclusive_scan(v, sh, total);
    if (b < nb) bsum[b] = carry + ex;
    carry += total;
  }
  const int bm = block_max(mx, sh);
  if (threadIdx.x == 0) {
    start[m] = carry;
    *max_count = bm;
  }
}

// Scan phase 3: add each block's offset.
__global__ void __launch_bounds__(kBlock) k_scan_add(int* __restrict__ start, int m, const int* __restrict__ bsum) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < m) start[c] += bsum[c / kScanItems];
}

__global__ void __launch_bounds__(kBlock) k_bin_scatter(const int* __restrict__ cid, const int* __restrict__ slot,
                                                        int n, const int* __restrict__ start,
                                                        int* __restrict__ perm_tmp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  perm_tmp[start[cid[i]] + slot[i]] = i;
}

// One thread per cell: each atom's rank among the cell's atoms by original
// index is its stable position.
__global__ void __launch_bounds__(kBlock) k_cell_rank(const int* __restrict__ start, int ncell,
                                                      const int* __restrict__ perm_tmp, int* __restrict__ perm) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int b = start[c], e = start[c + 1];
  for (int k = b; k < e; ++k) {
    const int v = perm_tmp[k];
    int rank = 0;
    for (int j = b; j < e; ++j) rank += perm_tmp[j] < v;
    perm[b + rank] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_gather_sorted(const int* __restrict__ perm, int n,
                                                          const double4* __restrict__ xw,
                                                          const int* __restrict__ cid,
                                                          double4* __restrict__ xs, int* __restrict__ cell_s,
                                                          float4* __restrict__ xr, float* __restrict__ xif,
                                                          CellGeom g) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n + kSortedPad) return;
  if (s >= n) {
    // padding rows: far outside any cutoff, zero weight
    xs[s] = make_double4(1e300, 1e300, 1e300, 0.0);
    if (xr) {
      xr[s] = make_float4(1e30f, 1e30f, 1e30f, 0.0f);
      xif[s] = 0.0f;
    }
    return;
  }
  int i = perm[s];
  double4 p = xw[i];
  int c = cid[i];
  xs[s] = p;
  cell_s[s] = c;
  if (xr) {
    // cell-relative FP32 coordinates and the cell x index (exact in FP32)
    // for the mixed-precision pair kernel
    int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    xr[s] = make_float4((float)(p.x - cx * g.w[0]), (float)(p.y - cy * g.w[1]), (float)(p.z - cz * g.w[2]),
                        (float)cx);
    xif[s] = (float)p.w;
  }
}

// Pair-kernel target order: atoms of the cells taken in brick order.
__global__ void __launch_bounds__(kBlock) k_brick_counts(const int* __restrict__ order, const int* __restrict__ start,
                                                         int ncell, int* __restrict__ bcount) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const int c = order[k];
  bcount[k] = start[c + 1] - start[c];
}

__global__ void __launch_bounds__(kBlock) k_brick_targets(const int* __restrict__ order,
                                                          const int* __restrict__ start,
                                                          const int* __restrict__ bstart, int ncell,
                                                          int* __restrict__ tgt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const int c = order[k];
  const int b = start[c], e = start[c + 1], o = bstart[k];
  for (int i = b; i < e; ++i) tgt[o + (i - b)] = i;
}

// Sum of xi over the atoms (fixed order: per-block partials, then one block).
__global__ void __launch_bounds__(kBlock) k_sum_xi_blocks(const double4* __restrict__ xs, int n,
                                                          double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  sh[threadIdx.x] = s < n ? xs[s].w : 0.0;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kBlock) k_sum_final(const double* __restrict__ partial, int nb,
                                                      double* __restrict__ out) {
  __shared__ double sh[kBlock];
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) a += partial[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
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

int scan_blocks(int ncell) { return nblocks(ncell, kScanItems); }

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
  if (n > 0) {
    k_bin_count<<<nblocks(n, kBlock), kBlock, 0, s>>>(pos, c6, n, g, P->d_cid, P->d_slot, P->d_count, P->d_xw,
                                                      P->d_flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_scan(P, P->d_count, g.ncell, P->d_cell_start, s)) != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  k_bin_scatter<<<nblocks(n, kBlock), kBlock, 0, s>>>(P->d_cid, P->d_slot, n, P->d_cell_start, P->d_perm_tmp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_cell_rank<<<nblocks(g.ncell, kBlock), kBlock, 0, s>>>(P->d_cell_start, g.ncell, P->d_perm_tmp, P->d_perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_gather_sorted<<<nblocks(n + kSortedPad, kBlock), kBlock, 0, s>>>(P->d_perm, n, P->d_xw, P->d_cid, P->d_xs,
                                                                     P->d_cell_s, P->d_xr, P->d_xif, g);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (P->precision == MLS_MIXED) {
    // sum of xi: the mean of every grid level's charges (partition of unity)
    const int nb = nblocks(n, kBlock);
    k_sum_xi_blocks<<<nb, kBlock, 0, s>>>(P->d_xs, n, P->d_partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_sum_final<<<1, kBlock, 0, s>>>(P->d_partial, nb, P->d_scratch);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (P->pair_fast) {
    // the per-cell counts are no longer needed: reuse that array (ncell entries)
    k_brick_counts<<<nblocks(g.ncell, kBlock), kBlock, 0, s>>>(P->d_cell_order, P->d_cell_start, g.ncell,
                                                               P->d_count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_scan(P, P->d_count, g.ncell, P->d_bcount, s)) != hipSuccess) return e;
    k_brick_targets<<<nblocks(g.ncell, kBlock), kBlock, 0, s>>>(P->d_cell_order, P->d_cell_start, P->d_bcount,
                                                                g.ncell, P->d_tgt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scan(mls_plan_s* P, const int* count, int m, int* start, hipStream_t s) {
  const int nb = scan_blocks(m);
  k_scan_blocks<<<nb, kBlock, 0, s>>>(count, m, start, P->d_bsum, P->d_bmax);
  hipError_t e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_scan_sums<<<1, kBlock, 0, s>>>(P->d_bsum, P->d_bmax, nb, start, m, P->d_ncell_max);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_scan_add<<<nblocks(m, kBlock), kBlock, 0, s>>>(start, m, P->d_bsum);
  return hipGetLastError();
}

}  // namespace mls
