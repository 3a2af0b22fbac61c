// Linked-cell binning (Sec. III.D): wrap positions into the box, assign each
// atom to its cell, and counting-sort the atoms by cell, stable in the
// original index.  The result is integer and bit-exact:
//   1. per atom: wrapped position, cell id, arrival slot in its cell (atomic)
//   2. exclusive scan of the cell counts (block scan, scan of block sums, add)
//   3. scatter (index, cell) to start[cell] + slot (arrival order)
//   4. per atom: reorder by original index (rank among its cell's atoms)
//   5. gather the sorted position/xi array and cell ids (and, in mixed
//      precision, the per-block sums of xi)
#include <algorithm>

#include "device_math.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

struct FillI {
  using Args = FillArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int i = blk * kBlock + threadIdx.x;
    if (i < a.n) a.p[i] = 0;
  }
};

struct FillD {
  using Args = FillDArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int i = blk * kBlock + threadIdx.x;
    if (i < a.n) a.p[i] = 0.0;
  }
};

// Sanitised, wrapped position and xi of atom i (flags: 1 = position, 2 = C6).
// Non-finite positions and coordinates too large for the wrap become the
// origin, non-finite or negative C6 become 0.
__device__ __forceinline__ double4 wrap_values(double x, double y, double z, double c, const CellGeom& g,
                                               double scale, int& bad) {
  bad = 0;
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
  return make_double4(X, Y, Z, sqrt(scale * c));
}

__device__ __forceinline__ double4 wrapped_atom(const double* __restrict__ pos, const double* __restrict__ c6,
                                                int i, const CellGeom& g, double scale, int& bad) {
  return wrap_values(pos[3 * (size_t)i], pos[3 * (size_t)i + 1], pos[3 * (size_t)i + 2], c6[i], g, scale, bad);
}

// Linked cell of a wrapped position (clamped: a wrapped coordinate equal to
// the box length after rounding stays in the last cell).
__device__ __forceinline__ int cell_of(const double4& p, const CellGeom& g) {
  const int cx = max(0, min((int)(p.x * g.inv_w[0]), g.nc[0] - 1));
  const int cy = max(0, min((int)(p.y * g.inv_w[1]), g.nc[1] - 1));
  const int cz = max(0, min((int)(p.z * g.inv_w[2]), g.nc[2] - 1));
  return (cz * g.nc[1] + cy) * g.nc[0] + cx;
}

struct BinCount {
  using Args = BinCountArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    __shared__ double sh[kBlock];
    if (a.cond && *a.cond == 0) return;   // neighbour reuse: no binning this time
    const int i = blk * kBlock + threadIdx.x;
    double xi = 0.0;
    if (i < a.n) {
      const CellGeom& g = a.g;
      if (a.xref)
        for (int d = 0; d < 3; ++d) a.xref[3 * (size_t)i + d] = a.pos[3 * (size_t)i + d];
      int bad;
      const double4 p = wrapped_atom(a.pos, a.c6, i, g, a.c6_scale, bad);
      if (bad) atomicOr(a.flags, bad);
      const int id = cell_of(p, g);
      a.cid[i] = id;
      a.xw[i] = p;
      a.slot[i] = atomicAdd(&a.count[id], 1);
      xi = p.w;
    }
    if (a.xi_partial) {
      // per-block sum of xi over atoms in original order (fixed order)
      sh[threadIdx.x] = xi;
      __syncthreads();
      for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) a.xi_partial[blk] = sh[0];
    }
  }
};

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

struct ScanBlocks {
  using Args = ScanArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    __shared__ int sh[kBlock];
    if (a.cond && *a.cond == 0) return;
    const int base = blk * kScanItems + threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0, mx = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = base + k < a.m ? a.count[base + k] : 0;
      sum += v[k];
      mx = max(mx, v[k]);
    }
    // the counts are consumed here: leave them zero for the next binning
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
      if (base + k < a.m) a.count[base + k] = 0;
    int total;
    int run = block_exclusive_scan(sum, sh, total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (base + k < a.m) a.start[base + k] = run;
      run += v[k];
    }
    const int bm = block_max(mx, sh);
    if (threadIdx.x == 0) {
      a.bsum[blk] = total;
      a.bmax[blk] = bm;
    }
  }
};

// Scan phase 2: one block turns the block totals into exclusive offsets and
// writes the grand total start[m] and the largest cell count.
struct ScanSums {
  using Args = ScanArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int) {
    __shared__ int sh[kBlock];
    if (a.cond && *a.cond == 0) return;
    const int nb = (a.m + kScanItems - 1) / kScanItems;
    int carry = 0, mx = 0;
    for (int b0 = 0; b0 < nb; b0 += kBlock) {
      const int b = b0 + threadIdx.x;
      const int v = b < nb ? a.bsum[b] : 0;
      if (b < nb) mx = max(mx, a.bmax[b]);
      int total;
      const int ex = block_exclusive_scan(v, sh, total);
      if (b < nb) a.bsum[b] = carry + ex;
      carry += total;
    }
    const int bm = block_max(mx, sh);
    if (threadIdx.x == 0) {
      a.start[a.m] = carry;
      *a.max_count = bm;
    }
  }
};

// Scan phase 3: add each block's offset.
struct ScanAdd {
  using Args = ScanArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    if (a.cond && *a.cond == 0) return;
    const int c = blk * kBlock + threadIdx.x;
    if (c < a.m) a.start[c] += a.bsum[c / kScanItems];
  }
};

struct BinScatter {
  using Args = ScatterArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    if (a.cond && *a.cond == 0) return;
    const int i = blk * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const int c = a.cid[i];
    a.perm_tmp[a.start[c] + a.slot[i]] = make_int2(i, c);
  }
};

// One thread per atom: its rank among its cell's atoms by original index is
// its stable position (work per thread: the size of its cell).
struct CellRank {
  using Args = RankArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int s = blk * kBlock + threadIdx.x;
    if (s >= a.n) return;
    const int2 vc = a.perm_tmp[s];
    const int v = vc.x, c = vc.y;
    const int b = a.start[c], e = a.start[c + 1];
    int rank = 0;
    for (int j = b; j < e; ++j) rank += a.perm_tmp[j].x < v;
    a.perm[b + rank] = v;
  }
};

// FP32 rows of sorted atom d from its wrapped position p: the filter
// coordinates of the pair kernels (absolute x, cell-relative y and z; three
// arrays of xf_stride floats) and, for mixed-precision plans, the
// cell-relative coordinates with the cell x index (exact in FP32) and xi.
// The cell is the one BinCount took from the same wrapped position.
__device__ __forceinline__ void store_fp32_rows(float4* xr, float* xif, float* xf, int xfs, const CellGeom& g, int d,
                                                const double4& p) {
  if (!xf) return;
  const int cx = max(0, min((int)(p.x * g.inv_w[0]), g.nc[0] - 1));
  const int cy = max(0, min((int)(p.y * g.inv_w[1]), g.nc[1] - 1));
  const int cz = max(0, min((int)(p.z * g.inv_w[2]), g.nc[2] - 1));
  const float ry = (float)(p.y - cy * g.w[1]), rz = (float)(p.z - cz * g.w[2]);
  xf[d] = (float)p.x;
  xf[xfs + d] = ry;
  xf[2 * xfs + d] = rz;
  if (xr) {
    xr[d] = make_float4((float)(p.x - cx * g.w[0]), ry, rz, (float)cx);
    xif[d] = (float)p.w;
  }
}

// Padding rows: far outside any cutoff, zero weight.
__device__ __forceinline__ void store_fp32_pad(float4* xr, float* xif, float* xf, int xfs, int s) {
  if (xf)
    for (int k = 0; k < 3; ++k) xf[k * xfs + s] = 1e30f;
  if (xr) {
    xr[s] = make_float4(1e30f, 1e30f, 1e30f, 0.0f);
    xif[s] = 0.0f;
  }
}

struct RankGather {
  using Args = RankGatherArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    if (a.cond && *a.cond == 0) return;
    const int s = blk * kBlock + threadIdx.x;
    if (s < a.n) {
      const int2 vc = a.perm_tmp[s];
      const int v = vc.x, c = vc.y;
      const int b = a.start[c], e = a.start[c + 1];
      int rank = 0;
      for (int j = b; j < e; ++j) rank += a.perm_tmp[j].x < v;
      const int d = b + rank;   // stable position of atom v
      a.perm[d] = v;
      const double4 p = a.xw[v];
      a.xs[d] = p;
      a.cell_s[d] = c;
      store_fp32_rows(a.xr, a.xif, a.xf, a.xf_stride, a.g, d, p);
    } else if (s < a.n + kSortedPad) {
      // padding rows: far outside any cutoff, zero weight
      a.xs[s] = make_double4(1e300, 1e300, 1e300, 0.0);
      store_fp32_pad(a.xr, a.xif, a.xf, a.xf_stride, s);
    }
  }
};

// Bucketed counting sort (single plans).  Device-wide atomics on random
// cells are the slow part of the counting sort above (a few 10^10 per second
// on this chip, whatever their scope), so here the atoms are first ordered
// by bucket, a run of 2^shift consecutive cell ids, with block histograms and
// LDS atomics only; then one block orders each bucket by cell:
//   A. BinBucket: wrapped position, cell id, the block's bucket histogram
//      (and, in mixed precision, the per-256-atom sums of xi)
//   B. ScanBlocks over all histograms in bucket-major order (each scan block
//      exclusive on its own; the consumers add the totals of the scan blocks
//      before theirs, so the two other scan phases are not needed)
//   C. BucketScatter: (index, cell) into the bucket's range, LDS slots
//   D. BucketSort: per bucket, count its cells, write their starts, order
//      the bucket by cell (LDS slots), then each atom's rank among its
//      cell's atoms by original index gives its stable position, and the
//      sorted arrays are gathered as in RankGather.  A bucket of up to
//      kSortCap atoms is held in registers and LDS; a larger one goes
//      through tmp2 in global memory.
// The result is the same integer permutation as the counting sort above.
constexpr int kBinThreads = 512;
constexpr int kBinPer = 4;
constexpr int kBinItems = kBinThreads * kBinPer;
constexpr int kMaxBuckets = 4096;
constexpr int kBucketShiftMin = 9, kBucketShiftMax = 11;
constexpr int64_t kMaxHist = (int64_t)1 << 24;
constexpr int kSortThreads = 1024;
constexpr int kSortPer = 4;
constexpr int kSortCap = kSortThreads * kSortPer;

template <int T>
__device__ __forceinline__ int block_sum_i(int v, int* ws) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int w = 0; w < T / 64; ++w) t += ws[w];
  __syncthreads();
  return t;
}

struct BinBucket {
  using Args = BinBucketArgs;
  static constexpr int kThreads = kBinThreads;
  static __device__ void run(const Args& a, int blk) {
    __shared__ int hist[kMaxBuckets];
    __shared__ double sh[kBinThreads];
    if (a.cond && *a.cond == 0) return;
    for (int b = threadIdx.x; b < a.nbucket; b += kBinThreads) hist[b] = 0;
    // every load of the block in flight before the first use
    double x[kBinPer], y[kBinPer], z[kBinPer], c[kBinPer];
#pragma unroll
    for (int u = 0; u < kBinPer; ++u) {
      const size_t i = min(blk * kBinItems + u * kBinThreads + (int)threadIdx.x, a.n - 1);
      x[u] = a.pos[3 * i];
      y[u] = a.pos[3 * i + 1];
      z[u] = a.pos[3 * i + 2];
      c[u] = a.c6[i];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kBinPer; ++u) {
      const int i = blk * kBinItems + u * kBinThreads + threadIdx.x;
      double xi = 0.0;
      if (i < a.n) {
        if (a.xref) {
          a.xref[3 * (size_t)i] = x[u];
          a.xref[3 * (size_t)i + 1] = y[u];
          a.xref[3 * (size_t)i + 2] = z[u];
        }
        int bad;
        const double4 p = wrap_values(x[u], y[u], z[u], c[u], a.g, a.c6_scale, bad);
        if (bad) atomicOr(a.flags, bad);
        const int id = cell_of(p, a.g);
        a.cid[i] = id;
        a.xw[i] = p;
        atomicAdd(&hist[id >> a.shift], 1);
        xi = p.w;
      }
      if (a.xi_partial) {
        // the sum of xi over each 256 consecutive atoms (fixed order: within
        // each wave by the xor tree, then the four waves in order)
        double v = xi;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if ((threadIdx.x & 63) == 0) sh[(u & 1) * (kBinThreads / 64) + (threadIdx.x >> 6)] = v;
        __syncthreads();
        const int t = threadIdx.x & 255;
        const int base = blk * kBinItems + u * kBinThreads + (threadIdx.x & ~255);
        if (t == 0 && base < a.n) {
          const double* w = sh + (u & 1) * (kBinThreads / 64) + (threadIdx.x >> 6);
          a.xi_partial[base >> 8] = ((w[0] + w[1]) + w[2]) + w[3];
        }
      }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < a.nbucket; b += kBinThreads) a.hist[(size_t)b * a.nblk + blk] = hist[b];
  }
};

struct BucketScatter {
  using Args = BucketScatterArgs;
  static constexpr int kThreads = kBinThreads;
  static constexpr int kMaxScanBlocks = (int)(kMaxHist / kScanItems);
  static __device__ void run(const Args& a, int blk) {
    __shared__ int next[kMaxBuckets];
    __shared__ int sbo[kMaxScanBlocks];
    __shared__ int ws[kBinThreads / 64];
    if (a.cond && *a.cond == 0) return;
    int c[kBinPer];
#pragma unroll
    for (int u = 0; u < kBinPer; ++u) c[u] = a.cid[min(blk * kBinItems + u * kBinThreads + (int)threadIdx.x, a.n - 1)];
    // exclusive prefix of the scan blocks' totals
    const int m = a.nbucket * a.nblk, nsb = (m + kScanItems - 1) / kScanItems;
    int carry = 0;
    for (int k0 = 0; k0 < nsb; k0 += kBinThreads) {
      const int k = k0 + threadIdx.x;
      int total;
      const int ex = block_scan_excl<kBinThreads>(k < nsb ? a.bsum[k] : 0, ws, total);
      if (k < nsb) sbo[k] = carry + ex;
      carry += total;
    }
    __syncthreads();
    // where this block's atoms of each bucket start
    for (int b = threadIdx.x; b < a.nbucket; b += kBinThreads) {
      const int i = b * a.nblk + blk;
      next[b] = a.hist[i] + sbo[i / kScanItems];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kBinPer; ++u) {
      const int i = blk * kBinItems + u * kBinThreads + threadIdx.x;
      if (i < a.n) {
        const int p = atomicAdd(&next[c[u] >> a.shift], 1);
        a.tmp[p] = make_int2(i, c[u]);
      }
    }
  }
};

struct BucketSort {
  using Args = BucketSortArgs;
  static constexpr int kThreads = kSortThreads;
  static constexpr int kCells = 1 << kBucketShiftMax;
  static_assert(kCells == 2 * kSortThreads, "two cells per thread in the scan of the cell counts");

  // Exclusive scan of the bucket's cell counts cur[0, nc) into cst (cst[nc]:
  // the bucket's atoms), the cells' starts to global memory, cur := cst.
  static __device__ void cell_starts(const Args& a, int b, int c0, int nc, int lo, int* cst, int* cur, int* ws) {
    const int t2 = 2 * threadIdx.x;
    const int v0 = t2 < nc ? cur[t2] : 0, v1 = t2 + 1 < nc ? cur[t2 + 1] : 0;
    int total;
    const int ex = block_scan_excl<kSortThreads>(v0 + v1, ws, total);
    if (t2 < nc) cst[t2] = ex;
    if (t2 + 1 < nc) cst[t2 + 1] = ex + v0;
    if (threadIdx.x == 0) cst[nc] = total;
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += kSortThreads) {
      a.start[c0 + c] = lo + cst[c];
      cur[c] = cst[c];
    }
    if (b == a.nbucket - 1 && threadIdx.x == 0) a.start[a.g.ncell] = a.n;
    __syncthreads();
  }

  __device__ static void emit(const Args& a, int v, int c, int d, const double4& p) {
    a.perm[d] = v;
    a.xs[d] = p;
    a.cell_s[d] = c;
    store_fp32_rows(a.xr, a.xif, a.xf, a.xf_stride, a.g, d, p);
  }

  static __device__ void run(const Args& a, int b) {
    __shared__ int cst[kCells + 1], cur[kCells];
    __shared__ int2 srt[kSortCap];
    __shared__ int ws[kSortThreads / 64];
    if (a.cond && *a.cond == 0) return;
    const int c0 = b << a.shift;
    const int nc = min(1 << a.shift, a.g.ncell - c0);
    // the bucket's range in tmp: its scanned histogram entry plus the totals
    // of the scan blocks before it
    const int m = a.nbucket * a.nblk;
    const int i0 = b * a.nblk, i1 = (b + 1) * a.nblk;
    int s0 = 0, s1 = 0;
    for (int k = threadIdx.x; k < i1 / kScanItems; k += kSortThreads) {
      const int v = a.bsum[k];
      s1 += v;
      if (k < i0 / kScanItems) s0 += v;
    }
    s0 = block_sum_i<kSortThreads>(s0, ws);
    s1 = block_sum_i<kSortThreads>(s1, ws);
    const int lo = i0 < m ? s0 + a.hist[i0] : a.n;
    const int hi = i1 < m ? s1 + a.hist[i1] : a.n;
    const int cnt = hi - lo;
    for (int c = threadIdx.x; c < nc; c += kSortThreads) cur[c] = 0;
    __syncthreads();
    if (cnt <= kSortCap) {
      int2 e[kSortPer];
#pragma unroll
      for (int k = 0; k < kSortPer; ++k) {
        const int j = threadIdx.x + k * kSortThreads;
        e[k] = j < cnt ? a.tmp[lo + j] : make_int2(0, c0);
      }
#pragma unroll
      for (int k = 0; k < kSortPer; ++k)
        if ((int)threadIdx.x + k * kSortThreads < cnt) atomicAdd(&cur[e[k].y - c0], 1);
      __syncthreads();
      cell_starts(a, b, c0, nc, lo, cst, cur, ws);
      // the bucket in cell order (arrival order within a cell)
#pragma unroll
      for (int k = 0; k < kSortPer; ++k)
        if ((int)threadIdx.x + k * kSortThreads < cnt) srt[atomicAdd(&cur[e[k].y - c0], 1)] = e[k];
      __syncthreads();
      int v[kSortPer], c[kSortPer], d[kSortPer];
#pragma unroll
      for (int k = 0; k < kSortPer; ++k) {
        const int s = threadIdx.x + k * kSortThreads;
        v[k] = 0;
        c[k] = c0;
        d[k] = -1;
        if (s < cnt) {
          const int2 vc = srt[s];
          v[k] = vc.x;
          c[k] = vc.y;
          const int cb = cst[vc.y - c0], ce = cst[vc.y - c0 + 1];
          int rank = 0;
          for (int j = cb; j < ce; ++j) rank += srt[j].x < vc.x;
          d[k] = lo + cb + rank;   // stable position of atom v
        }
      }
      double4 p[kSortPer];
#pragma unroll
      for (int k = 0; k < kSortPer; ++k) p[k] = a.xw[v[k]];   // every gather in flight
#pragma unroll
      for (int k = 0; k < kSortPer; ++k)
        if (d[k] >= 0) emit(a, v[k], c[k], d[k], p[k]);
    } else {
      for (int j = lo + threadIdx.x; j < hi; j += kSortThreads) atomicAdd(&cur[a.tmp[j].y - c0], 1);
      __syncthreads();
      cell_starts(a, b, c0, nc, lo, cst, cur, ws);
      for (int j = lo + threadIdx.x; j < hi; j += kSortThreads) {
        const int2 t = a.tmp[j];
        a.tmp2[lo + atomicAdd(&cur[t.y - c0], 1)] = t;
      }
      __syncthreads();
      for (int s = lo + threadIdx.x; s < hi; s += kSortThreads) {
        const int2 vc = a.tmp2[s];
        const int cb = lo + cst[vc.y - c0], ce = lo + cst[vc.y - c0 + 1];
        int rank = 0;
        for (int j = cb; j < ce; ++j) rank += a.tmp2[j].x < vc.x;
        emit(a, vc.x, vc.y, cb + rank, a.xw[vc.x]);
      }
    }
    if (b == a.nbucket - 1) {
      // padding rows: far outside any cutoff, zero weight
      for (int s = a.n + threadIdx.x; s < a.n + kSortedPad; s += kSortThreads) {
        a.xs[s] = make_double4(1e300, 1e300, 1e300, 0.0);
        store_fp32_pad(a.xr, a.xif, a.xf, a.xf_stride, s);
      }
    }
  }
};

// Neighbour reuse: *cond = 1 when some atom has moved more than skin/2
// since the positions of the last binning (or a position is not finite).
struct DispCheck {
  using Args = DispCheckArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int i = blk * kBlock + threadIdx.x;
    bool far = false;
    if (i < a.n) {
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double u = a.pos[3 * (size_t)i + d] - a.xref[3 * (size_t)i + d];
        d2 += u * u;
      }
      far = !(d2 <= a.lim2);
    }
    if (__any(far) && (threadIdx.x & 63) == 0) atomicOr(a.cond, 1);
  }
};

// Neighbour reuse without a binning (*cond == 0): the atom in sorted slot s
// keeps its cell; its new position is stored as the cell centre plus the
// periodic image of its offset from the centre nearest to the centre, so it
// lies within skin/2 of its cell (positions may leave [0, L) by as much).
// The image is unique: the atom is within w/2 + skin/2 < L/2 of the centre
// (cells at least a + skin wide when there are fewer than five per side, at
// least (a + skin)/2 otherwise; one cell per side is the whole box).
struct Regather {
  using Args = RegatherArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    if (*a.cond != 0) return;
    const int s = blk * kBlock + threadIdx.x;
    if (s >= a.n) return;
    const CellGeom& g = a.g;
    const int i = a.perm[s], c = a.cell_s[s];
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    const int cc[3] = {cx, cy, cz};
    double x[3], r[3];
    for (int d = 0; d < 3; ++d) {
      const double corner = cc[d] * g.w[d];
      const double centre = corner + 0.5 * g.w[d];
      double rel = a.pos[3 * (size_t)i + d] - centre;
      rel -= g.L[d] * rint(rel * g.invL[d]);
      x[d] = centre + rel;
      r[d] = x[d] - corner;
    }
    const double w = a.xs[s].w;
    a.xs[s] = make_double4(x[0], x[1], x[2], w);
    if (a.xr) a.xr[s] = make_float4((float)r[0], (float)r[1], (float)r[2], (float)cx);
    if (a.xf) {
      a.xf[s] = (float)x[0];
      a.xf[a.xf_stride + s] = (float)r[1];
      a.xf[2 * a.xf_stride + s] = (float)r[2];
    }
  }
};

struct GatherSorted {
  using Args = GatherArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    __shared__ double sh[kBlock];
    const int s = blk * kBlock + threadIdx.x;
    double xi = 0.0;
    if (s < a.n) {
      const int i = a.perm[s];
      const double4 p = a.xw[i];
      // the cell of BinCount, recomputed from the same wrapped position (no
      // second random read)
      const CellGeom& g = a.g;
      const int cx = max(0, min((int)(p.x * g.inv_w[0]), g.nc[0] - 1));
      const int cy = max(0, min((int)(p.y * g.inv_w[1]), g.nc[1] - 1));
      const int cz = max(0, min((int)(p.z * g.inv_w[2]), g.nc[2] - 1));
      const int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
      a.xs[s] = p;
      a.cell_s[s] = c;
      xi = p.w;
      store_fp32_rows(a.xr, a.xif, a.xf, a.xf_stride, g, s, p);
    } else if (s < a.n + kSortedPad) {
      // padding rows: far outside any cutoff, zero weight
      a.xs[s] = make_double4(1e300, 1e300, 1e300, 0.0);
      store_fp32_pad(a.xr, a.xif, a.xf, a.xf_stride, s);
    }
    if (a.xi_partial) {
      // per-block sum of xi (fixed order)
      sh[threadIdx.x] = xi;
      __syncthreads();
      for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) a.xi_partial[blk] = sh[0];
    }
  }
};

// Lorentz-Berthelot: sigma in sorted order (padding rows 0) and its flag.
struct LbGather {
  using Args = LbGatherArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int s = blk * kBlock + threadIdx.x;
    if (s >= a.n + kSortedPad) return;
    double v = 0.0;
    if (s < a.n) {
      v = a.sigma[a.perm[s]];
      if (!isfinite(v) || !(v >= 0.0)) {
        atomicOr(a.flags, 2);
        v = 0.0;
      }
    }
    a.sig_s[s] = v;
    if (a.sig_f) a.sig_f[s] = (float)v;
  }
};

// Lorentz-Berthelot charge vector k in sorted order:
// xi_{i,k} = sigma_i^k sqrt(binom(6,k) 2 eps_i) / 8 = sigma_i^k sqrt(binom(6,k)) e_i / 8,
// e_i = sqrt(2 eps_i) being the xi of the binning.
struct LbCharge {
  using Args = LbChargeArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int s = blk * kBlock + threadIdx.x;
    if (s >= a.n + kSortedPad) return;
    double q = 0.0;
    if (s < a.n) {
      const double sg = a.sig_s[s];
      double sk = 1.0;
      for (int j = 0; j < a.k; ++j) sk *= sg;
      const int binom = a.k == 0 || a.k == 6 ? 1 : (a.k == 1 || a.k == 5 ? 6 : (a.k == 2 || a.k == 4 ? 15 : 20));
      q = sk * sqrt((double)binom) * a.xs[s].w * 0.125;
    }
    a.charge[s] = q;
    if (a.partial) {
      // per-block sum of the charges (fixed order; padding rows add 0)
      __shared__ double sh[kBlock];
      sh[threadIdx.x] = q;
      __syncthreads();
      for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
      }
      if (threadIdx.x == 0) a.partial[blk] = sh[0];
    }
  }
};

// Sum of xi over the atoms from the gather's per-block partials (fixed order).
struct SumXiFinal {
  using Args = SumXiArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int) {
    __shared__ double sh[kBlock];
    const int nb = (a.rows + kBlock - 1) / kBlock;
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) v += a.partial[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) *a.out = sh[0];
  }
};

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

int bin_block_items() { return kBinItems; }

bool bin_buckets(int64_t ncell, int64_t n_max, int& shift, int& nbucket) {
  for (int s = kBucketShiftMin; s <= kBucketShiftMax; ++s) {
    const int64_t nb = (ncell + ((int64_t)1 << s) - 1) >> s;
    if (nb > kMaxBuckets) continue;
    if (nb * ((n_max + kBinItems - 1) / kBinItems) > kMaxHist) return false;
    shift = s;
    nbucket = (int)nb;
    return true;
  }
  return false;
}

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
  return launch_binning_scaled(P, n, pos, c6, 1.0, s);
}

hipError_t launch_lb_gather(mls_plan_s* P, int n, const double* sigma, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return launch_one<LbGather>(LbGatherArgs{P->d_perm, n, sigma, P->d_sig, P->d_flags, P->d_sigf},
                              nblocks(n + kSortedPad, kBlock), s);
}

hipError_t launch_lb_charge(mls_plan_s* P, int n, int k, hipStream_t s) {
  const bool mixed = P->precision == MLS_MIXED;
  if (n > 0) {
    hipError_t e = launch_one<LbCharge>(
        LbChargeArgs{P->d_xs, P->d_sig, n, k, lb_charge_buf(P, k), mixed ? lb_partial_buf(P, k) : nullptr},
        nblocks(n + kSortedPad, kBlock), s);
    if (e != hipSuccess) return e;
  }
  // mixed precision: the sum of this vector's charges, the mean the stencil
  // subtracts (0 without atoms)
  if (!mixed) return hipSuccess;
  return launch_one<SumXiFinal>(SumXiArgs{n > 0 ? n + kSortedPad : 0, lb_partial_buf(P, k), lb_sum_buf(P, k)}, 1, s);
}

// The binning kernels; with `cond` they all do nothing when *cond == 0, and
// with `xref` the count kernel records the positions.
static hipError_t binning_core(mls_plan_s* P, int n, const double* pos, const double* c6, double scale,
                               const int* cond, double* xref, hipStream_t s) {
  // The cell counts start at zero: cleared once at plan creation, then by
  // every scan after it has read them.
  const CellGeom& g = P->cg;
  const bool mixed = P->precision == MLS_MIXED;
  hipError_t e;
  if (P->bin_nbucket) {
    const int nblk = nblocks(n, kBinItems), m = P->bin_nbucket * nblk;
    if (n > 0) {
      BinBucketArgs a{pos, c6, n, g, P->d_cid, P->d_xw, P->d_flags, scale, mixed ? P->d_partial : nullptr, cond,
                      xref, P->bin_shift, P->bin_nbucket, nblk, P->d_bin_hist};
      if ((e = launch_one<BinBucket>(a, nblk, s)) != hipSuccess) return e;
    }
    // in place, per scan block: the histograms become the start of each
    // (bucket, block) run within its scan block
    ScanArgs sa{P->d_bin_hist, m, P->d_bin_hist, P->d_bsum, P->d_bmax, P->d_ncell_max, cond};
    if ((e = launch_one<ScanBlocks>(sa, scan_blocks(m), s)) != hipSuccess) return e;
    if (n > 0) {
      BucketScatterArgs ca{P->d_cid, n, P->bin_shift, P->bin_nbucket, nblk, P->d_bin_hist, P->d_bsum,
                           P->d_perm_tmp, cond};
      if ((e = launch_one<BucketScatter>(ca, nblk, s)) != hipSuccess) return e;
    }
    BucketSortArgs da{P->d_bin_hist, P->d_bsum, nblk, P->bin_shift, P->bin_nbucket, P->d_perm_tmp, P->d_perm_tmp2, n,
                      P->d_cell_start, P->d_perm, P->d_xw, P->d_xs, P->d_cell_s, P->d_xr, P->d_xif, g, cond,
                      P->d_xf, P->xf_stride};
    return launch_one<BucketSort>(da, P->bin_nbucket, s);
  }
  if (n > 0) {
    BinCountArgs a{pos, c6, n, g, P->d_cid, P->d_slot, P->d_count, P->d_xw, P->d_flags, scale,
                   mixed ? P->d_partial : nullptr, cond, xref};
    if ((e = launch_one<BinCount>(a, nblocks(n, kBlock), s)) != hipSuccess) return e;
  }
  ScanArgs sa{P->d_count, g.ncell, P->d_cell_start, P->d_bsum, P->d_bmax, P->d_ncell_max, cond};
  if ((e = launch_one<ScanBlocks>(sa, scan_blocks(g.ncell), s)) != hipSuccess) return e;
  if ((e = launch_one<ScanSums>(sa, 1, s)) != hipSuccess) return e;
  if ((e = launch_one<ScanAdd>(sa, nblocks(g.ncell, kBlock), s)) != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  if ((e = launch_one<BinScatter>(ScatterArgs{P->d_cid, P->d_slot, n, P->d_cell_start, P->d_perm_tmp, cond},
                                  nblocks(n, kBlock), s)) != hipSuccess)
    return e;
  RankGatherArgs ra{P->d_cell_start, P->d_perm_tmp, n, P->d_perm, P->d_xw, P->d_xs, P->d_cell_s, P->d_xr,
                    P->d_xif, g, cond, P->d_xf, P->xf_stride};
  return launch_one<RankGather>(ra, nblocks(n + kSortedPad, kBlock), s);
}

hipError_t launch_binning_scaled(mls_plan_s* P, int n, const double* pos, const double* c6, double scale,
                                 hipStream_t s) {
  return binning_core(P, n, pos, c6, scale, nullptr, nullptr, s);
}

hipError_t launch_binning_ref(mls_plan_s* P, int n, const double* pos, const double* c6, hipStream_t s) {
  return binning_core(P, n, pos, c6, 1.0, nullptr, P->d_xref, s);
}

hipError_t launch_binning_reuse(mls_plan_s* P, int n, const double* pos, const double* c6, hipStream_t s) {
  hipError_t e;
  if ((e = launch_one<FillI>(FillArgs{P->d_rebin, 1}, 1, s)) != hipSuccess) return e;
  if (n > 0) {
    const double half = 0.5 * P->skin;
    DispCheckArgs da{pos, P->d_xref, n, half * half, P->d_rebin};
    if ((e = launch_one<DispCheck>(da, nblocks(n, kBlock), s)) != hipSuccess) return e;
  }
  if ((e = binning_core(P, n, pos, c6, 1.0, P->d_rebin, P->d_xref, s)) != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  RegatherArgs ra{pos, P->d_perm, P->d_cell_s, n, P->cg, P->d_rebin, P->d_xs, P->d_xr, P->d_xf,
                  P->xf_stride};
  return launch_one<Regather>(ra, nblocks(n, kBlock), s);
}

hipError_t launch_sum_xi(mls_plan_s* P, int n, hipStream_t s) {
  if (P->precision != MLS_MIXED || n == 0) return hipSuccess;
  // sum of xi: the mean of every grid level's charges (partition of unity),
  // from the binning's per-block partial sums
  SumXiArgs sa{n, P->d_partial, P->d_scratch};
  return launch_one<SumXiFinal>(sa, 1, s);
}

hipError_t launch_scan(mls_plan_s* P, int* count, int m, int* start, hipStream_t s) {
  ScanArgs a{count, m, start, P->d_bsum, P->d_bmax, P->d_ncell_max};
  hipError_t e;
  if ((e = launch_one<ScanBlocks>(a, scan_blocks(m), s)) != hipSuccess) return e;
  if ((e = launch_one<ScanSums>(a, 1, s)) != hipSuccess) return e;
  return launch_one<ScanAdd>(a, nblocks(m, kBlock), s);
}

hipError_t launch_batched_binning(const BatchPhase& ph, hipStream_t s) {
  switch (ph.kernel) {
    case BK_FILL_I: return launch_batched_phase<FillI>(ph, s);
    case BK_FILL_D: return launch_batched_phase<FillD>(ph, s);
    case BK_BIN_COUNT: return launch_batched_phase<BinCount>(ph, s);
    case BK_SCAN_BLOCKS: return launch_batched_phase<ScanBlocks>(ph, s);
    case BK_SCAN_SUMS: return launch_batched_phase<ScanSums>(ph, s);
    case BK_SCAN_ADD: return launch_batched_phase<ScanAdd>(ph, s);
    case BK_SCATTER: return launch_batched_phase<BinScatter>(ph, s);
    case BK_RANK: return launch_batched_phase<CellRank>(ph, s);
    case BK_GATHER: return launch_batched_phase<GatherSorted>(ph, s);
    case BK_SUM_XI_FINAL: return launch_batched_phase<SumXiFinal>(ph, s);
    case BK_LB_GATHER: return launch_batched_phase<LbGather>(ph, s);
    case BK_LB_CHARGE: return launch_batched_phase<LbCharge>(ph, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mls
