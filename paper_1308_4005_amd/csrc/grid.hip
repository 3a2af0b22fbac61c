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

// ------------------------------------------------------------ anterpolation
template <int P>
struct AnterpAtomic {
  using Args = AnterpArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int s = blk * kBlock + threadIdx.x;
    if (s >= a.n) return;
    const GridGeom& gg = a.gg;
    const double4 p = a.xs[s];
    const double qi = a.charge ? a.charge[s] : p.w;
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
        const double wzy = qi * w[2][jz] * w[1][jy];
        double* row = a.q + ((size_t)idx[2][jz] * gg.n[1] + idx[1][jy]) * gg.n[0];
#pragma unroll
        for (int jx = 0; jx < P; ++jx) unsafeAtomicAdd(row + idx[0][jx], wzy * w[0][jx]);
      }
  }
};

// Owner-computes anterpolation: a block owns the finest-grid points whose
// positions fall inside a box of CBx x CBy x CBz linked cells (point m of
// dimension d belongs to cell-block b when ceil(c0 n/nc) <= m < ceil(c1 n/nc)).
// It gathers the atoms of those cells and of an nh-cell halo (with their
// periodic image shifts), adds each atom's p^3 contributions that land on
// owned points into an LDS tile, and stores the tile without global atomics.
constexpr int kAntTile = 16;     // max owned points per dimension
constexpr int kAntThreads = 256;
static_assert(kAntTileRows == kAntThreads, "one cell row per thread in the run scan");
constexpr int kMaxSeg = 1024;
constexpr int kAntScan = kMaxSeg / kAntThreads;   // scan slots per thread

template <int P, class W>
struct AnterpOwned {
  using Args = AnterpArgs;
  static constexpr int kThreads = kAntThreads;
  static __device__ void run(const Args& a, int b) {
    __shared__ double tile[kAntTile * kAntTile * kAntTile];
    __shared__ int seg_begin[kMaxSeg];
    __shared__ int seg_off[kMaxSeg + 1];
    __shared__ int seg_shift[kMaxSeg][3];
    __shared__ int nseg_s;
    __shared__ int scan_sh[kAntThreads];
    const CellGeom& cg = a.cg;
    const GridGeom& gg = a.gg;
    const AntGeom& ag = a.ag;
    const int* __restrict__ cstart = a.cstart;
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
    // contiguous runs of sorted atoms: one thread per row of cells along x;
    // a row splits into at most rx runs where the periodic image changes
    // (empty slots get length 0)
    const int span[3] = {c1[0] - c0[0] + 2 * ag.nh[0], c1[1] - c0[1] + 2 * ag.nh[1], c1[2] - c0[2] + 2 * ag.nh[2]};
    const int rx = min(span[0], (span[0] + cg.nc[0] - 1) / cg.nc[0] + 1);
    const int nrows = span[1] * span[2];
    const int nslot = nrows * rx;   // <= kMaxSeg (checked on the host)
    for (int r = threadIdx.x; r < nrows; r += kAntThreads) {
      const int cy = c0[1] - ag.nh[1] + r % span[1];
      const int cz = c0[2] - ag.nh[2] + r / span[1];
      const int iz = floordiv(cz, cg.nc[2]);
      const int iy = floordiv(cy, cg.nc[1]);
      const int rowc = ((cz - iz * cg.nc[2]) * cg.nc[1] + (cy - iy * cg.nc[1])) * cg.nc[0];
      int k = r * rx;
      int cx = c0[0] - ag.nh[0];
      const int cxe = c1[0] + ag.nh[0];
      while (cx < cxe) {
        const int ix = floordiv(cx, cg.nc[0]);
        const int wx = cx - ix * cg.nc[0];
        const int run = min(cxe - cx, cg.nc[0] - wx);
        const int a0 = cstart[rowc + wx];
        seg_begin[k] = a0;
        seg_off[k] = cstart[rowc + wx + run] - a0;   // length, turned into offsets below
        seg_shift[k][0] = ix;
        seg_shift[k][1] = iy;
        seg_shift[k][2] = iz;
        ++k;
        cx += run;
      }
      for (; k < (r + 1) * rx; ++k) seg_off[k] = 0;
    }
    __syncthreads();
    // exclusive scan of the lengths (kAntScan consecutive slots per thread)
    {
      int len[kAntScan];
      int sum = 0;
      const int base = threadIdx.x * kAntScan;
#pragma unroll
      for (int k = 0; k < kAntScan; ++k) {
        len[k] = base + k < nslot ? seg_off[base + k] : 0;
        sum += len[k];
      }
      scan_sh[threadIdx.x] = sum;
      __syncthreads();
      for (int off = 1; off < kAntThreads; off <<= 1) {
        const int u = threadIdx.x >= off ? scan_sh[threadIdx.x - off] : 0;
        __syncthreads();
        scan_sh[threadIdx.x] += u;
        __syncthreads();
      }
      int run = scan_sh[threadIdx.x] - sum;
#pragma unroll
      for (int k = 0; k < kAntScan; ++k) {
        if (base + k < nslot) seg_off[base + k] = run;
        run += len[k];
      }
      if (threadIdx.x == kAntThreads - 1) {
        seg_off[nslot] = run;
        nseg_s = nslot;
      }
    }
    __syncthreads();
    const int ns = nseg_s;
    const int tot = seg_off[ns];
    // the block's atom list is cut into 64 contiguous chunks, one per lane
    // position; the waves take turns within a chunk.  The 64 lanes of a wave
    // then work on atoms far apart in the list (different cells), so their
    // LDS additions rarely land on the same grid points.
    const int lanepos = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWaves = kAntThreads / 64;
    const int chunk = (tot + 63) / 64;
    const int i0 = lanepos * chunk, i1 = min(i0 + chunk, tot);
    int sg = 0;
    {
      // first segment holding i0 (binary search over the run offsets)
      int lo = 0, hi = ns;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg_off[mid] <= i0) lo = mid; else hi = mid;
      }
      sg = lo;
    }
    for (int i = i0 + wave; i < i1; i += kWaves) {
      while (seg_off[sg + 1] <= i) ++sg;
      const int ia = seg_begin[sg] + (i - seg_off[sg]);
      const double4 p = a.xs[ia];
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
      const W xiw = (W)(a.charge ? a.charge[ia] : p.w);
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
      a.q[((size_t)(lo[2] + lz) * gg.n[1] + (lo[1] + ly)) * gg.n[0] + lo[0] + lx] =
          tile[(lz * kAntTile + ly) * kAntTile + lx];
    }
  }
};

// Two-phase anterpolation.  Phase 1: a block takes the atoms of one block of
// linked cells only (no halo), adds their p^3 contributions into an LDS tile
// spanning every finest point those atoms reach (unwrapped indices), and
// stores the tile into its own box of the expanded grid.  Phase 2: every
// finest point sums the (at most 4 x 4 x 4, usually 1 to 8) expanded-grid
// values that belong to it, periodic images included, in a fixed order.
// Weights in W (FP32 in mixed precision), charges accumulated in FP64.
// CAP: the LDS tile's capacity in doubles, the one the tables were built for.
template <int P, class W, int CAP = kAntTileMax>
struct AnterpTile {
  using Args = AnterpTileArgs;
  static constexpr int kThreads = kAntThreads;
  static __device__ void run(const Args& a, int b) {
    __shared__ double tile[CAP];
    __shared__ int seg_begin[kAntTileRows];
    __shared__ int seg_off[kAntTileRows + 1];
    __shared__ int scan_ws[kAntThreads / 64];
    const AntTiles& T = a.t;
    const int* __restrict__ tab = a.tab;
    const CellGeom& cg = a.cg;
    const GridGeom& gg = a.gg;
    const int bi[3] = {b % T.nb[0], (b / T.nb[0]) % T.nb[1], b / (T.nb[0] * T.nb[1])};
    int c0[3], c1[3], e0[3], len[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c0[d] = tab[T.off_c[d] + bi[d]];
      c1[d] = tab[T.off_c[d] + bi[d] + 1];
      e0[d] = tab[T.off_e[d] + bi[d]];
      len[d] = tab[T.off_len[d] + bi[d]];
    }
    const int vol = len[0] * len[1] * len[2];   // <= CAP (host-checked)
    for (int i = threadIdx.x; i < vol; i += kAntThreads) tile[i] = 0.0;
    // the block's atoms: one contiguous run of sorted atoms per cell row (y, z)
    const int ny = c1[1] - c0[1];
    const int nrows = ny * (c1[2] - c0[2]);   // <= kAntTileRows = kAntThreads (host-checked)
    int len_r = 0;
    if ((int)threadIdx.x < nrows) {
      const int cy = c0[1] + threadIdx.x % ny, cz = c0[2] + threadIdx.x / ny;
      const int row = (cz * cg.nc[1] + cy) * cg.nc[0];
      const int a0 = a.cstart[row + c0[0]];
      seg_begin[threadIdx.x] = a0;
      len_r = a.cstart[row + c1[0]] - a0;
    }
    // exclusive scan of the run lengths (one run per thread)
    {
      int all = 0;
      const int ex = block_scan_excl<kAntThreads>(len_r, scan_ws, all);
      seg_off[threadIdx.x] = ex;
      if (threadIdx.x == kAntThreads - 1) seg_off[kAntThreads] = all;
    }
    __syncthreads();
    const int tot = seg_off[nrows];
    // atoms far apart in the list go to the 64 lanes of a wave (their LDS
    // additions rarely meet); the waves take turns within a lane's chunk
    const int lanepos = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWaves = kAntThreads / 64;
    const int chunk = (tot + 63) / 64;
    const int i0 = lanepos * chunk, i1 = min(i0 + chunk, tot);
    int sg = 0;
    {
      int lo = 0, hi = nrows;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg_off[mid] <= i0) lo = mid; else hi = mid;
      }
      sg = lo;
    }
    const int pitch_y = len[0], pitch_z = len[0] * len[1];
    for (int i = i0 + wave; i < i1; i += kWaves) {
      while (seg_off[sg + 1] <= i) ++sg;
      const int ia = seg_begin[sg] + (i - seg_off[sg]);
      const double4 p = a.xs[ia];
      const double pc[3] = {p.x, p.y, p.z};
      W w[3][P];
      int l0[3];
      bool inside = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double t = pc[d] * gg.invh[d];
        const double m0 = floor(t);
        basis_weights<P, W>((W)(t - m0), w[d]);
        l0[d] = (int)m0 - (P / 2 - 1) - e0[d];
        inside = inside && l0[d] >= 0 && l0[d] + P <= len[d];
      }
      if (!inside) {
        // cannot happen for atoms of the block's cells (the reached ranges
        // carry a margin); reported instead of writing outside the tile
        atomicOr(a.flags, 4);
        continue;
      }
      const W qi = (W)(a.charge ? a.charge[ia] : p.w);
      double* base = tile + l0[2] * pitch_z + l0[1] * pitch_y + l0[0];
#pragma unroll
      for (int jz = 0; jz < P; ++jz)
#pragma unroll
        for (int jy = 0; jy < P; ++jy) {
          const W wzy = qi * w[2][jz] * w[1][jy];
          double* row = base + jz * pitch_z + jy * pitch_y;
#pragma unroll
          for (int jx = 0; jx < P; ++jx) atomicAdd(row + jx, (double)(wzy * w[0][jx]));
        }
    }
    __syncthreads();
    const int X0 = tab[T.off_x0[0] + bi[0]], Y0 = tab[T.off_x0[1] + bi[1]], Z0 = tab[T.off_x0[2] + bi[2]];
    BoxWalk wk(threadIdx.x, kAntThreads, len);
    for (int i = threadIdx.x; i < vol; i += kAntThreads) {
      a.scratch[((size_t)(Z0 + wk.z) * T.NX[1] + (Y0 + wk.y)) * T.NX[0] + (X0 + wk.x)] = tile[i];
      wk.step(len);
    }
  }
};

struct AnterpCollect {
  using Args = AnterpCollectArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int m = blk * kBlock + threadIdx.x;
    if (m >= a.g.size) return;
    const int mx = m % a.g.n[0], my = (m / a.g.n[0]) % a.g.n[1], mz = m / (a.g.n[0] * a.g.n[1]);
    const AntTiles& T = a.t;
    const int4 cx = reinterpret_cast<const int4*>(a.tab + T.off_cov[0])[mx];
    const int4 cy = reinterpret_cast<const int4*>(a.tab + T.off_cov[1])[my];
    const int4 cz = reinterpret_cast<const int4*>(a.tab + T.off_cov[2])[mz];
    const int xs[4] = {cx.x, cx.y, cx.z, cx.w}, ys[4] = {cy.x, cy.y, cy.z, cy.w}, zs[4] = {cz.x, cz.y, cz.z, cz.w};
    double sum = 0.0;
    for (int kz = 0; kz < 4 && zs[kz] >= 0; ++kz)
      for (int ky = 0; ky < 4 && ys[ky] >= 0; ++ky) {
        const double* row = a.scratch + ((size_t)zs[kz] * T.NX[1] + ys[ky]) * T.NX[0];
        for (int kx = 0; kx < 4 && xs[kx] >= 0; ++kx) sum += row[xs[kx]];
      }
    a.q[m] = sum;
  }
};

// ------------------------------------------------------------ restriction
// Per-dimension taps around fine index 2M: offsets 0, +-1, +-3 (, +-5).
template <int P>
__device__ __forceinline__ void restrict_at(const TransferArgs& a, int M) {
    const GridDims& f = a.gs;
    const GridDims& c = a.gd;
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
    for (int i = 0; i < K; ++i) {
      double sy = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double* row = a.src + ((size_t)iz[i] * f.n[1] + iy[j]) * f.n[0];
        double sx = 0.0;
#pragma unroll
        for (int cc = 0; cc < K; ++cc) sx += w[cc] * row[ix[cc]];
        sy += w[j] * sx;
      }
      acc += w[i] * sy;
    }
    a.dst[M] = acc;
}

template <int P>
struct Restrict {
  using Args = TransferArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int M = blk * kBlock + threadIdx.x;
    if (M < a.gd.size) restrict_at<P>(a, M);
  }
};

// ------------------------------------------------------------ prolongation
// Fine index j receives coarse M with j - 2M in {0} (j even) or the odd
// offsets +-1, +-3 (, +-5) (j odd).  One thread per coarse point M writes the
// 2 x 2 x 2 fine points 2M + {0,1}: both parities need only the coarse points
// M - P/2 + 1 .. M + P/2 per dimension (the even one uses M alone), so the
// thread walks those P z-planes, interpolates each plane in x then y, and
// adds it into the 8 outputs.
template <int P, bool ROLL = false>
__device__ __forceinline__ void prolong_at(const TransferArgs& a, int M) {
    const GridDims& c = a.gs;
    const GridDims& f = a.gd;
    const int X = M % c.n[0], Y = (M / c.n[0]) % c.n[1], Z = M / (c.n[0] * c.n[1]);
    constexpr int H = P / 2;
    double w[P];   // weight of coarse M - H + 1 + t for the odd fine point 2M + 1
    int ix[P], iy[P], iz[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const int o = 2 * H - 1 - 2 * t;   // (2M + 1) - 2 (M - H + 1 + t)
      w[t] = rp_weight_odd<P>(((o < 0 ? -o : o) - 1) / 2);
      ix[t] = wrapi(X - H + 1 + t, c.n[0]);
      iy[t] = wrapi(Y - H + 1 + t, c.n[1]);
      iz[t] = wrapi(Z - H + 1 + t, c.n[2]);
    }
    double acc[2][2][2];   // [z parity][y parity][x parity]
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[1][0][q] = acc[1][1][q] = acc[0][0][q] = acc[0][1][q] = 0.0;
    // The z planes run in a loop, the plane's weight and index rotated into
    // slot 0.  ROLL: not unrolled (p = 4: 56 VGPRs, the batched form; p = 6:
    // 70 instead of 448).  Otherwise two planes per iteration (p = 4: 96
    // VGPRs, five waves per SIMD, 32 loads in flight per thread): the finest
    // level of a 10^6-atom plan, 2744 waves, then fits the chip in one round,
    // where all four planes unrolled (188 VGPRs, two waves per SIMD) took 1.3
    // rounds (prolongation stage 0.036 -> 0.035 ms)
    double wz[P];
    int izr[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
      wz[t] = w[t];
      izr[t] = iz[t];
    }
    constexpr int kUnrollZ = ROLL ? 1 : 2;
#pragma unroll kUnrollZ
    for (int tz = 0; tz < P; ++tz) {
      double ye[2] = {0.0, 0.0}, yo[2] = {0.0, 0.0};   // y even / odd, [x parity]
#pragma unroll
      for (int ty = 0; ty < P; ++ty) {
        const double* row = a.src + ((size_t)izr[0] * c.n[1] + iy[ty]) * c.n[0];
        double v[P];
#pragma unroll
        for (int tx = 0; tx < P; ++tx) v[tx] = row[ix[tx]];
        double xo = 0.0;
#pragma unroll
        for (int tx = 0; tx < P; ++tx) xo += w[tx] * v[tx];
        const double xe = v[H - 1];
        if (ty == H - 1) {
          ye[0] = xe;
          ye[1] = xo;
        }
        yo[0] += w[ty] * xe;
        yo[1] += w[ty] * xo;
      }
      if (tz == H - 1) {
        acc[0][0][0] = ye[0];
        acc[0][0][1] = ye[1];
        acc[0][1][0] = yo[0];
        acc[0][1][1] = yo[1];
      }
      acc[1][0][0] += wz[0] * ye[0];
      acc[1][0][1] += wz[0] * ye[1];
      acc[1][1][0] += wz[0] * yo[0];
      acc[1][1][1] += wz[0] * yo[1];
#pragma unroll
      for (int t = 0; t + 1 < P; ++t) {
        wz[t] = wz[t + 1];
        izr[t] = izr[t + 1];
      }
    }
#pragma unroll
    for (int pz = 0; pz < 2; ++pz)
#pragma unroll
      for (int py = 0; py < 2; ++py) {
        const size_t J = ((size_t)(2 * Z + pz) * f.n[1] + (2 * Y + py)) * f.n[0] + 2 * X;
        a.dst[J] = (a.add ? a.add[J] : 0.0) + acc[pz][py][0];
        a.dst[J + 1] = (a.add ? a.add[J + 1] : 0.0) + acc[pz][py][1];
      }
}

template <int P, bool ROLL = false>
struct Prolong {
  using Args = TransferArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int M = blk * kBlock + threadIdx.x;
    if (M < a.gs.size) prolong_at<P, ROLL>(a, M);
  }
};

// Small levels: a grid transfer of a few thousand points has too few threads
// to hide its loads (each thread of the forms above issues (p+1)^3 or p^3 of
// them one after another), so there a group of lanes shares one coarse point.
// Restriction: 8 lanes per coarse point split its (p+1)^2 (z, y) rows, each
// lane sums its rows' x taps, and the group adds its partial sums (fixed
// order).  Prolongation: one lane per z-plane of the coarse point's p^3
// neighbourhood (groups of 4 for p = 4, 8 for p = 6), the group adds the
// planes' contributions to the 8 fine points, and each lane writes some of
// them.  The sums are the same as above up to the order of the terms.
constexpr int kRestrictGroup = 8;

// tap t of a transfer in one dimension: offset 0 (t = 0), -(2k+1) (t = 1+2k),
// +(2k+1) (t = 2+2k)
template <int P>
__device__ __forceinline__ void restrict_tap(int t, int& off, double& w) {
  const int k = (t - 1) >> 1;
  off = t == 0 ? 0 : ((t & 1) ? -(2 * k + 1) : 2 * k + 1);
  w = t == 0 ? 1.0 : rp_weight_odd<P>(k);
}

template <int P>
struct RestrictSplit {
  using Args = TransferArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int t = blk * kBlock + threadIdx.x;
    const int M = t / kRestrictGroup, g = t % kRestrictGroup;
    const GridDims& f = a.gs;
    const GridDims& c = a.gd;
    constexpr int K = P + 1;
    double acc = 0.0;
    if (M < c.size) {
      const int X = M % c.n[0], Y = (M / c.n[0]) % c.n[1], Z = M / (c.n[0] * c.n[1]);
      int ix[K];
      double w[K];
#pragma unroll
      for (int cc = 0; cc < K; ++cc) {
        int o;
        restrict_tap<P>(cc, o, w[cc]);
        ix[cc] = wrapi(2 * X + o, f.n[0]);
      }
      for (int r = g; r < K * K; r += kRestrictGroup) {
        const int i = r / K, j = r - (r / K) * K;
        int oi, oj;
        double wi, wj;
        restrict_tap<P>(i, oi, wi);
        restrict_tap<P>(j, oj, wj);
        const double* row = a.src + ((size_t)wrapi(2 * Z + oi, f.n[2]) * f.n[1] + wrapi(2 * Y + oj, f.n[1])) * f.n[0];
        double sx = 0.0;
#pragma unroll
        for (int cc = 0; cc < K; ++cc) sx += w[cc] * row[ix[cc]];
        acc += (wi * wj) * sx;
      }
    }
#pragma unroll
    for (int off = 1; off < kRestrictGroup; off <<= 1) acc += __shfl_xor(acc, off);
    if (M < c.size && g == 0) a.dst[M] = acc;
  }
};

template <int P>
struct ProlongSplit {
  using Args = TransferArgs;
  static constexpr int kThreads = kBlock;
  static constexpr int G = P <= 4 ? 4 : 8;   // lanes per coarse point, one per z-plane
  static __device__ void run(const Args& a, int blk) {
    const int t = blk * kBlock + threadIdx.x;
    const int M = t / G, g = t % G;
    const GridDims& c = a.gs;
    const GridDims& f = a.gd;
    constexpr int H = P / 2;
    // this lane's plane tz = g: [z parity][y parity][x parity] contributions
    double v8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v8[q] = 0.0;
    const bool live = M < c.size;
    const int Mc = live ? M : 0;
    const int X = Mc % c.n[0], Y = (Mc / c.n[0]) % c.n[1], Z = Mc / (c.n[0] * c.n[1]);
    if (live && g < P) {
      double w[P];
      int ix[P], iy[P];
#pragma unroll
      for (int u = 0; u < P; ++u) {
        const int o = 2 * H - 1 - 2 * u;
        w[u] = rp_weight_odd<P>(((o < 0 ? -o : o) - 1) / 2);
        ix[u] = wrapi(X - H + 1 + u, c.n[0]);
        iy[u] = wrapi(Y - H + 1 + u, c.n[1]);
      }
      const int og = 2 * H - 1 - 2 * g;
      const double wz = rp_weight_odd<P>(((og < 0 ? -og : og) - 1) / 2);
      const int iz = wrapi(Z - H + 1 + g, c.n[2]);
      double ye[2] = {0.0, 0.0}, yo[2] = {0.0, 0.0};
#pragma unroll
      for (int ty = 0; ty < P; ++ty) {
        const double* row = a.src + ((size_t)iz * c.n[1] + iy[ty]) * c.n[0];
        double v[P];
#pragma unroll
        for (int tx = 0; tx < P; ++tx) v[tx] = row[ix[tx]];
        double xo = 0.0;
#pragma unroll
        for (int tx = 0; tx < P; ++tx) xo += w[tx] * v[tx];
        const double xe = v[H - 1];
        if (ty == H - 1) {
          ye[0] = xe;
          ye[1] = xo;
        }
        yo[0] += w[ty] * xe;
        yo[1] += w[ty] * xo;
      }
      if (g == H - 1) {   // the even fine z takes the centre plane alone
        v8[0] = ye[0];
        v8[1] = ye[1];
        v8[2] = yo[0];
        v8[3] = yo[1];
      }
      v8[4] = wz * ye[0];
      v8[5] = wz * ye[1];
      v8[6] = wz * yo[0];
      v8[7] = wz * yo[1];
    }
#pragma unroll
    for (int off = 1; off < G; off <<= 1)
#pragma unroll
      for (int q = 0; q < 8; ++q) v8[q] += __shfl_xor(v8[q], off);
    if (!live) return;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q % G != g) continue;
      const int pz = q >> 2, py = (q >> 1) & 1, px = q & 1;
      const size_t J = ((size_t)(2 * Z + pz) * f.n[1] + (2 * Y + py)) * f.n[0] + 2 * X + px;
      a.dst[J] = (a.add ? a.add[J] : 0.0) + v8[q];
    }
  }
};

// ------------------------------------------------------------ interpolation + assembly
// Interpolated value and gradient (in grid units) of one grid at an atom with
// weights w, dw and wrapped indices idx.  The p z-planes are walked in a loop
// that is not unrolled (few registers, more waves); the plane's z weight and
// offset sit in slot 0 of local copies rotated after each plane.
template <int P, class W>
__device__ __forceinline__ void interp_grid(const double* __restrict__ E1, const GridGeom& gg,
                                            const W (&w)[3][P], const W (&dw)[3][P], const int (&idx)[3][P],
                                            double& u, double& gx, double& gy, double& gz) {
  W wz[P], dwz[P];
  int iz[P];
  size_t yrow[P];
#pragma unroll
  for (int t = 0; t < P; ++t) {
    wz[t] = w[2][t];
    dwz[t] = dw[2][t];
    iz[t] = idx[2][t];
    yrow[t] = (size_t)idx[1][t] * gg.n[0];
  }
  const size_t plane = (size_t)gg.n[0] * gg.n[1];
  u = gx = gy = gz = 0.0;
#pragma unroll 1
  for (int jz = 0; jz < P; ++jz) {
    const double* E1z = E1 + (size_t)iz[0] * plane;
    double ru = 0.0, rgx = 0.0, rgy = 0.0;
#pragma unroll
    for (int jy = 0; jy < P; ++jy) {
      const double* row = E1z + yrow[jy];
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
    u += (double)wz[0] * ru;
    gx += (double)wz[0] * rgx;
    gy += (double)wz[0] * rgy;
    gz += (double)dwz[0] * ru;
#pragma unroll
    for (int t = 0; t + 1 < P; ++t) {
      wz[t] = wz[t + 1];
      dwz[t] = dwz[t + 1];
      iz[t] = iz[t + 1];
    }
  }
}

template <int P, class W>
__device__ __forceinline__ void interp_setup(const double4& p, const GridGeom& gg, W (&w)[3][P], W (&dw)[3][P],
                                             int (&idx)[3][P]) {
  const double pc[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double t = pc[d] * gg.invh[d];
    const double m0 = floor(t);
    basis_weights_d<P, W>((W)(t - m0), w[d], dw[d]);
    const int base = (int)m0 - (P / 2 - 1);
#pragma unroll
    for (int j = 0; j < P; ++j) idx[d][j] = wrapi(base + j, gg.n[d]);
  }
}

// block reduction of the two energy sums (fixed order: deterministic)
__device__ __forceinline__ void energy_partials(double su, double sxx, double* __restrict__ partial, int blk) {
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
    partial[2 * blk] = r1[0];
    partial[2 * blk + 1] = r2[0];
  }
}

template <int P, class W>
struct Interp {
  using Args = InterpArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const GridGeom& gg = a.gg;
    const int s = blk * kBlock + threadIdx.x;
    double su = 0.0, sxx = 0.0;
    if (s < a.n) {
      const double4 p = a.xs[s];
      // the per-atom loads that do not depend on the grid go first, so their
      // latency overlaps the grid gathers
      const int i = a.perm[s];
      double e0 = 0.0, fl0 = 0.0, fl1 = 0.0, fl2 = 0.0;
      if (!a.grid_only) {
        e0 = a.e0[s];
        fl0 = a.floc[3 * (size_t)s + 0];
        fl1 = a.floc[3 * (size_t)s + 1];
        fl2 = a.floc[3 * (size_t)s + 2];
      }
      if (a.frep) {
        fl0 += a.frep[3 * (size_t)s + 0];
        fl1 += a.frep[3 * (size_t)s + 1];
        fl2 += a.frep[3 * (size_t)s + 2];
      }
      W w[3][P], dw[3][P];
      int idx[3][P];
      interp_setup<P, W>(p, gg, w, dw, idx);
      double u, gx, gy, gz;
      interp_grid<P, W>(a.E1, gg, w, dw, idx, u, gx, gy, gz);
      const double xi = p.w;
      const double utot = e0 + u;
      if (a.out.forces) {
        a.out.forces[3 * (size_t)i + 0] = fl0 + xi * gx * gg.invh[0];
        a.out.forces[3 * (size_t)i + 1] = fl1 + xi * gy * gg.invh[1];
        a.out.forces[3 * (size_t)i + 2] = fl2 + xi * gz * gg.invh[2];
      }
      if (a.out.potential) a.out.potential[i] = utot;
      if (a.out.dE_dc6) a.out.dE_dc6[i] = -(utot - a.cself * xi) / (2.0 * xi);
      su = xi * utot;
      sxx = xi * xi;
    }
    energy_partials(su, sxx, a.partial, blk);
  }
};

// Interpolation over the anterpolation's blocks of linked cells (the same
// tables): a block loads the finest-grid values its atoms reach (at most
// CAP, unwrapped, with the periodic wrap applied on load) into LDS,
// eight loads in flight per thread, then every atom of its cells gathers its
// p^3 values from LDS instead of global memory.  Outputs as Interp; the
// energy sums are per block (fixed order).
template <int P, class W, int CAP = kAntTileMax>
struct InterpTile {
  using Args = InterpTileArgs;
  static constexpr int kThreads = kAntThreads;
  static __device__ void run(const Args& ta, int b) {
    __shared__ double tile[CAP];
    __shared__ int seg_begin[kAntTileRows];
    __shared__ int seg_off[kAntTileRows + 1];
    __shared__ int scan_ws[kAntThreads / 64];
    const InterpArgs& a = ta.a;
    const AntTiles& T = ta.t;
    const int* __restrict__ tab = ta.tab;
    const CellGeom& cg = ta.cg;
    const GridGeom& gg = a.gg;
    const int bi[3] = {b % T.nb[0], (b / T.nb[0]) % T.nb[1], b / (T.nb[0] * T.nb[1])};
    int c0[3], c1[3], e0[3], len[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c0[d] = tab[T.off_c[d] + bi[d]];
      c1[d] = tab[T.off_c[d] + bi[d] + 1];
      e0[d] = tab[T.off_e[d] + bi[d]];
      len[d] = tab[T.off_len[d] + bi[d]];
    }
    const int vol = len[0] * len[1] * len[2];   // <= CAP (host-checked)
    const size_t plane = (size_t)gg.n[0] * gg.n[1];
    constexpr int kFill = 8;
    // element coordinates stepped, not divided out; the reached ranges lie
    // within [-n, 2n) per dimension (host-checked), so one conditional wrap
    BoxWalk wk(threadIdx.x, kAntThreads, len);
    for (int i0 = threadIdx.x; i0 < vol; i0 += kFill * kAntThreads) {
      double v[kFill];
#pragma unroll
      for (int u = 0; u < kFill; ++u) {
        // past the end: an element of the last plane, loaded but not stored
        const int lz = min(wk.z, len[2] - 1);
        v[u] = a.E1[(size_t)wrap_near(e0[2] + lz, gg.n[2]) * plane +
                    (size_t)wrap_near(e0[1] + wk.y, gg.n[1]) * gg.n[0] + wrap_near(e0[0] + wk.x, gg.n[0])];
        wk.step(len);
      }
#pragma unroll
      for (int u = 0; u < kFill; ++u)
        if (i0 + u * kAntThreads < vol) tile[i0 + u * kAntThreads] = v[u];
    }
    // the block's atoms: one contiguous run of sorted atoms per cell row (y, z)
    const int ny = c1[1] - c0[1];
    const int nrows = ny * (c1[2] - c0[2]);   // <= kAntTileRows = kAntThreads (host-checked)
    int len_r = 0;
    if ((int)threadIdx.x < nrows) {
      const int cy = c0[1] + threadIdx.x % ny, cz = c0[2] + threadIdx.x / ny;
      const int row = (cz * cg.nc[1] + cy) * cg.nc[0];
      const int a0 = ta.cstart[row + c0[0]];
      seg_begin[threadIdx.x] = a0;
      len_r = ta.cstart[row + c1[0]] - a0;
    }
    {
      int all = 0;
      const int ex = block_scan_excl<kAntThreads>(len_r, scan_ws, all);
      seg_off[threadIdx.x] = ex;
      if (threadIdx.x == kAntThreads - 1) seg_off[kAntThreads] = all;
    }
    __syncthreads();
    const int tot = seg_off[nrows];
    const int pitch_y = len[0], pitch_z = len[0] * len[1];
    double su = 0.0, sxx = 0.0;
    int sg = 0;
    for (int i = threadIdx.x; i < tot; i += kAntThreads) {
      while (seg_off[sg + 1] <= i) ++sg;
      const int s = seg_begin[sg] + (i - seg_off[sg]);
      const double4 p = a.xs[s];
      const int ia = a.perm[s];
      double e0v = 0.0, fl0 = 0.0, fl1 = 0.0, fl2 = 0.0;
      if (!a.grid_only) {
        e0v = a.e0[s];
        fl0 = a.floc[3 * (size_t)s + 0];
        fl1 = a.floc[3 * (size_t)s + 1];
        fl2 = a.floc[3 * (size_t)s + 2];
      }
      if (a.frep) {
        fl0 += a.frep[3 * (size_t)s + 0];
        fl1 += a.frep[3 * (size_t)s + 1];
        fl2 += a.frep[3 * (size_t)s + 2];
      }
      const double pc[3] = {p.x, p.y, p.z};
      W w[3][P], dw[3][P];
      int l0[3];
      bool inside = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double t = pc[d] * gg.invh[d];
        const double m0 = floor(t);
        basis_weights_d<P, W>((W)(t - m0), w[d], dw[d]);
        l0[d] = (int)m0 - (P / 2 - 1) - e0[d];
        inside = inside && l0[d] >= 0 && l0[d] + P <= len[d];
      }
      if (!inside) {
        // cannot happen for atoms of the block's cells (the reached ranges
        // carry a margin); reported instead of reading outside the tile
        atomicOr(ta.flags, 4);
        continue;
      }
      const double* base = tile + l0[2] * pitch_z + l0[1] * pitch_y + l0[0];
      double u = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      // the z planes in a loop that is not unrolled (few registers, more
      // waves), the plane's weights rotated into slot 0
      W wz[P], dwz[P];
#pragma unroll
      for (int t = 0; t < P; ++t) {
        wz[t] = w[2][t];
        dwz[t] = dw[2][t];
      }
#pragma unroll 1
      for (int jz = 0; jz < P; ++jz) {
        double ru = 0.0, rgx = 0.0, rgy = 0.0;
#pragma unroll
        for (int jy = 0; jy < P; ++jy) {
          const double* row = base + jy * pitch_y;
          double v = 0.0, vd = 0.0;
#pragma unroll
          for (int jx = 0; jx < P; ++jx) {
            const double e = row[jx];
            v += (double)w[0][jx] * e;
            vd += (double)dw[0][jx] * e;
          }
          ru += (double)w[1][jy] * v;
          rgx += (double)w[1][jy] * vd;
          rgy += (double)dw[1][jy] * v;
        }
        u += (double)wz[0] * ru;
        gx += (double)wz[0] * rgx;
        gy += (double)wz[0] * rgy;
        gz += (double)dwz[0] * ru;
        base += pitch_z;
#pragma unroll
        for (int t = 0; t + 1 < P; ++t) {
          wz[t] = wz[t + 1];
          dwz[t] = dwz[t + 1];
        }
      }
      const double xi = p.w;
      const double utot = e0v + u;
      if (a.out.forces) {
        a.out.forces[3 * (size_t)ia + 0] = fl0 + xi * gx * gg.invh[0];
        a.out.forces[3 * (size_t)ia + 1] = fl1 + xi * gy * gg.invh[1];
        a.out.forces[3 * (size_t)ia + 2] = fl2 + xi * gz * gg.invh[2];
      }
      if (a.out.potential) a.out.potential[ia] = utot;
      if (a.out.dE_dc6) a.out.dE_dc6[ia] = -(utot - a.cself * xi) / (2.0 * xi);
      su += xi * utot;
      sxx += xi * xi;
    }
    __syncthreads();
    energy_partials(su, sxx, a.partial, b);
  }
};

// Lorentz-Berthelot: the grid potential of vector 6 - k weighted with
// xi_{i,k} = sigma_i^k sqrt(binom(6,k)) e_i / 8 (e_i = sqrt(2 eps_i) = xs.w),
// summed over k; the local part is e_i e0_i with e0 from the pair kernel; the
// self term is C_ii = e_i^2 sigma_i^6.
template <int P>
struct InterpLb {
  using Args = InterpLbArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const GridGeom& gg = a.gg;
    const int s = blk * kBlock + threadIdx.x;
    double su = 0.0, sxx = 0.0;
    if (s < a.n) {
      const double4 p = a.xs[s];
      double w[3][P], dw[3][P];
      int idx[3][P];
      interp_setup<P, double>(p, gg, w, dw, idx);
      const double sg = a.sig[s];
      double phi = 0.0, fx = 0.0, fy = 0.0, fz = 0.0, sk = 1.0;
      for (int k = 0; k <= 6; ++k) {
        const int binom = k == 0 || k == 6 ? 1 : (k == 1 || k == 5 ? 6 : (k == 2 || k == 4 ? 15 : 20));
        const double xik = sk * sqrt((double)binom) * p.w * 0.125;
        double u, gx, gy, gz;
        interp_grid<P, double>(a.E1[6 - k], gg, w, dw, idx, u, gx, gy, gz);
        phi += xik * u;
        fx += xik * gx;
        fy += xik * gy;
        fz += xik * gz;
        sk *= sg;
      }
      const int i = a.perm[s];
      if (a.forces) {
        a.forces[3 * (size_t)i + 0] = a.floc[3 * (size_t)s + 0] + fx * gg.invh[0];
        a.forces[3 * (size_t)i + 1] = a.floc[3 * (size_t)s + 1] + fy * gg.invh[1];
        a.forces[3 * (size_t)i + 2] = a.floc[3 * (size_t)s + 2] + fz * gg.invh[2];
      }
      su = p.w * a.e0[s] + phi;
      const double s3 = sg * sg * sg;
      sxx = p.w * p.w * s3 * s3;
    }
    energy_partials(su, sxx, a.partial, blk);
  }
};

struct EnergyFinal {
  using Args = EnergyArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int) {
    __shared__ double r1[kBlock], r2[kBlock], r3[kBlock];
    double x = 0.0, y = 0.0, z = 0.0;
    for (int i = threadIdx.x; i < a.nb; i += kBlock) {
      x += a.partial[2 * i];
      y += a.partial[2 * i + 1];
    }
    {
      // up to n / 64 block sums of the pair kernel: eight loads in flight
      double zz[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int i = threadIdx.x;
      for (; i + 7 * kBlock < a.rep_nb; i += 8 * kBlock)
#pragma unroll
        for (int u = 0; u < 8; ++u) zz[u] += a.rep_partial[i + u * kBlock];
      for (; i < a.rep_nb; i += kBlock) zz[0] += a.rep_partial[i];
      z = ((zz[0] + zz[1]) + (zz[2] + zz[3])) + ((zz[4] + zz[5]) + (zz[6] + zz[7]));
    }
    r1[threadIdx.x] = x;
    r2[threadIdx.x] = y;
    r3[threadIdx.x] = z;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        r1[threadIdx.x] += r1[threadIdx.x + off];
        r2[threadIdx.x] += r2[threadIdx.x + off];
        r3[threadIdx.x] += r3[threadIdx.x + off];
      }
      __syncthreads();
    }
    // dispersion (Sec. II.B) plus, from the MD entry points, the repulsion
    if (threadIdx.x == 0) {
      const double E = -0.5 * (r1[0] - a.cself * r2[0]) + 0.5 * r3[0];
      *a.energy = a.add ? *a.energy + E : E;
    }
  }
};

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
    // atoms within (half + 1) grid spacings of the owned range, plus the
    // skin margin by which an atom may sit outside its cell
    const double hw = P->cg.L[d] / n;
    ag.nh[d] = (int)std::ceil(((half + 1) * hw + P->cg.margin) / P->cg.w[d] - 1e-12);
    const int span = cb + 2 * ag.nh[d];
    // rows along x split at every periodic wrap
    segs *= (d == 0 ? std::min(span, (span + nc - 1) / nc + 1) : span);
  }
  return segs <= kMaxSeg;
}

bool ant_tiles_build(const mls_plan_s* P, AntTiles& T, std::vector<int>& tab, size_t& scratch, int cap) {
  const GridGeom gg = finest_geom(P);
  const CellGeom& cg = P->cg;
  const int half = P->order / 2;
  int cmax = std::min(cg.nc[0], std::min(cg.nc[1], cg.nc[2]));
  for (int cb = std::max(cmax, 1); cb >= 1; --cb) {
    std::vector<int> c[3], e[3], len[3];
    int maxlen[3] = {0, 0, 0}, maxc[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
      const int nc = cg.nc[d];
      const int nb = (nc + cb - 1) / cb;
      for (int b = 0; b <= nb; ++b) c[d].push_back((int)((int64_t)b * nc / nb));
      for (int b = 0; b < nb; ++b) {
        // finest points reached by atoms with c0 w <= x < c1 w: floor(x/h) in
        // [lo, hi], taps floor(x/h) - (p/2 - 1) .. floor(x/h) + p/2
        // (widened by the skin margin: atoms may sit that far outside their cells)
        const double t0 = (c[d][b] * cg.w[d] - cg.margin) * gg.invh[d];
        const double t1 = (c[d][b + 1] * cg.w[d] + cg.margin) * gg.invh[d];
        const int lo = (int)std::floor(t0 - 1e-7), hi = (int)std::floor(t1 + 1e-7);
        e[d].push_back(lo - (half - 1));
        len[d].push_back(hi - lo + P->order);
        // the interpolation tile wraps reached indices with one conditional
        // add or subtract: they must lie in [-n, 2n)
        if (e[d].back() < -gg.n[d] || e[d].back() + len[d].back() > 2 * gg.n[d]) return false;
        maxlen[d] = std::max(maxlen[d], len[d].back());
        maxc[d] = std::max(maxc[d], c[d][b + 1] - c[d][b]);
      }
    }
    if ((int64_t)maxlen[0] * maxlen[1] * maxlen[2] > cap || maxc[1] * maxc[2] > kAntTileRows) continue;
    // tables
    tab.clear();
    for (int d = 0; d < 3; ++d) {
      const int nb = (int)e[d].size();
      T.nb[d] = nb;
      T.off_c[d] = (int)tab.size();
      tab.insert(tab.end(), c[d].begin(), c[d].end());
      T.off_e[d] = (int)tab.size();
      tab.insert(tab.end(), e[d].begin(), e[d].end());
      T.off_len[d] = (int)tab.size();
      tab.insert(tab.end(), len[d].begin(), len[d].end());
      T.off_x0[d] = (int)tab.size();
      int x0 = 0;
      for (int b = 0; b < nb; ++b) {
        tab.push_back(x0);
        x0 += len[d][b];
      }
      T.NX[d] = x0;
    }
    for (int d = 0; d < 3; ++d) {
      while (tab.size() % 4) tab.push_back(0);
      T.off_cov[d] = (int)tab.size();
      const int n = gg.n[d];
      for (int m = 0; m < n; ++m) {
        int cov[4] = {-1, -1, -1, -1}, k = 0;
        for (int b = 0; b < T.nb[d]; ++b)
          for (int img = -2; img <= 2; ++img) {
            const int l = m + img * n - e[d][b];
            if (l >= 0 && l < len[d][b]) {
              if (k == 4) return false;
              cov[k++] = tab[T.off_x0[d] + b] + l;
            }
          }
        tab.insert(tab.end(), cov, cov + 4);
      }
    }
    scratch = (size_t)T.NX[0] * T.NX[1] * T.NX[2];
    return true;
  }
  return false;
}

template <int CAP>
hipError_t launch_ant_tile(int order, bool mixed, const AnterpTileArgs& t, int nb, hipStream_t s) {
  if (order == 4)
    return mixed ? launch_one<AnterpTile<4, float, CAP>>(t, nb, s) : launch_one<AnterpTile<4, double, CAP>>(t, nb, s);
  return mixed ? launch_one<AnterpTile<6, float, CAP>>(t, nb, s) : launch_one<AnterpTile<6, double, CAP>>(t, nb, s);
}

template <int CAP>
hipError_t launch_interp_tile(int order, bool mixed, const InterpTileArgs& t, int nb, hipStream_t s) {
  if (order == 4)
    return mixed ? launch_one<InterpTile<4, float, CAP>>(t, nb, s) : launch_one<InterpTile<4, double, CAP>>(t, nb, s);
  return mixed ? launch_one<InterpTile<6, float, CAP>>(t, nb, s) : launch_one<InterpTile<6, double, CAP>>(t, nb, s);
}

hipError_t launch_anterpolate(mls_plan_s* P, int n, hipStream_t s) {
  Level& L1 = P->lv[0];
  if (P->ant_tiles) {
    double* scratch = P->ant_scratch ? P->ant_scratch : P->d_ant_scratch;
    AnterpTileArgs t{P->d_xs, P->d_cell_start, P->cg, finest_geom(P), P->ant, P->d_ant_tab, scratch, P->charge,
                     P->d_flags};
    const int nb = P->ant.nb[0] * P->ant.nb[1] * P->ant.nb[2];
    const bool mixed = P->precision == MLS_MIXED;
    hipError_t e;
    if (P->ant_cap == kAntTileSmall) e = launch_ant_tile<kAntTileSmall>(P->order, mixed, t, nb, s);
    else e = launch_ant_tile<kAntTileMax>(P->order, mixed, t, nb, s);
    if (e != hipSuccess) return e;
    AnterpCollectArgs c{P->ant, P->d_ant_tab, scratch, L1.q, L1.g};
    return launch_one<AnterpCollect>(c, nblocks(L1.g.size, kBlock), s);
  }
  AnterpArgs a{P->d_xs, P->d_cell_start, n, P->cg, finest_geom(P), AntGeom{}, L1.q, P->charge};
  if (anterp_owned_geom(P, a.ag)) {
    // every owned point is written, so no zero fill is needed
    const int nb = a.ag.nb[0] * a.ag.nb[1] * a.ag.nb[2];
    const bool mixed = P->precision == MLS_MIXED;
    if (P->order == 4 && !mixed) return launch_one<AnterpOwned<4, double>>(a, nb, s);
    if (P->order == 4) return launch_one<AnterpOwned<4, float>>(a, nb, s);
    if (!mixed) return launch_one<AnterpOwned<6, double>>(a, nb, s);
    return launch_one<AnterpOwned<6, float>>(a, nb, s);
  }
  hipError_t e = launch_zero(L1.q, L1.g.size, s);
  if (e != hipSuccess || n == 0) return e;
  if (P->order == 4) return launch_one<AnterpAtomic<4>>(a, nblocks(n, kBlock), s);
  return launch_one<AnterpAtomic<6>>(a, nblocks(n, kBlock), s);
}

hipError_t launch_prolong_into(mls_plan_s* P, const TransferArgs& a, hipStream_t s);

hipError_t launch_restrictions(mls_plan_s* P, hipStream_t s) {
  for (int k = 2; k <= P->levels; ++k) {
    hipError_t e = launch_restrict(P, k - 1, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_prolongations(mls_plan_s* P, hipStream_t s, bool drop_e1) {
  for (int k = P->levels - 1; k >= 1; --k) {
    hipError_t e;
    if (k == 1 && drop_e1) {
      Level& F = P->lv[0];
      Level& C = P->lv[1];
      e = launch_prolong_into(P, TransferArgs{C.E, C.g, nullptr, F.E, F.g}, s);
    } else {
      e = launch_prolong(P, k, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_restrict(mls_plan_s* P, int k_fine, hipStream_t s) {
  Level& F = P->lv[k_fine - 1];
  Level& C = P->lv[k_fine];
  TransferArgs a{F.q, F.g, nullptr, C.q, C.g};
  if (C.g.size <= P->split_restrict) {
    const int nb = nblocks((int64_t)C.g.size * kRestrictGroup, kBlock);
    return P->order == 4 ? launch_one<RestrictSplit<4>>(a, nb, s) : launch_one<RestrictSplit<6>>(a, nb, s);
  }
  if (P->order == 4) return launch_one<Restrict<4>>(a, nblocks(C.g.size, kBlock), s);
  return launch_one<Restrict<6>>(a, nblocks(C.g.size, kBlock), s);
}

hipError_t launch_prolong_into(mls_plan_s* P, const TransferArgs& a, hipStream_t s) {
  if (a.gs.size <= P->split_prolong) {
    if (P->order == 4) return launch_one<ProlongSplit<4>>(a, nblocks((int64_t)a.gs.size * ProlongSplit<4>::G, kBlock), s);
    return launch_one<ProlongSplit<6>>(a, nblocks((int64_t)a.gs.size * ProlongSplit<6>::G, kBlock), s);
  }
  if (P->order == 4) return launch_one<Prolong<4>>(a, nblocks(a.gs.size, kBlock), s);
  return launch_one<Prolong<6, true>>(a, nblocks(a.gs.size, kBlock), s);
}

hipError_t launch_prolong(mls_plan_s* P, int k_fine, hipStream_t s) {
  Level& F = P->lv[k_fine - 1];
  Level& C = P->lv[k_fine];
  return launch_prolong_into(P, TransferArgs{C.E, C.g, F.e, F.E, F.g}, s);
}

hipError_t launch_interpolate(mls_plan_s* P, int n, double* energy, double* forces, double* potential,
                              double* dE_dc6, hipStream_t s, int mode) {
  const bool with_repulsion = (mode & kInterpRep) != 0;
  int nb = nblocks(n, kBlock);
  if (n > 0) {
    InterpArgs a{P->d_xs, P->d_perm, n, finest_geom(P), (mode & kInterpLevel1) ? P->lv[0].e : P->lv[0].E,
                 P->d_e0, P->d_floc, P->cself, OutPtrs{forces, potential, dE_dc6}, P->d_partial};
    if (with_repulsion) a.frep = P->d_frep;
    a.grid_only = (mode & kInterpGridOnly) ? 1 : 0;
    const bool mixed = P->precision == MLS_MIXED;
    const int nt = P->ant.nb[0] * P->ant.nb[1] * P->ant.nb[2];
    hipError_t e;
    if (P->ant_tiles && nt <= P->n_partial + 1) {
      // the anterpolation's cell blocks, their finest-grid reach staged in LDS
      // (one energy partial per block)
      InterpTileArgs t{a, P->d_cell_start, P->cg, P->ant, P->d_ant_tab, P->d_flags};
      nb = nt;
      if (P->ant_cap == kAntTileSmall) e = launch_interp_tile<kAntTileSmall>(P->order, mixed, t, nt, s);
      else e = launch_interp_tile<kAntTileMax>(P->order, mixed, t, nt, s);
    } else if (P->order == 4 && !mixed) {
      e = launch_one<Interp<4, double>>(a, nb, s);
    } else if (P->order == 4) {
      e = launch_one<Interp<4, float>>(a, nb, s);
    } else if (!mixed) {
      e = launch_one<Interp<6, double>>(a, nb, s);
    } else {
      e = launch_one<Interp<6, float>>(a, nb, s);
    }
    if (e != hipSuccess) return e;
  }
  // no atoms: an empty sum, E = 0
  EnergyArgs ea{P->d_partial, nb, (mode & kInterpNoSelf) ? 0.0 : P->cself, energy};
  if (with_repulsion) {
    ea.rep_partial = P->d_md_partial;
    ea.rep_nb = n > 0 ? P->rep_nb : 0;
  }
  ea.add = (mode & kInterpGridOnly) ? 1 : 0;
  return launch_one<EnergyFinal>(ea, 1, s);
}

hipError_t launch_interpolate_lb(mls_plan_s* P, int n, double* energy, double* forces, hipStream_t s) {
  const int nb = nblocks(n, kBlock);
  if (n > 0) {
    InterpLbArgs a{P->d_xs, P->d_sig, P->d_perm, n, finest_geom(P), {}, P->d_e0, P->d_floc, forces, P->d_partial};
    for (int k = 0; k < 7; ++k) a.E1[k] = P->lb_lv[k][0].E;
    hipError_t e = P->order == 4 ? launch_one<InterpLb<4>>(a, nb, s) : launch_one<InterpLb<6>>(a, nb, s);
    if (e != hipSuccess) return e;
  }
  return launch_one<EnergyFinal>(EnergyArgs{P->d_partial, nb, P->cself, energy}, 1, s);
}

// Batched phases of this file; variant = order | 0x100 for FP32 weights.
hipError_t launch_batched_grid(const BatchPhase& ph, hipStream_t s) {
  const bool p6 = (ph.variant & 0xff) == 6, mixed = (ph.variant & 0x100) != 0;
  switch (ph.kernel) {
    case BK_ANT_ATOMIC:
      return p6 ? launch_batched_phase<AnterpAtomic<6>>(ph, s) : launch_batched_phase<AnterpAtomic<4>>(ph, s);
    case BK_ANT_OWNED:
      if (p6) return mixed ? launch_batched_phase<AnterpOwned<6, float>>(ph, s)
                           : launch_batched_phase<AnterpOwned<6, double>>(ph, s);
      return mixed ? launch_batched_phase<AnterpOwned<4, float>>(ph, s)
                   : launch_batched_phase<AnterpOwned<4, double>>(ph, s);
    case BK_ANT_TILE:
      if (p6) return mixed ? launch_batched_phase<AnterpTile<6, float>>(ph, s)
                           : launch_batched_phase<AnterpTile<6, double>>(ph, s);
      return mixed ? launch_batched_phase<AnterpTile<4, float>>(ph, s)
                   : launch_batched_phase<AnterpTile<4, double>>(ph, s);
    case BK_ANT_COLLECT: return launch_batched_phase<AnterpCollect>(ph, s);
    case BK_RESTRICT:
      return p6 ? launch_batched_phase<Restrict<6>>(ph, s) : launch_batched_phase<Restrict<4>>(ph, s);
    case BK_PROLONG:
      return p6 ? launch_batched_phase<Prolong<6, true>>(ph, s) : launch_batched_phase<Prolong<4, true>>(ph, s);
    case BK_INTERP:
      if (p6) return mixed ? launch_batched_phase<Interp<6, float>>(ph, s)
                           : launch_batched_phase<Interp<6, double>>(ph, s);
      return mixed ? launch_batched_phase<Interp<4, float>>(ph, s) : launch_batched_phase<Interp<4, double>>(ph, s);
    case BK_ENERGY: return launch_batched_phase<EnergyFinal>(ph, s);
    case BK_INTERP_LB: return p6 ? launch_batched_phase<InterpLb<6>>(ph, s) : launch_batched_phase<InterpLb<4>>(ph, s);
    default: return hipErrorInvalidValue;
  }
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
