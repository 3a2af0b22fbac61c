// Evaluation on the grids (eq:evaluation, k = 1..l):
//   levels k < l:  e^k[mu] = 2^(-6(k-1)) sum_{delta: |delta o h_1| < 2a} g_1(|delta o h_1|) q^k[(mu - delta) mod n_k]
//                  (the cutoff 2^k a and spacing 2^(k-1) h_1 give the same offsets on every level and
//                  g_k(2^(k-1) s) = 2^(-6(k-1)) g_1(s), Sec. II.A.4)
//   level l:       e^l[mu] = sum_nu K_l[(mu - nu) mod n_l] q^l[nu]   with the pre-summed periodic kernel of
//                  eq:last-grid-periodic-transformed (all-to-all, FP64).
//
// Level stencil kernel (k_stencil_stream): a block owns a TX x TY column of
// output points and a chunk of ZC planes.  It streams input planes z through
// LDS (one xy plane plus an R-wide periodic halo at a time).  For every tap
// column (|dx|,|dy|) the up to four mirror images q[x+-dx, y+-dy] are summed
// once and then applied to the 2 hz + 1 outputs z_in - hz .. z_in + hz held
// in a rolling register window acc[0..2R]; after each plane the oldest output
// is complete, written, and the window shifts.
#include <algorithm>

#include "device_math.h"
#include "mls_internal.h"

namespace mls {

int stencil_window(const mls_plan_s* P);

namespace {

constexpr int kBlock = 256;

// Reference-structured stencil: one thread per output point, taps from the
// level-1 table (used for halos wider than the instantiated window).
__global__ void __launch_bounds__(kBlock) k_stencil_taps_f64(const double* __restrict__ q, GridDims g,
                                                             const Tap* __restrict__ taps, int ntaps, double scale,
                                                             double* __restrict__ e) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= g.size) return;
  const int x = mu % g.n[0], y = (mu / g.n[0]) % g.n[1], z = mu / (g.n[0] * g.n[1]);
  double acc = 0.0;
  for (int t = 0; t < ntaps; ++t) {
    const Tap tp = taps[t];
    const int sx = wrapi(x - tp.dx, g.n[0]);
    const int sy = wrapi(y - tp.dy, g.n[1]);
    const int sz = wrapi(z - tp.dz, g.n[2]);
    acc += tp.w * q[((size_t)sz * g.n[1] + sy) * g.n[0] + sx];
  }
  e[mu] = scale * acc;
}

// Apply one tap column with half height hz (compile-time) to the window.
template <class T, int R, int HZ>
__device__ __forceinline__ void apply_column(T (&acc)[2 * R + 1], T s, const T* __restrict__ w) {
  acc[R] += w[0] * s;
#pragma unroll
  for (int d = 1; d <= HZ; ++d) {
    const T wd = w[d] * s;
    acc[R + d] += wd;
    acc[R - d] += wd;
  }
}

template <class T, int R, int H = 0>
__device__ __forceinline__ void apply_switch(int hz, T (&acc)[2 * R + 1], T s, const T* __restrict__ w) {
  if constexpr (H <= R) {
    if (hz == H) {
      apply_column<T, R, H>(acc, s, w);
      return;
    }
    apply_switch<T, R, H + 1>(hz, acc, s, w);
  }
}

// W waves share one 8 x 8 output column and one LDS plane; wave w applies
// the tap columns [wave_rows[w], wave_rows[w+1]) (balanced by cost on the
// host) and the W partial sums of each finished output are added in LDS.
// The wrapped halo offsets of the plane are computed once per block, and the
// next plane is prefetched into registers while the current one is used.
template <class T, int R, int W>
__global__ void __launch_bounds__(64 * W) k_stencil_stream(const T* __restrict__ q, GridDims g,
                                                           const StencilRow* __restrict__ rows,
                                                           const int* __restrict__ wave_rows,
                                                           const T* __restrict__ wts, T scale, int zc,
                                                           T* __restrict__ e) {
  constexpr int TX = 8, TY = 8;
  constexpr int SX = TX + 2 * R, SY = TY + 2 * R, NP = SX * SY, NT = 64 * W;
  constexpr int PER = (NP + NT - 1) / NT;
  __shared__ T plane[NP];
  __shared__ T red[W][64];
  const int tid = threadIdx.x, lane = tid & 63;
  // wave index made provably uniform: row and weight reads become scalar
  // loads and the hz dispatch scalar branches
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tx = lane & 7, ty = lane >> 3;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int z0 = blockIdx.z * zc;
  const int zend = min(z0 + zc, g.n[2]);
  const int x = x0 + tx, y = y0 + ty;
  const bool owner = x < g.n[0] && y < g.n[1];
  const size_t pstride = (size_t)g.n[0] * g.n[1];
  int off[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = tid + k * NT;
    const int lx = i % SX, ly = i / SX;
    off[k] = i < NP ? wrapi(y0 - R + ly, g.n[1]) * g.n[0] + wrapi(x0 - R + lx, g.n[0]) : 0;
  }
  const int r0 = wave_rows[wv], r1 = wave_rows[wv + 1];
  T acc[2 * R + 1];
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) acc[k] = T(0);
  T pre[PER];
  {
    const T* src = q + (size_t)wrapi(z0 - R, g.n[2]) * pstride;
#pragma unroll
    for (int k = 0; k < PER; ++k) pre[k] = src[off[k]];
  }
  const T* c = plane + (ty + R) * SX + (tx + R);
  for (int zin = z0 - R; zin < zend + R; ++zin) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (tid + k * NT < NP) plane[tid + k * NT] = pre[k];
    __syncthreads();
    if (zin + 1 < zend + R) {
      const T* src = q + (size_t)wrapi(zin + 1, g.n[2]) * pstride;
#pragma unroll
      for (int k = 0; k < PER; ++k) pre[k] = src[off[k]];
    }
    for (int r = r0; r < r1; ++r) {
      const StencilRow row = rows[r];
      T s;
      if (row.dx == 0 && row.dy == 0) {
        s = c[0];
      } else if (row.dx == 0) {
        s = c[-row.dy * SX] + c[row.dy * SX];
      } else if (row.dy == 0) {
        s = c[-row.dx] + c[row.dx];
      } else {
        s = (c[-row.dy * SX - row.dx] + c[-row.dy * SX + row.dx]) + (c[row.dy * SX - row.dx] + c[row.dy * SX + row.dx]);
      }
      apply_switch<T, R>(row.hz, acc, s, wts + row.woff);
    }
    // output z = zin - R is complete: add the W partial sums
    red[wv][lane] = acc[0];
    __syncthreads();
    const int zout = zin - R;
    if (wv == 0 && owner && zout >= z0 && zout < zend) {
      T sum = red[0][lane];
#pragma unroll
      for (int w = 1; w < W; ++w) sum += red[w][lane];
      e[(size_t)zout * pstride + (size_t)y * g.n[0] + x] = scale * sum;
    }
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) acc[k] = acc[k + 1];
    acc[2 * R] = T(0);
  }
}

// ---------------------------------------------------------------------------
// Tiled level stencil.  A block owns an 8 x 8 x ZC box of output points of
// one level (all levels share one launch through a tile table).  It loads the
// box plus an R-wide periodic halo into LDS once.  Its W waves split the tap
// columns (|dx|,|dy|); for each column the wave reads the column's weights
// once and runs a fully unrolled loop over the ZC + 2 hz input planes: the
// four mirror images q[x+-dx, y+-dy] are summed (on the axes the duplicate
// images are compensated by weights pre-divided on the host) and added with
// weight w[|dz|] into all ZC outputs held in registers.  The W partial sums
// are added in LDS at the end.
}  // namespace

// z extent of a single plan's stencil tile for halo window R: 16 for FP32
// tiles up to R = 6, else 8 (an FP64 tile of depth 16 takes (8 + 2R)^2 (16 +
// 2R) doubles, 90 KB at R = 6: one block per CU; at depth 8, 64 KB: two)
constexpr int tile_zc(int R, bool f64) { return R <= 6 && !f64 ? 16 : 8; }

int stencil_tile_zc(int R, bool f64) { return tile_zc(R, f64); }

namespace {

struct StencilLaunch {
  StencilLevel lv[16];
  int nlev;
};

template <class T, int HZ, int ZC>
__device__ __forceinline__ void tile_column(T (&acc)[ZC], const T* __restrict__ c, int o0, int o1, int o2, int o3,
                                            int pstride, const T* __restrict__ w) {
  T wr[HZ + 1];
#pragma unroll
  for (int d = 0; d <= HZ; ++d) wr[d] = w[d];
#pragma unroll
  for (int zi = -HZ; zi < ZC + HZ; ++zi) {
    const T* p = c + zi * pstride;
    const T s = (p[o0] + p[o1]) + (p[o2] + p[o3]);
#pragma unroll
    for (int dz = -HZ; dz <= HZ; ++dz) {
      const int zo = zi + dz;
      if (zo >= 0 && zo < ZC) acc[zo] += wr[dz < 0 ? -dz : dz] * s;
    }
  }
}

template <class T, int R, int ZC, int H = 0>
__device__ __forceinline__ void tile_switch(int hz, T (&acc)[ZC], const T* c, int o0, int o1, int o2, int o3,
                                            int pstride, const T* w) {
  if constexpr (H <= R) {
    if (hz == H) {
      tile_column<T, H, ZC>(acc, c, o0, o1, o2, o3, pstride, w);
      return;
    }
    tile_switch<T, R, ZC, H + 1>(hz, acc, c, o0, o1, o2, o3, pstride, w);
  }
}

// FP32 tiles hold q - mean (mean = sum_i xi / points, the exact mean by the
// partition of unity); the constant part adds back as mean * sum of weights,
// since a periodic convolution maps a constant c to c times the weight sum.
template <class T, int R, int ZC, int W>
__device__ __forceinline__ void stencil_tile(const StencilLevel& V, const int4 tinfo) {
  constexpr int SX = 8 + 2 * R, SY = 8 + 2 * R, SZ = ZC + 2 * R;
  constexpr int PS = SX * SY, NP = PS * SZ, NT = 64 * W;
  // the tile doubles as the reduction buffer of the W partial sums
  constexpr int NL = NP > W * ZC * 64 ? NP : W * ZC * 64;
  __shared__ T tile[NL];
  __shared__ int wrapx[SX], wrapy[SY], wrapz[SZ];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int x0 = tinfo.y * 8, y0 = tinfo.z * 8, z0 = tinfo.w * ZC;
  if (tid < SX) wrapx[tid] = wrapi(x0 - R + tid, V.n[0]);
  if (tid < SY) wrapy[tid] = wrapi(y0 - R + tid, V.n[1]);
  if (tid < SZ) wrapz[tid] = wrapi(z0 - R + tid, V.n[2]);
  __syncthreads();
  const size_t gps = (size_t)V.n[0] * V.n[1];
  const double* __restrict__ q = V.q;
  const double mean = sizeof(T) < sizeof(double) ? *V.sum_xi * V.inv_size : 0.0;
  // the fill issues kFill global loads per thread before it waits for them
  // (one load per wait leaves the block waiting on memory latency NP / NT
  // times); indexes past the box are clamped, so every load is in range
  constexpr int kIters = (NP + NT - 1) / NT, kFill = 8;
  for (int b0 = 0; b0 < kIters; b0 += kFill) {
    double v[kFill];
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int i = min(tid + (b0 + u) * NT, NP - 1);
      const int lx = i % SX, ly = (i / SX) % SY, lz = i / PS;
      v[u] = q[(size_t)wrapz[lz] * gps + (size_t)wrapy[ly] * V.n[0] + wrapx[lx]];
    }
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int i = tid + (b0 + u) * NT;
      if (i < NP) tile[i] = (T)(v[u] - mean);
    }
  }
  __syncthreads();
  // lanes 0-31 take the even rows, 32-63 the odd ones: with a row pitch of
  // 20 words (R = 6) each half-wave's four rows then cover disjoint banks
  const int tx = lane & 7, ty = ((lane >> 3) & 3) * 2 + (lane >> 5);
  const T* c = tile + R * PS + (ty + R) * SX + (tx + R);
  T acc[ZC];
#pragma unroll
  for (int k = 0; k < ZC; ++k) acc[k] = T(0);
  // the column index is wave-uniform, so the rows and weights are scalar
  // loads (staging them in LDS measured slower)
  const StencilRow* __restrict__ rows = V.rows;
  const T* __restrict__ wts = (const T*)V.wts;
  const int r0 = V.wave_rows[wv], r1 = V.wave_rows[wv + 1];
  for (int r = r0; r < r1; ++r) {
    const StencilRow row = rows[r];
    const int o0 = -row.dy * SX - row.dx, o1 = -row.dy * SX + row.dx;
    const int o2 = row.dy * SX - row.dx, o3 = row.dy * SX + row.dx;
    tile_switch<T, R, ZC>(row.hz, acc, c, o0, o1, o2, o3, PS, wts + row.woff);
  }
  // add the W partial sums (the tile is reused as the reduction buffer)
  __syncthreads();
#pragma unroll
  for (int k = 0; k < ZC; ++k) tile[(wv * ZC + k) * 64 + lane] = acc[k];
  __syncthreads();
  const int x = x0 + tx, y = y0 + ty;
  if (x < V.n[0] && y < V.n[1]) {
    for (int k = wv; k < ZC; k += W) {
      const int z = z0 + k;
      if (z >= V.n[2]) break;
      T sum = tile[k * 64 + lane];
#pragma unroll
      for (int w2 = 1; w2 < W; ++w2) sum += tile[(w2 * ZC + k) * 64 + lane];
      V.e[(size_t)z * gps + (size_t)y * V.n[0] + x] = V.scale * ((double)sum + mean * V.wsum);
    }
  }
}

// One plan: all levels of the plan in one launch, level descriptors by value.
template <class T, int R, int ZC, int W>
__global__ void __launch_bounds__(64 * W) k_stencil_tile(StencilLaunch L, const int4* __restrict__ tiles) {
  const int4 tinfo = tiles[xcd_block(blockIdx.x, gridDim.x)];
  stencil_tile<T, R, ZC, W>(L.lv[tinfo.x], tinfo);
}

// MFMA recast of the FP32 tile (window R <= 6, 8 x 8 x 16 outputs per block).
// For one tap column (dx, dy) the z sum is a banded Toeplitz product:
// e[z][xy] += sum_t A[z][t] B[t][xy] with A[z][t] = w(|t - hz - z|) (input
// plane t counted from hz below the tile) and B[t][xy] the four mirror
// images q[x -+ dx, y -+ dy] of plane t summed, as in the VALU tile.  Each
// v_mfma_f32_16x16x4_f32 takes 16 output planes (M), 16 xy points (N) and
// four input planes (K): a column needs S = ceil((16 + 2 hz) / 4) chunks for
// each of the tile's four 16-point xy blocks.  The A operands come from a
// host table (one coalesced load per chunk, shared by the four blocks); B is
// folded from LDS.  The W waves split the columns and add their partial
// tiles in LDS, as the VALU tile does.  Operand layouts (lane = row + 16 *
// column of A, column + 16 * row of B; D[i][j] in lane j + 16 (i / 4),
// register i % 4) were checked on the device.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int R, int HZ>
__device__ __forceinline__ void mfma_column(mfma_f4 (&acc)[4], const float* __restrict__ tile, const int (&base)[4],
                                            int o0, int o1, int o2, int o3, const float* __restrict__ at) {
  constexpr int SX = 8 + 2 * R, PS = SX * SX;
  constexpr int S = (16 + 2 * HZ + 3) / 4;
#pragma unroll
  for (int sc = 0; sc < S; ++sc) {
    const float a = at[64 * sc];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const float* p = tile + base[nb] + 4 * sc * PS;
      const float b = (p[o0] + p[o1]) + (p[o2] + p[o3]);
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[nb], 0, 0, 0);
    }
  }
}

template <int R, int H = 0>
__device__ __forceinline__ void mfma_switch(int hz, mfma_f4 (&acc)[4], const float* tile, int (&base)[4], int o0,
                                            int o1, int o2, int o3, const float* at) {
  if constexpr (H <= R) {
    if (hz == H) {
      constexpr int SX = 8 + 2 * R, PS = SX * SX;
      // chunk 0 starts hz planes below the tile's first output plane
      int b[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) b[nb] = base[nb] + (R - H) * PS;
      mfma_column<R, H>(acc, tile, b, o0, o1, o2, o3, at);
      return;
    }
    mfma_switch<R, H + 1>(hz, acc, tile, base, o0, o1, o2, o3, at);
  }
}

template <int R, int W>
__global__ void __launch_bounds__(64 * W) k_stencil_mfma(StencilLaunch L, const int4* __restrict__ tiles) {
  constexpr int ZC = 16;
  // four zero planes above the halo: the last K chunk of a column may reach
  // up to three planes past its band
  constexpr int SX = 8 + 2 * R, SY = 8 + 2 * R, SZH = ZC + 2 * R, SZ = SZH + 4;
  constexpr int PS = SX * SY, NP = PS * SZ, NT = 64 * W;
  constexpr int NL = NP > W * ZC * 64 ? NP : W * ZC * 64;
  __shared__ float tile[NL];
  __shared__ int wrapx[SX], wrapy[SY], wrapz[SZH];
  const int4 tinfo = tiles[xcd_block(blockIdx.x, gridDim.x)];
  const StencilLevel& V = L.lv[tinfo.x];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int x0 = tinfo.y * 8, y0 = tinfo.z * 8, z0 = tinfo.w * ZC;
  if (tid < SX) wrapx[tid] = wrapi(x0 - R + tid, V.n[0]);
  if (tid < SY) wrapy[tid] = wrapi(y0 - R + tid, V.n[1]);
  if (tid < SZH) wrapz[tid] = wrapi(z0 - R + tid, V.n[2]);
  __syncthreads();
  const size_t gps = (size_t)V.n[0] * V.n[1];
  const double* __restrict__ q = V.q;
  const double mean = *V.sum_xi * V.inv_size;
  constexpr int kIters = (NP + NT - 1) / NT, kFill = 8;
  for (int b0 = 0; b0 < kIters; b0 += kFill) {
    double v[kFill];
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int i = min(tid + (b0 + u) * NT, NP - 1);
      const int lx = i % SX, ly = (i / SX) % SY, lz = min(i / PS, SZH - 1);
      v[u] = q[(size_t)wrapz[lz] * gps + (size_t)wrapy[ly] * V.n[0] + wrapx[lx]];
    }
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int i = tid + (b0 + u) * NT;
      if (i < NP) tile[i] = i < PS * SZH ? (float)(v[u] - mean) : 0.0f;
    }
  }
  __syncthreads();
  // B operand of lane (k = lane / 16, j = lane % 16): plane k of the chunk,
  // xy point j of block nb (x = j % 8, y = 2 nb + j / 8)
  const int kk = lane >> 4, j = lane & 15;
  int base[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) base[nb] = kk * PS + (2 * nb + (j >> 3) + R) * SX + ((j & 7) + R);
  mfma_f4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
  const StencilRow* __restrict__ rows = V.rows;
  const float* __restrict__ atab = (const float*)V.wts;
  const int r0 = V.wave_rows[wv], r1 = V.wave_rows[wv + 1];
  for (int r = r0; r < r1; ++r) {
    const StencilRow row = rows[r];
    const int o0 = -row.dy * SX - row.dx, o1 = -row.dy * SX + row.dx;
    const int o2 = row.dy * SX - row.dx, o3 = row.dy * SX + row.dx;
    mfma_switch<R>(row.hz, acc, tile, base, o0, o1, o2, o3, atab + row.woff + lane);
  }
  // add the W partial tiles (the tile is reused): D[i][j] of block nb is
  // output plane i = 4 (lane / 16) + register, xy point 16 nb + j
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) tile[(wv * ZC + 4 * kk + rg) * 64 + 16 * nb + j] = acc[nb][rg];
  __syncthreads();
  for (int o = tid; o < ZC * 64; o += NT) {
    const int z = o >> 6, xy = o & 63;
    const int x = x0 + (xy & 7), y = y0 + (xy >> 3), zz = z0 + z;
    if (x >= V.n[0] || y >= V.n[1] || zz >= V.n[2]) continue;
    float sum = 0.0f;
#pragma unroll
    for (int w2 = 0; w2 < W; ++w2) sum += tile[(w2 * ZC + z) * 64 + xy];
    V.e[(size_t)zz * gps + (size_t)y * V.n[0] + x] = V.scale * ((double)sum + mean * V.wsum);
  }
}

// Batched: tiles of many plans' levels; tinfo.x indexes the descriptor array.
template <class T, int R, int ZC, int W>
__global__ void __launch_bounds__(64 * W) k_stencil_tile_batched(const StencilLevel* __restrict__ lv,
                                                                 const int4* __restrict__ tiles, int ntiles) {
  for (int t = xcd_block(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x) {
    const int4 tinfo = tiles[t];
    stencil_tile<T, R, ZC, W>(lv[tinfo.x], tinfo);
    __syncthreads();
  }
}

// Coarsest level: all-to-all over the level (a periodic convolution of the
// charges with the pre-summed kernel K), with K and the charges staged in LDS
// when they fit (kCoarseLds points each).
//
// Rows path (batched launches), for a level whose x extent N is at most 8
// and whose staging fits: a lane owns one output row (y, z) and keeps its N sums in
// registers; the eight waves of the block split the source rows (y', z').
// Per source row a lane reads the N values of the kernel row
// ((y - y') mod n_y, (z - z') mod n_z) and the wave reads the N charges of
// the row (the same address in every lane), then the x-direction convolution
// of the two rows, N^2 FMAs with the (x - x') mod N offsets fixed at compile
// time, runs in registers.  Each K value read from LDS serves N FMAs.  The
// waves' partial rows are added in LDS in wave order (fixed order).  K rows
// sit at an odd stride in LDS so that the 8-byte reads of one wave spread
// over the banks.
//
// General path, for single plans and the levels the rows path does not
// take: a wave per output point (a.outs
// points per wave, one after another): the lanes split the source rows, each
// lane takes its (y - y', z - z') offset once per row and walks x' with
// (x - x') mod n_x, then the lanes add their partial sums across the wave
// (fixed order).
constexpr int kCoarseLds = 2048;
constexpr int kCoarseRowsMaxX = 8;

// One LDS buffer for either path, declared at namespace scope so that every
// access by name compiles to an LDS access (a pointer into it passed around
// could be taken for a generic one and read with flat loads).
__shared__ double coarse_lds[2 * kCoarseLds];

// x extent of a level the rows path takes, else 0
__host__ __device__ inline int coarse_rows_n(const GridDims& g) {
  const int N = g.n[0], nrow = g.n[1] * g.n[2];
  if (N < 1 || N > kCoarseRowsMaxX) return 0;
  return (int64_t)nrow * (N | 1) <= kCoarseLds && (int64_t)nrow * N <= kCoarseLds ? N : 0;
}

template <int N>
__device__ __forceinline__ void coarsest_rows(const CoarsestArgs& a, int blk) {
  constexpr int S = N | 1;   // LDS stride of a K row, in doubles
  constexpr int kPer = kCoarseLds / kCoarsestThreads;
  double* const sk = coarse_lds;
  double* const sq = coarse_lds + kCoarseLds;
  const int n1 = a.g.n[1], n2 = a.g.n[2], nrow = n1 * n2, npt = nrow * N;
  {
    // every load of the staging in flight before the first store
    double vq[kPer], vk[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = min((int)threadIdx.x + u * kCoarsestThreads, npt - 1);
      vq[u] = a.q[i];
      vk[u] = a.K[i];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = threadIdx.x + u * kCoarsestThreads;
      if (i < npt) {
        const int r = i / N;
        sk[r * S + (i - r * N)] = vk[u];
        sq[i] = vq[u];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = blk * 64 + lane;
  const int y = row < nrow ? row % n1 : 0, z = row < nrow ? row / n1 : 0;
  const int r0 = (nrow * wv) / kCoarsestWaves, r1 = (nrow * (wv + 1)) / kCoarsestWaves;
  double acc[N];
#pragma unroll
  for (int x = 0; x < N; ++x) acc[x] = 0.0;
  int ys = r0 % n1, zs = r0 / n1;
  for (int r = r0; r < r1; ++r) {
    const int ky = y - ys + (y < ys ? n1 : 0), kz = z - zs + (z < zs ? n2 : 0);
    const int kb = (kz * n1 + ky) * S;
    double k[N], q[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      k[j] = sk[kb + j];
      q[j] = sq[r * N + j];
    }
#pragma unroll
    for (int xs = 0; xs < N; ++xs)
#pragma unroll
      for (int x = 0; x < N; ++x) acc[x] = fma(k[(x - xs + N) % N], q[xs], acc[x]);
    if (++ys == n1) {
      ys = 0;
      ++zs;
    }
  }
  __syncthreads();   // staging no longer read: the buffer takes the partial rows
  double* const red = coarse_lds;
#pragma unroll
  for (int x = 0; x < N; ++x) red[(wv * N + x) * 64 + lane] = acc[x];
  __syncthreads();
  if (threadIdx.x < 64 * N) {
    const int x = threadIdx.x >> 6;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kCoarsestWaves; ++w) v += red[(w * N + x) * 64 + lane];
    if (row < nrow) a.e[row * N + x] = v;
  }
}

template <bool STAGED>
__device__ __forceinline__ void coarsest_sums(const CoarsestArgs& a, int blk) {
  const GridDims& g = a.g;
  double* const sk = coarse_lds;
  double* const sq = coarse_lds + kCoarseLds;
  if constexpr (STAGED) {
    constexpr int kPer = kCoarseLds / kCoarsestThreads;
    double vq[kPer], vk[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = min((int)threadIdx.x + u * kCoarsestThreads, g.size - 1);
      vq[u] = a.q[i];
      vk[u] = a.K[i];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = threadIdx.x + u * kCoarsestThreads;
      if (i < g.size) {
        sq[i] = vq[u];
        sk[i] = vk[u];
      }
    }
    __syncthreads();
  }
  const double* __restrict__ gK = a.K;
  const double* __restrict__ gq = a.q;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], n01 = n0 * n1, nrow = n1 * n2;
  const int b1 = 64 % n1, b2 = 64 / n1, ys0 = lane % n1, zs0 = lane / n1;
  for (int m = 0; m < a.outs; ++m) {
    const int mu = (blk * a.outs + m) * kCoarsestWaves + wv;
    if (mu >= g.size) break;
    const int x = mu % n0, y = (mu / n0) % n1, z = mu / n01;
    double acc = 0.0;
    // (ys, zs) of row r = lane + 64 t, advanced with a carry (no division
    // per row)
    int ys = ys0, zs = zs0;
    for (int r = lane; r < nrow; r += 64) {
      const int ky = y - ys + (y < ys ? n1 : 0), kz = z - zs + (z < zs ? n2 : 0);
      const int kr = kz * n01 + ky * n0, qr = r * n0;
#pragma unroll 4
      for (int xs = 0; xs < n0; ++xs) {
        const int kx = x - xs + (x < xs ? n0 : 0);
        if constexpr (STAGED) acc = fma(sk[kr + kx], sq[qr + xs], acc);
        else acc = fma(gK[kr + kx], gq[qr + xs], acc);
      }
      ys += b1;
      const int cy = ys >= n1;
      ys -= cy ? n1 : 0;
      zs += b2 + cy;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) a.e[mu] = acc;
  }
}

struct Coarsest {
  using Args = CoarsestArgs;
  static constexpr int kThreads = kCoarsestThreads;
  static __device__ void run(const Args& a, int blk) {
    switch (a.rows) {
      case 1: coarsest_rows<1>(a, blk); break;
      case 2: coarsest_rows<2>(a, blk); break;
      case 3: coarsest_rows<3>(a, blk); break;
      case 4: coarsest_rows<4>(a, blk); break;
      case 5: coarsest_rows<5>(a, blk); break;
      case 6: coarsest_rows<6>(a, blk); break;
      case 7: coarsest_rows<7>(a, blk); break;
      case 8: coarsest_rows<8>(a, blk); break;
      default:
        if (a.g.size <= kCoarseLds) coarsest_sums<true>(a, blk);
        else coarsest_sums<false>(a, blk);
    }
  }
};
inline int nblocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

constexpr int kTX = 8, kTY = 8;

template <class T, int R>
hipError_t launch_stream(const mls_plan_s* P, const T* q, GridDims g, const T* w, T scale, T* e, hipStream_t s) {
  constexpr int W = kStencilWaves;
  // z chunk: halve while the launch has fewer than ~1.5k waves, but keep the
  // 2R warm-up planes below half of the chunk
  const int xy = nblocks(g.n[0], kTX) * nblocks(g.n[1], kTY);
  int zc = g.n[2];
  while (zc > 4 * R && (int64_t)xy * W * nblocks(g.n[2], zc) < P->stencil_min_waves) zc = (zc + 1) / 2;
  dim3 grid(nblocks(g.n[0], kTX), nblocks(g.n[1], kTY), nblocks(g.n[2], zc));
  k_stencil_stream<T, R, W><<<grid, 64 * W, 0, s>>>(q, g, P->d_rows, P->d_wave_rows, w, scale, zc, e);
  return hipGetLastError();
}

template <class T>
hipError_t launch_stream_r(const mls_plan_s* P, int R, const T* q, GridDims g, const T* w, T scale, T* e,
                           hipStream_t s) {
  switch (R) {
    case 1: case 2: case 3: case 4: return launch_stream<T, 4>(P, q, g, w, scale, e, s);
    case 5: case 6: return launch_stream<T, 6>(P, q, g, w, scale, e, s);
    case 7: case 8: return launch_stream<T, 8>(P, q, g, w, scale, e, s);
    case 9: case 10: return launch_stream<T, 10>(P, q, g, w, scale, e, s);
    case 11: case 12: return launch_stream<T, 12>(P, q, g, w, scale, e, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Blocks of the coarsest-level kernel for grid g with `outs` output points
// per wave.
int coarsest_rows_form(const GridDims& g) { return coarse_rows_n(g); }

int coarsest_blocks(const GridDims& g, int outs, int rows) {
  if (rows) return (g.n[1] * g.n[2] + 63) / 64;
  return (int)(((int64_t)g.size + (int64_t)kCoarsestWaves * outs - 1) / ((int64_t)kCoarsestWaves * outs));
}

int stencil_window(const mls_plan_s* P) {
  return std::max(P->stencil_R[0], std::max(P->stencil_R[1], P->stencil_R[2]));
}

template <class T, int R>
hipError_t launch_tile(mls_plan_s* P, const T* wts, hipStream_t s, int kmax) {
  constexpr int kTileZ = tile_zc(R, sizeof(T) == 8);
  StencilLaunch L{};
  L.nlev = P->levels - 1;
  int t = 0;
  for (int k = 1; k < P->levels; ++k) {
    Level& Lv = P->lv[k - 1];
    StencilLevel& V = L.lv[k - 1];
    V.q = Lv.q;
    V.e = Lv.e;
    for (int d = 0; d < 3; ++d) V.n[d] = Lv.g.n[d];
    V.tiles_z = nblocks(Lv.g.n[2], kTileZ);
    V.tile0 = t;
    V.scale = std::ldexp(1.0, -6 * (k - 1));
    V.inv_size = 1.0 / (double)Lv.g.size;
    V.rows = P->d_rows;
    V.wave_rows = P->d_wave_rows;
    V.wts = wts;
    V.sum_xi = P->sum_q ? P->sum_q : P->d_scratch;
    V.wsum = P->taps_wsum;
    t += nblocks(Lv.g.n[0], 8) * nblocks(Lv.g.n[1], 8) * V.tiles_z;
    // the tile table lists the levels in order: levels 1..kmax are its head
    if (k == kmax) break;
  }
  k_stencil_tile<T, R, kTileZ, kStencilWaves><<<t, 64 * kStencilWaves, 0, s>>>(L, P->d_tiles);
  return hipGetLastError();
}

hipError_t launch_tile_f64(mls_plan_s* P, int R, hipStream_t s, int kmax) {
  const double* w = P->d_row_w_tile;
  switch (R) {
    case 1: case 2: case 3: case 4: return launch_tile<double, 4>(P, w, s, kmax);
    case 5: case 6: return launch_tile<double, 6>(P, w, s, kmax);
    case 7: case 8: return launch_tile<double, 8>(P, w, s, kmax);
    default: return hipErrorInvalidValue;
  }
}

// FP32 tiles reach R = 12: (8 + 2R)^2 (8 + 2R) floats, 88 KB at R = 10 and
// 128 KB at R = 12 (one block per CU; an FP64 tile of that size does not fit)
hipError_t launch_tile_f32(mls_plan_s* P, int R, hipStream_t s, int kmax) {
  const float* w = P->d_row_wf_tile;
  switch (R) {
    case 1: case 2: case 3: case 4: return launch_tile<float, 4>(P, w, s, kmax);
    case 5: case 6: return launch_tile<float, 6>(P, w, s, kmax);
    case 7: case 8: return launch_tile<float, 8>(P, w, s, kmax);
    case 9: case 10: return launch_tile<float, 10>(P, w, s, kmax);
    case 11: case 12: return launch_tile<float, 12>(P, w, s, kmax);
    default: return hipErrorInvalidValue;
  }
}

template <int R>
hipError_t launch_mfma(mls_plan_s* P, hipStream_t s, int kmax) {
  StencilLaunch L{};
  L.nlev = P->levels - 1;
  int t = 0;
  for (int k = 1; k < P->levels; ++k) {
    Level& Lv = P->lv[k - 1];
    StencilLevel& V = L.lv[k - 1];
    V.q = Lv.q;
    V.e = Lv.e;
    for (int d = 0; d < 3; ++d) V.n[d] = Lv.g.n[d];
    V.tiles_z = nblocks(Lv.g.n[2], 16);
    V.tile0 = t;
    V.scale = std::ldexp(1.0, -6 * (k - 1));
    V.inv_size = 1.0 / (double)Lv.g.size;
    V.rows = P->d_rows_mfma;
    V.wave_rows = P->d_wave_rows;
    V.wts = P->d_mfma_a;
    V.sum_xi = P->sum_q ? P->sum_q : P->d_scratch;
    V.wsum = P->taps_wsum;
    t += nblocks(Lv.g.n[0], 8) * nblocks(Lv.g.n[1], 8) * V.tiles_z;
    if (k == kmax) break;
  }
  k_stencil_mfma<R, kStencilWaves><<<t, 64 * kStencilWaves, 0, s>>>(L, P->d_tiles);
  return hipGetLastError();
}

hipError_t launch_tile_mfma(mls_plan_s* P, int R, hipStream_t s, int kmax) {
  switch (R) {
    case 1: case 2: case 3: case 4: return launch_mfma<4>(P, s, kmax);
    case 5: case 6: return launch_mfma<6>(P, s, kmax);
    default: return hipErrorInvalidValue;
  }
}

int stencil_path(const mls_plan_s* P) {
  if (P->levels < 2) return MLS_STENCIL_NONE;
  const int R = stencil_window(P);
  if (P->stencil_mfma) return MLS_STENCIL_TILE_MFMA_F32;
  if (P->stencil_kernel == 1 && P->precision == MLS_MIXED && R >= 1 && R <= 12) return MLS_STENCIL_TILE_F32;
  if (P->stencil_kernel == 1 && R >= 1 && R <= 8) return MLS_STENCIL_TILE_F64;
  if (R >= 1 && R <= 12) return MLS_STENCIL_STREAM_F64;
  return MLS_STENCIL_TAPS_F64;
}

hipError_t launch_stencils(mls_plan_s* P, hipStream_t s, int kmax) {
  if (P->levels < 2) return hipSuccess;
  if (kmax <= 0 || kmax > P->levels - 1) kmax = P->levels - 1;
  const int R = stencil_window(P);
  const int path = stencil_path(P);
  if (path == MLS_STENCIL_TILE_MFMA_F32) return launch_tile_mfma(P, R, s, kmax);
  if (path == MLS_STENCIL_TILE_F32) return launch_tile_f32(P, R, s, kmax);
  if (path == MLS_STENCIL_TILE_F64) return launch_tile_f64(P, R, s, kmax);
  const int ntaps = (int)P->taps.size();
  for (int k = 1; k <= kmax; ++k) {
    Level& L = P->lv[k - 1];
    const double scale = std::ldexp(1.0, -6 * (k - 1));
    hipError_t e;
    if (path == MLS_STENCIL_STREAM_F64) {
      e = launch_stream_r<double>(P, R, L.q, L.g, P->d_row_w, scale, L.e, s);
    } else {
      k_stencil_taps_f64<<<nblocks(L.g.size, kBlock), kBlock, 0, s>>>(L.q, L.g, P->d_taps, ntaps, scale, L.e);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_coarsest(mls_plan_s* P, hipStream_t s) {
  Level& L = P->lv[P->levels - 1];
  return launch_one<Coarsest>(CoarsestArgs{L.q, L.g, P->d_Kl, L.e, 1, 0}, coarsest_blocks(L.g, 1, 0), s);
}

bool stencil_tile_ok(int R, int zc) {
  if (R < 1 || R > 8) return false;
  if (zc == 8) return true;
  return zc == 16 && R <= 6;
}

template <class T, int R, int ZC>
hipError_t launch_tiles_batched(const BatchPhase& ph, hipStream_t s) {
  const int grid = ph.grid > 0 ? std::min(ph.grid, ph.nwork) : ph.nwork;
  k_stencil_tile_batched<T, R, ZC, kStencilWaves><<<grid, 64 * kStencilWaves, 0, s>>>(
      (const StencilLevel*)ph.args, (const int4*)ph.work, ph.nwork);
  return hipGetLastError();
}

// Batched phases of this file.  Stencil variant = window template (4, 6, 8)
// | z extent << 8 | 0x10000 for FP32 tiles.
hipError_t launch_batched_stencil(const BatchPhase& ph, hipStream_t s) {
  if (ph.nwork == 0) return hipSuccess;
  if (ph.kernel == BK_COARSEST) return launch_batched_phase<Coarsest>(ph, s);
  if (ph.kernel != BK_STENCIL) return hipErrorInvalidValue;
  const int R = ph.variant & 0xff, zc = (ph.variant >> 8) & 0xff;
  const bool f32 = (ph.variant & 0x10000) != 0;
  if (f32) {
    if (R == 4 && zc == 16) return launch_tiles_batched<float, 4, 16>(ph, s);
    if (R == 4 && zc == 8) return launch_tiles_batched<float, 4, 8>(ph, s);
    if (R == 6 && zc == 16) return launch_tiles_batched<float, 6, 16>(ph, s);
    if (R == 6 && zc == 8) return launch_tiles_batched<float, 6, 8>(ph, s);
    if (R == 8 && zc == 8) return launch_tiles_batched<float, 8, 8>(ph, s);
  } else {
    if (R == 4 && zc == 16) return launch_tiles_batched<double, 4, 16>(ph, s);
    if (R == 4 && zc == 8) return launch_tiles_batched<double, 4, 8>(ph, s);
    if (R == 6 && zc == 16) return launch_tiles_batched<double, 6, 16>(ph, s);
    if (R == 6 && zc == 8) return launch_tiles_batched<double, 6, 8>(ph, s);
    if (R == 8 && zc == 8) return launch_tiles_batched<double, 8, 8>(ph, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mls
