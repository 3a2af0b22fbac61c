// Local part of the evaluation step (eq:evaluation with k = 0): for every
// atom i, over all atoms j and periodic images n with (j,n) != (i,0) and
// r = |x_i - x_j - n o L| < a,
//     e0_i   = sum xi_j g_0(r),        g_0 = r^-6 - a^-6 gamma(r/a)   (eq:g_0)
//     F_i   += xi_i sum xi_j (g_0'(r)/r) d,   d = x_i - x_j - n o L
// with g_0'(r)/r = -6 r^-8 + a^-8 (15 rho^10 - 9 rho^22), rho = r/a, from
// eq:gamma.  Pairs are found through the linked cells of the binning step;
// the neighbour-cell offsets carry their image shift, which covers boxes
// narrower than three cells.
#include "device_math.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kBlock = 128;

// 1/s for g_0(r) and g_0'(r)/r from s = r^2 (caller guarantees 0 < s < a^2).
// FP64: the hardware reciprocal refined by two Newton steps (cheaper than
// the correctly rounded division sequence, accurate to the last bit or so).
// FP32: the hardware reciprocal alone (within about one ulp; the mixed path's
// force error stays two orders below its 1e-5 bound).
__device__ __forceinline__ double recip(double s) {
  double r = __builtin_amdgcn_rcp(s);
  r = fma(fma(-s, r, 1.0), r, r);
  return fma(fma(-s, r, 1.0), r, r);
}
__device__ __forceinline__ float recip(float s) { return __builtin_amdgcn_rcpf(s); }

// g_0(r) and g_0'(r)/r from s = r^2 (caller guarantees 0 < s < a^2), with
// rho = r/a and v = rho^12:
//   g_0     = r^-6 - a^-6 gamma_k(rho),            gamma_k = sum_j gc[j] v^j
//   g_0'/r  = -6 r^-8 - a^-8 rho^10 sum_j gq[j] v^j
// K = 2 is eq:gamma with its constants folded in; K = 0 takes any member of
// the family (k <= 4) from the plan's coefficients, zero-padded to degree 4.
template <class T, int K, class C>
__device__ __forceinline__ void g0_pair(T s, const C& pc, T& g, T& fr) {
  T ir2 = recip(s);
  T ir6 = ir2 * ir2 * ir2;
  T u = s * pc.inv_a2;         // rho^2
  T u2 = u * u;
  if constexpr (K == 2) {
    // eq:gamma: gamma = 15/8 - 5/4 v + 3/8 v^2 with v = rho^12 = u3^2, and
    // gamma'(rho)/rho = -15 rho^10 + 9 rho^22 = rho^10 (9 v - 15)
    const T u3 = u2 * u;
    const T v = u3 * u3;
    const T c0 = T(-15.0 / 8.0) * pc.inv_a6, c1 = T(5.0 / 4.0) * pc.inv_a6, c2 = T(-3.0 / 8.0) * pc.inv_a6;
    g = ir6 + fma(v, fma(v, c2, c1), c0);
    const T t = fma(v, T(-9) * pc.inv_a8, T(15) * pc.inv_a8);
    fr = fma(T(-6) * ir6, ir2, (u3 * u2) * t);
  } else {
    T u4 = u2 * u2;
    T u5 = u4 * u;
    T u6 = u4 * u2;
    T P = pc.gc[4];
    P = fma(P, u6, pc.gc[3]);
    P = fma(P, u6, pc.gc[2]);
    P = fma(P, u6, pc.gc[1]);
    P = fma(P, u6, pc.gc[0]);
    T Q = pc.gq[3];
    Q = fma(Q, u6, pc.gq[2]);
    Q = fma(Q, u6, pc.gq[1]);
    Q = fma(Q, u6, pc.gq[0]);
    g = ir6 - pc.inv_a6 * P;
    fr = T(-6) * ir6 * ir2 - pc.inv_a8 * u5 * Q;
  }
}

// Source weight of a pair: xi_j (geometric mixing), or under Lorentz-Berthelot
// e_j ((sigma_i + sigma_j) / 2)^6 with e_j = sqrt(2 eps_j) = xs.w, so that the
// target's factor e_i times it is C_ij of eq:xi-lj.
template <bool LB>
__device__ __forceinline__ double src_weight(double wj, const double* __restrict__ sig, double sig_i, int j) {
  if constexpr (LB) {
    const double m = 0.5 * (sig_i + sig[j]);
    const double m3 = m * m * m;
    return wj * (m3 * m3);
  } else {
    return wj;
  }
}

// FP64: one thread per cell-sorted target atom.
template <int K, bool LB = false>
struct PairGeneric {
  using Args = PairArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int s = blk * kBlock + threadIdx.x;
    if (s >= a.n) return;
    const CellGeom& g = a.g;
    const PairConst& pc = a.pc;
    const double4* __restrict__ xs = a.xs;
    const double4 xi = xs[s];
    const double sig_i = LB ? a.sig[s] : 0.0;
    const int c = a.cell_s[s];
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    double e = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int oz = -g.noff[2]; oz <= g.noff[2]; ++oz) {
      int tz = cz + oz;
      const int iz = floordiv(tz, g.nc[2]);
      tz -= iz * g.nc[2];
      const double sz = iz * g.L[2];
      for (int oy = -g.noff[1]; oy <= g.noff[1]; ++oy) {
        int ty = cy + oy;
        const int iy = floordiv(ty, g.nc[1]);
        ty -= iy * g.nc[1];
        const double sy = iy * g.L[1];
        for (int ox = -g.noff[0]; ox <= g.noff[0]; ++ox) {
          int tx = cx + ox;
          const int ix = floordiv(tx, g.nc[0]);
          tx -= ix * g.nc[0];
          const double sx = ix * g.L[0];
          const bool home = (ix | iy | iz) == 0;
          const int t = (tz * g.nc[1] + ty) * g.nc[0] + tx;
          const int j0 = a.cstart[t], j1 = a.cstart[t + 1];
          for (int j = j0; j < j1; ++j) {
            const double4 xj = xs[j];
            const double dx = xi.x - (xj.x + sx);
            const double dy = xi.y - (xj.y + sy);
            const double dz = xi.z - (xj.z + sz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < pc.a2 && !(home && j == s)) {
              double gg, fr;
              g0_pair<double, K>(r2, pc, gg, fr);
              const double wj = src_weight<LB>(xj.w, a.sig, sig_i, j);
              e += wj * gg;
              const double f = wj * fr;
              fx += f * dx;
              fy += f * dy;
              fz += f * dz;
            }
          }
        }
      }
    }
    a.e0[s] = e;
    a.floc[3 * (size_t)s + 0] = xi.w * fx;
    a.floc[3 * (size_t)s + 1] = xi.w * fy;
    a.floc[3 * (size_t)s + 2] = xi.w * fz;
  }
};

// FP64, one wave per target, for boxes too narrow for half-cutoff cells
// (few, crowded cells, often several images of one atom inside the cutoff).
// The wave walks the target's neighbour cells as contiguous runs of sorted
// atoms (a run ends where the periodic image changes) and its 64 lanes split
// each run; the lane sums are added in LDS.  Same cells, images and pairs as
// PairGeneric.
template <int K, bool LB = false>
struct PairWave {
  using Args = PairArgs;
  static constexpr int kThreads = 64;
  static __device__ void run(const Args& a, int s) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x;
    const CellGeom& g = a.g;
    const PairConst& pc = a.pc;
    const double4* __restrict__ xs = a.xs;
    const double4 xi = xs[s];
    const double sig_i = LB ? a.sig[s] : 0.0;
    const int c = a.cell_s[s];
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    double e = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int oz = -g.noff[2]; oz <= g.noff[2]; ++oz) {
      int tz = cz + oz;
      const int iz = floordiv(tz, g.nc[2]);
      tz -= iz * g.nc[2];
      const double sz = iz * g.L[2];
      for (int oy = -g.noff[1]; oy <= g.noff[1]; ++oy) {
        int ty = cy + oy;
        const int iy = floordiv(ty, g.nc[1]);
        ty -= iy * g.nc[1];
        const double sy = iy * g.L[1];
        const int row = (tz * g.nc[1] + ty) * g.nc[0];
        int u = cx - g.noff[0];
        const int uend = cx + g.noff[0];
        while (u <= uend) {
          const int ix = floordiv(u, g.nc[0]);
          const int tx = u - ix * g.nc[0];
          const int run = min(uend - u + 1, g.nc[0] - tx);
          const int j1 = a.cstart[row + tx + run];
          const double sx = ix * g.L[0];
          const bool home = (ix | iy | iz) == 0;
          for (int j = a.cstart[row + tx] + lane; j < j1; j += 64) {
            const double4 xj = xs[j];
            const double dx = xi.x - (xj.x + sx);
            const double dy = xi.y - (xj.y + sy);
            const double dz = xi.z - (xj.z + sz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < pc.a2 && !(home && j == s)) {
              double gg, fr;
              g0_pair<double, K>(r2, pc, gg, fr);
              const double wj = src_weight<LB>(xj.w, a.sig, sig_i, j);
              e += wj * gg;
              const double f = wj * fr;
              fx += f * dx;
              fy += f * dy;
              fz += f * dz;
            }
          }
          u += run;
        }
      }
    }
    red[0][lane] = e;
    red[1][lane] = fx;
    red[2][lane] = fy;
    red[3][lane] = fz;
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
      if (lane < off)
        for (int k = 0; k < 4; ++k) red[k][lane] += red[k][lane + off];
      __syncthreads();
    }
    if (lane == 0) {
      a.e0[s] = red[0][0];
      a.floc[3 * (size_t)s + 0] = xi.w * red[1][0];
      a.floc[3 * (size_t)s + 1] = xi.w * red[2][0];
      a.floc[3 * (size_t)s + 2] = xi.w * red[3][0];
    }
  }
};

// FP64, filter-and-drain over half-cutoff cells: one wave of 64 lanes takes
// 64 consecutive cell-sorted targets.  Each lane visits the 5 x 5 rows
// of cells around its target's cell, skips rows whose y/z gap to the target
// is at least a, and trims every other row to the cells the cutoff sphere
// can reach along x (at most two runs of cells: one per periodic image).  A
// cheap FP32 distance test (both precisions; see pair_scan_f32) appends
// sources inside the cutoff to the lane's LDS queue (a ring), four
// candidates per step; whenever a queue may overflow all lanes drain up to
// kDrain of their oldest entries through the full g_0 evaluation, and at the
// end everything left, so the expensive arithmetic runs on nearly full waves
// instead of being masked per candidate.  An FP64 entry packs the source
// index (< 2^25) with two bits per dimension for its image.
constexpr int kWaveQ = 64;    // lanes per block (one wave)
constexpr int kQueue = 32;    // entries per lane
// The FP32 kernel's ring is half as long: 4 KB of LDS per wave lets 24 waves
// share a CU (its VGPRs allow 24; 8 KB queues capped it at 20): pair kernel
// 0.46 -> 0.44 ms at 10^6 atoms.  The FP64 kernel is held to 16 waves per CU
// by its VGPRs, and a 16-entry ring only drains it more often (0.53 -> 0.64 ms).
constexpr int kQueueF = 16;   // entries per lane of the FP32 kernel
constexpr int kBatchF = 4;    // candidates per filter step

// 16-byte load from a 4-byte aligned address (four consecutive floats)
// element j of a uniform array through a 32-bit byte offset (the caller
// guarantees j * sizeof(T) < 2^32), so the load takes its base from scalar
// registers instead of a 64-bit per-lane address
template <class T>
__device__ __forceinline__ const T& at32(const T* base, int j) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (unsigned)j * (unsigned)sizeof(T));
}

__device__ __forceinline__ float4 load4f(const float* p) {
  float4 v;
  __builtin_memcpy(&v, p, sizeof(v));   // 4-byte aligned 16-byte load
  return v;
}

__device__ __forceinline__ int image_bits(int ix, int iy, int iz) { return (ix + 1) | ((iy + 1) << 2) | ((iz + 1) << 4); }

// Four FP64 sums of one lane (energy, force x, y, z), kept in LDS at stride
// kWaveQ while the lane's rows are scanned: only the drains read and write
// them, so the filter loop carries none of them (held in registers, the four
// were copied on every filter step, 11 of the loop's 70 instructions).
// Each drain starts with a compiler memory barrier (sums_fence): without it
// the sums were hoisted out of the loop into registers again (the queue and
// the sums are distinct LDS arrays), and volatile accesses instead made every
// update wait for its own load.
struct LaneSums {
  double* s;   // slot 0 of this lane
  __device__ __forceinline__ double& operator[](int k) const { return s[k * kWaveQ]; }
};

__device__ __forceinline__ void sums_fence() { asm volatile("" ::: "memory"); }

// Per-lane sums of a pair kernel: e_0 and the force in LDS, queue state in
// registers
struct PairAcc {
  LaneSums a;
  int cnt;
  int head;   // the lane's queue is a ring of kQueue slots
};

// Per-lane sums of the repulsive term (MD entry points): sum_j sqrt(C12_j)
// r^-12 and sum_j 12 sqrt(C12_j) r^-14 d over the pairs with r < rc.  Kept in
// registers: 2 KB more LDS per wave would cost these kernels occupancy (the
// FP64 one 16 -> 13 waves per CU, the FP32 one its last wave of 20).
struct RepAcc {
  double v[4];
  __device__ __forceinline__ double& operator[](int k) { return v[k]; }
  __device__ __forceinline__ double operator[](int k) const { return v[k]; }
};

// The kernels' LDS for the sums: four slots per lane.
constexpr int kSumSlots = 4 * kWaveQ;

// A drain during the scan consumes at most this many entries per lane: the
// lane that forced it is then well below the limit, and lanes with few
// entries idle for fewer steps than in a drain to empty.
constexpr int kDrain = 16;

// Full g_0 evaluation of up to `limit` queued sources per lane, oldest first.
// The loop body has no branches: slots past a lane's count (and the target
// itself) evaluate a harmless pair with zero weight, adding exactly 0.
template <int K, bool LB, bool R>
__device__ __forceinline__ void pair_drain_f64(const int* __restrict__ queue, int limit, int lane, int self_ent,
                                               int safe_j, const double4& xi, const double4* __restrict__ xs,
                                               const CellGeom& g, const PairConst& pc, const double* __restrict__ sig,
                                               double sig_i, PairAcc& A, const PairRep& rp, RepAcc& B) {
  sums_fence();
  const double r2_idle = 0.25 * pc.a2;
  const int cnt = A.cnt;
  // the lane's running sums, added to pair by pair as if held throughout
  double ae = A.a[0], afx = A.a[1], afy = A.a[2], afz = A.a[3];
  double be = 0.0, bfx = 0.0, bfy = 0.0, bfz = 0.0;
  if constexpr (R) {
    be = B[0];
    bfx = B[1];
    bfy = B[2];
    bfz = B[3];
  }
  for (int t = 0; t < limit && __any(t < cnt); ++t) {
    const int q = queue[((A.head + t) & (kQueue - 1)) * kWaveQ + lane];
    const bool ok = (t < cnt) & (q != self_ent);
    const int ent = ok ? q : image_bits(0, 0, 0);
    const int j = ok ? (ent >> 6) : safe_j;
    const double sx = (double)((ent & 3) - 1) * g.L[0];
    const double sy = (double)(((ent >> 2) & 3) - 1) * g.L[1];
    const double sz = (double)(((ent >> 4) & 3) - 1) * g.L[2];
    const double4 xj = at32(xs, j);
    const double dx = (xi.x - sx) - xj.x;
    const double dy = (xi.y - sy) - xj.y;
    const double dz = (xi.z - sz) - xj.z;
    const double d2 = dx * dx + dy * dy + dz * dz;
    // the FP32 filter passes a superset: the pair set is decided here, in
    // FP64, by r^2 < a^2 (rejected entries add exactly 0)
    const bool in = ok & (d2 < pc.a2);
    const double r2 = in ? d2 : r2_idle;
    double gg, fr;
    g0_pair<double, K>(r2, pc, gg, fr);
    const double wj = in ? src_weight<LB>(xj.w, sig, sig_i, j) : 0.0;
    ae += wj * gg;
    const double f = wj * fr;
    afx += f * dx;
    afy += f * dy;
    afz += f * dz;
    if constexpr (R) {
      const double ir2 = recip(r2);
      const double ir6 = ir2 * ir2 * ir2;
      const double v = (in && r2 < rp.rc2 ? rp.x12[j] : 0.0) * ir6 * ir6;
      const double fv = 12.0 * v * ir2;
      be += v;
      bfx += fv * dx;
      bfy += fv * dy;
      bfz += fv * dz;
    }
  }
  A.a[0] = ae;
  A.a[1] = afx;
  A.a[2] = afy;
  A.a[3] = afz;
  if constexpr (R) {
    B[0] = be;
    B[1] = bfx;
    B[2] = bfy;
    B[3] = bfz;
  }
  const int done = min(cnt, limit);
  A.head = (A.head + done) & (kQueue - 1);
  A.cnt = cnt - done;
}

// Scan sources [j, j1) seen through image bits `img`, row offsets dy, dz
// (convergent: every lane calls it; lanes with an empty range just take part
// in the votes).  Candidates are tested by the FP32 filter of the mixed
// kernel (absolute x, cell-relative y and z, one 16-byte load per coordinate
// and batch of four, threshold a2f widened for FP32 rounding): it passes a
// superset of the pairs inside the cutoff, and the drain decides each pair
// in FP64.  Reads may run up to three rows past j1 (padded array); lanes
// past their range load nothing.  The filter loop touches no accumulator: it
// stops when a queue may overflow, the queues are partly drained, and the
// filter resumes.
template <int K, bool LB, bool R>
__device__ __forceinline__ void pair_scan_f64(int j, int j1, int img, int dy, int dz, int* __restrict__ queue,
                                              int lane, int self_ent, int safe_j, const double4& xi, const float3& xf_i,
                                              const double4* __restrict__ xs, const float* __restrict__ xf, int xfs,
                                              const CellGeom& g, const PairConst& pc,
                                              const double* __restrict__ sig, double sig_i, PairAcc& A,
                                              const PairRep& rp, RepAcc& B) {
  const float ax = fmaf((float)-((img & 3) - 1), pc.Lf[0], xf_i.x);
  const float ay = fmaf((float)-dy, pc.wf[1], xf_i.y);
  const float az = fmaf((float)-dz, pc.wf[2], xf_i.z);
  int* const qlane = queue + lane;
  const float* const xf1 = xf + xfs;
  const float* const xf2 = xf1 + xfs;
  // loop-carried, so a finished lane keeps stale values; b < rem masks them
  float4 X = make_float4(0.0f, 0.0f, 0.0f, 0.0f), Y = X, Z = X;
  for (;;) {
    int cnt = A.cnt;
    const int head = A.head;
    bool full = false;
    while (__any(j < j1)) {
      const int rem = j1 - j;   // sources left in the run (<= 0: none)
      if (j < j1) {
        // a 32-bit byte offset from the uniform array bases
        const unsigned off = (unsigned)j * 4u;
        X = load4f(reinterpret_cast<const float*>(reinterpret_cast<const char*>(xf) + off));
        Y = load4f(reinterpret_cast<const float*>(reinterpret_cast<const char*>(xf1) + off));
        Z = load4f(reinterpret_cast<const float*>(reinterpret_cast<const char*>(xf2) + off));
      }
      const float xb[4] = {X.x, X.y, X.z, X.w}, yb[4] = {Y.x, Y.y, Y.z, Y.w}, zb[4] = {Z.x, Z.y, Z.z, Z.w};
      const int ent0 = (j << 6) | img;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const float dxv = ax - xb[b], dyv = ay - yb[b], dzv = az - zb[b];
        const float r2 = dxv * dxv + dyv * dyv + dzv * dzv;
        const bool hit = (b < rem) & (r2 < pc.a2f);
        // the next free slot: write unconditionally, keep on a hit
        qlane[kWaveQ * ((head + cnt) & (kQueue - 1))] = ent0 + (b << 6);
        cnt += hit ? 1 : 0;
      }
      // finished lanes advance too: rem <= 0 masks them and the loads stay
      // guarded by j < j1 (j grows by at most 4 per step of the slowest lane)
      j += 4;
      if (__any(cnt > kQueue - 4)) {
        full = true;
        break;
      }
    }
    A.cnt = cnt;
    if (!full) break;
    pair_drain_f64<K, LB, R>(queue, kDrain, lane, self_ent, safe_j, xi, xs, g, pc, sig, sig_i, A, rp, B);
  }
}

__device__ __forceinline__ double gap1(double x, double lo, double w, double eps) {
  return fmax(0.0, fmax(lo - x, x - (lo + w)) - eps);
}

// Per-wave sum of one value (lanes of a 64-wide block).
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Repulsive outputs of target sc: its sorted forces and, per block (one
// wave), the sum of sqrt(C12_i) times the lanes' energy sums.
__device__ __forceinline__ void store_rep(const PairRep& rp, bool active, int sc, int lane, int blk,
                                          const RepAcc& B) {
  double e = 0.0;
  if (active) {
    const double ci = rp.x12[sc];
    e = ci * B[0];
    rp.frep[3 * (size_t)sc + 0] = ci * B[1];
    rp.frep[3 * (size_t)sc + 1] = ci * B[2];
    rp.frep[3 * (size_t)sc + 2] = ci * B[3];
  }
  e = wave_sum(e);
  if (lane == 0) rp.partial[blk] = e;
}

template <int K, bool LB = false, bool R = false>
struct PairTrimF64 {
  using Args = PairArgs;
  static constexpr int kThreads = kWaveQ;
  static __device__ void run(const Args& ar, int blk) {
  const double4* __restrict__ xs = ar.xs;
  const int* __restrict__ cstart = ar.cstart;
  const CellGeom& g = ar.g;
  const PairConst& pc = ar.pc;
  const int n = ar.n;
  __shared__ int queue[kQueue * kWaveQ];
  const int lane = threadIdx.x;
  const int k = blk * kWaveQ + lane;
  const bool active = k < n;
  const int sc = active ? k : n - 1;
  const double4 xi = xs[sc];
  const double sig_i = LB ? ar.sig[sc] : 0.0;
  const float* __restrict__ xf = ar.xf;
  const int xfs = ar.xf_stride;
  const float3 xf_i = make_float3(xf[sc], xf[xfs + sc], xf[2 * xfs + sc]);
  const int c = ar.cell_s[sc];
  const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
  // the target itself, seen in the home image, is skipped in the drain
  const int self_ent = active ? ((sc << 6) | image_bits(0, 0, 0)) : -1;
  __shared__ double sums[kSumSlots];
  for (int k = 0; k < kSumSlots / kWaveQ; ++k) sums[k * kWaveQ + lane] = 0.0;
  PairAcc A{LaneSums{sums + lane}, 0, 0};
  RepAcc B{{0.0, 0.0, 0.0, 0.0}};
  const PairRep& rp = ar.rep;
  const float reach = (float)(1.0 + 1e-5);
  for (int dz = -2; dz <= 2; ++dz) {
    const int uz = cz + dz;
    const int iz = uz < 0 ? -1 : (uz >= g.nc[2] ? 1 : 0);
    const int tz = uz - iz * g.nc[2];
    // gaps shrunk (and the reach below grown) by the skin margin: with
    // neighbour reuse atoms may sit that far outside their cells
    const double gz = gap1(xi.z, uz * g.w[2], g.w[2], 1e-12 * g.L[2] + g.margin);
    for (int dy = -2; dy <= 2; ++dy) {
      const int uy = cy + dy;
      const int iy = uy < 0 ? -1 : (uy >= g.nc[1] ? 1 : 0);
      const int ty = uy - iy * g.nc[1];
      const double gy = gap1(xi.y, uy * g.w[1], g.w[1], 1e-12 * g.L[1] + g.margin);
      const double rem = pc.a2 - (gy * gy + gz * gz);
      int clo = 0, chi = -1;
      if (active && rem > 0.0) {
        // x cells the cutoff sphere reaches in this row (conservatively widened)
        const double rx = (double)(sqrtf((float)rem) * reach) + 1e-6 * g.w[0] + g.margin;
        clo = max(cx - 2, (int)floor((xi.x - rx) * g.inv_w[0]));
        chi = min(cx + 2, (int)floor((xi.x + rx) * g.inv_w[0]));
      }
      // at most one box edge inside [clo, chi] (nc >= 5): two runs of cells
      int lo1 = clo, hi1 = chi, ix1 = 0, lo2 = 0, hi2 = -1, ix2 = 0;
      if (clo < 0) {
        lo1 = clo + g.nc[0]; hi1 = g.nc[0] - 1; ix1 = -1;
        lo2 = 0; hi2 = chi; ix2 = 0;
      } else if (chi >= g.nc[0]) {
        lo1 = clo; hi1 = g.nc[0] - 1; ix1 = 0;
        lo2 = 0; hi2 = chi - g.nc[0]; ix2 = 1;
      }
      const int row = (tz * g.nc[1] + ty) * g.nc[0];
      int j0 = 0, j1 = 0;
      if (lo1 <= hi1) {
        j0 = cstart[row + lo1];
        j1 = cstart[row + hi1 + 1];
      }
      int k0 = 0, k1 = 0;
      if (lo2 <= hi2) {
        k0 = cstart[row + lo2];
        k1 = cstart[row + hi2 + 1];
      }
      pair_scan_f64<K, LB, R>(j0, j1, image_bits(ix1, iy, iz), dy, dz, queue, lane, self_ent, sc, xi, xf_i, xs, xf,
                              xfs, g, pc, ar.sig, sig_i, A, rp, B);
      pair_scan_f64<K, LB, R>(k0, k1, image_bits(ix2, iy, iz), dy, dz, queue, lane, self_ent, sc, xi, xf_i, xs, xf,
                              xfs, g, pc, ar.sig, sig_i, A, rp, B);
    }
  }
  pair_drain_f64<K, LB, R>(queue, kQueue, lane, self_ent, sc, xi, xs, g, pc, ar.sig, sig_i, A, rp, B);
  if (active) {
    ar.e0[sc] = A.a[0];
    ar.floc[3 * (size_t)sc + 0] = xi.w * A.a[1];
    ar.floc[3 * (size_t)sc + 1] = xi.w * A.a[2];
    ar.floc[3 * (size_t)sc + 2] = xi.w * A.a[3];
  }
  if constexpr (R) store_rep(rp, active, sc, lane, blk, B);
  }
};

// ---------------------------------------------------------------------------
// FP32-mixed variant of the same scheme.  Sources carry cell-relative FP32
// coordinates (x - cx w, y - cy w, z - cz w) and their cell x index (exact in
// FP32) in the fourth component; xi is a separate FP32 array read only in the
// drain.  The displacement is rebuilt as
//   d_x = (cx_i - ix nc - cx_j) w_x + xr_i - xr_j,  d_y = yr_i - dy w_y - yr_j, ...
// with integer cell offsets, so no large coordinates enter FP32 arithmetic.
// Queue entries pack the source index (< 2^24), the x image and the row
// offsets dy, dz.  Pair arithmetic is FP32; each drain sums its terms in
// FP32, and e_0 and the forces accumulate the drains' sums in FP64.
struct PairAccM {
  LaneSums a;   // e_0 and the force, FP64, in LDS
  int cnt;
  int head;     // the lane's queue is a ring of kQueueF slots
};

// An FP32 drain consumes at most this many entries per lane: the lane that
// forced it is then below the limit again (at most 16 - 8 = 8 entries, one
// filter step adds at most 4 to the 12 that trigger a drain), and lanes with
// few entries idle for fewer steps than in a drain to empty (measured at 10^6
// atoms with the 16-entry ring: pair kernel 0.44 ms with 8 and with 4, 0.46
// ms with 12).
constexpr int kDrainF = 8;

// Per-lane target data of the FP32 scan.
struct PairLaneF {
  float xx, yy, zz;     // target cell-relative coordinates
  float cxf, ncf;       // target cell x index, cells along x
  int self_ent;         // the target's own home-row entry (-1 for idle lanes)
  int safe_j;           // a valid source index for idle drain slots
  float sig_i;          // Lorentz-Berthelot: the target's sigma
  float xa;             // target absolute x (filter)
};

// Queue entry: source index << 8 | x image ix (2 bits) | dy (3 bits) | dz (3
// bits), the three as two's-complement fields.
__device__ __forceinline__ int entry_bits(int ix, int dy, int dz) { return (ix & 3) | ((dy & 7) << 2) | ((dz & 7) << 5); }

// Full g_0 evaluation of up to `limit` queued sources per lane, oldest first.
// The loop body has no branches: slots past a lane's count (and the target
// itself) evaluate a harmless pair with zero weight, so every lane adds
// exactly 0 for them.
template <int K, bool R, bool LB>
__device__ __forceinline__ void pair_drain_f32(const int* __restrict__ queue, int limit, int lane,
                                               const PairLaneF& L, const float4* __restrict__ xr,
                                               const float* __restrict__ xif, const float* __restrict__ sig,
                                               const PairConstF& pc, PairAccM& A, const PairRep& rp, RepAcc& B) {
  sums_fence();
  const float r2_idle = 0.25f * pc.a2;
  const float rc2 = (float)rp.rc2;
  const int cnt = A.cnt;
  // the (at most 32) terms of one drain are summed in FP32, the drains' sums
  // in FP64
  float e = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
  float re = 0.0f, rfx = 0.0f, rfy = 0.0f, rfz = 0.0f;
  for (int t = 0; t < limit && __any(t < cnt); ++t) {
    const int q = queue[((A.head + t) & (kQueueF - 1)) * kWaveQ + lane];
    const bool ok = (t < cnt) & (q != L.self_ent);
    const int ent = ok ? q : 0;
    const int j = ok ? (int)((unsigned)ent >> 8) : L.safe_j;
    // idle slots load nothing (they take a harmless far pair of weight 0)
    float4 xj = make_float4(L.xx + pc.w[0], L.yy, L.zz, L.cxf);
    float wsrc = 0.0f;
    if (ok) {
      xj = at32(xr, j);
      wsrc = at32(xif, j);
    }
    const int ix = (ent << 30) >> 30, dy = (ent << 27) >> 29, dz = (ent << 24) >> 29;
    const float bx = fmaf((float)ix, -L.ncf, L.cxf);
    const float dxv = fmaf(bx - xj.w, pc.w[0], L.xx) - xj.x;
    const float dyv = fmaf((float)-dy, pc.w[1], L.yy) - xj.y;
    const float dzv = fmaf((float)-dz, pc.w[2], L.zz) - xj.z;
    const float r2 = ok ? dxv * dxv + dyv * dyv + dzv * dzv : r2_idle;
    float gg, fr;
    g0_pair<float, K>(r2, pc, gg, fr);
    float wj = wsrc;
    if constexpr (LB) {
      // source weight e_j ((sigma_i + sigma_j) / 2)^6, as in the FP64 kernels
      const float m = 0.5f * (L.sig_i + sig[j]);
      const float m3 = m * m * m;
      wj *= m3 * m3;
    }
    e = fmaf(wj, gg, e);
    const float f = wj * fr;
    fx = fmaf(f, dxv, fx);
    fy = fmaf(f, dyv, fy);
    fz = fmaf(f, dzv, fz);
    if constexpr (R) {
      const float ir2 = recip(r2);
      const float ir6 = ir2 * ir2 * ir2;
      const float v = (ok && r2 < rc2 ? rp.x12f[j] : 0.0f) * ir6 * ir6;
      const float fv = 12.0f * v * ir2;
      re += v;
      rfx = fmaf(fv, dxv, rfx);
      rfy = fmaf(fv, dyv, rfy);
      rfz = fmaf(fv, dzv, rfz);
    }
  }
  A.a[0] += (double)e;
  A.a[1] += (double)fx;
  A.a[2] += (double)fy;
  A.a[3] += (double)fz;
  if constexpr (R) {
    B[0] += (double)re;
    B[1] += (double)rfx;
    B[2] += (double)rfy;
    B[3] += (double)rfz;
  }
  const int done = min(cnt, limit);
  A.head = (A.head + done) & (kQueueF - 1);
  A.cnt = cnt - done;
}

// Scan sources [j, j1) of one row run (image ix along x, row offsets dy, dz).
// The filter loop touches no accumulator: it stops when a queue may
// overflow, the queues are partly drained, and the filter resumes.
// The filter takes x from the absolute FP32 coordinates (one subtraction per
// candidate instead of rebuilding the cell offset) and y, z cell-relative;
// its threshold a2f covers the rounding of absolute x (a few ulp of L), and
// the few extra pairs it passes, just outside a, add g_0 ~ 0 in the drain,
// which rebuilds the displacement exactly from the cell-relative data.  The
// coordinates are three arrays, so one 16-byte load brings one coordinate of
// a batch of four candidates; lanes past the end of their run load nothing.
// The vector memory pipeline, as much as the ALU, bounds this loop.

template <int K, bool R, bool LB>
__device__ __forceinline__ void pair_scan_f32(int j, int j1, int ix, int dy, int dz, int* __restrict__ queue,
                                              int lane, const PairLaneF& L, const float4* __restrict__ xr,
                                              const float* __restrict__ xf, int xfs, const float* __restrict__ xif,
                                              const float* __restrict__ sig, const PairConstF& pc, PairAccM& A,
                                              const PairRep& rp, RepAcc& B, float4& X, float4& Y, float4& Z) {
  static_assert(kBatchF == 4, "one 16-byte load per coordinate and batch");
  const float ax = fmaf((float)-ix, pc.L[0], L.xa);
  const float ay = fmaf((float)-dy, pc.w[1], L.yy);
  const float az = fmaf((float)-dz, pc.w[2], L.zz);
  const int bits = entry_bits(ix, dy, dz);
  int* const qlane = queue + lane;
  const float* const xf1 = xf + xfs;
  const float* const xf2 = xf1 + xfs;
  // X, Y, Z are the caller's, carried across runs: a finished lane keeps
  // stale values, which b < rem masks
  // one loop level, the drain inside it: the accumulators change only on the
  // drain path (a loop nest made the compiler copy them every filter step)
  int cnt = A.cnt, head = A.head;
  while (__any(j < j1)) {
    const int rem = j1 - j;   // sources left in the run (<= 0: none)
    if (j < j1) {
      // a 32-bit byte offset from the uniform array bases
      const unsigned off = (unsigned)j * 4u;
      X = load4f(reinterpret_cast<const float*>(reinterpret_cast<const char*>(xf) + off));
      Y = load4f(reinterpret_cast<const float*>(reinterpret_cast<const char*>(xf1) + off));
      Z = load4f(reinterpret_cast<const float*>(reinterpret_cast<const char*>(xf2) + off));
    }
    const float xb[4] = {X.x, X.y, X.z, X.w}, yb[4] = {Y.x, Y.y, Y.z, Y.w}, zb[4] = {Z.x, Z.y, Z.z, Z.w};
    const int ent0 = (j << 8) | bits;
#pragma unroll
    for (int b = 0; b < kBatchF; ++b) {
      const float dxv = ax - xb[b], dyv = ay - yb[b], dzv = az - zb[b];
      const float r2 = dxv * dxv + dyv * dyv + dzv * dzv;
      const bool hit = (b < rem) & (r2 < pc.a2f);
      qlane[kWaveQ * ((head + cnt) & (kQueueF - 1))] = ent0 + (b << 8);
      cnt += hit ? 1 : 0;
    }
    // finished lanes advance too: rem <= 0 masks them and the loads stay
    // guarded by j < j1 (j grows by at most 4 per step of the slowest lane)
    j += kBatchF;
    if (__builtin_expect(__any(cnt > kQueueF - kBatchF), 0)) {
      A.cnt = cnt;
      pair_drain_f32<K, R, LB>(queue, kDrainF, lane, L, xr, xif, sig, pc, A, rp, B);
      cnt = A.cnt;
      head = A.head;
    }
  }
  A.cnt = cnt;
}

template <int K, bool R = false, bool LB = false>
struct PairTrimF32 {
  using Args = PairArgsF;
  static constexpr int kThreads = kWaveQ;
  static __device__ void run(const Args& ar, int blk) {
  const float4* __restrict__ xr = ar.xr;
  const float* __restrict__ xif = ar.xif;
  const int* __restrict__ cstart = ar.cstart;
  const CellGeom& g = ar.g;
  const PairConstF& pc = ar.pc;
  const int n = ar.n;
  __shared__ int queue[kQueueF * kWaveQ];
  const int lane = threadIdx.x;
  const int k = blk * kWaveQ + lane;
  const bool active = k < n;
  const int sc = active ? k : n - 1;
  const float4 xi = xr[sc];
  const int c = ar.cell_s[sc];
  const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
  const float* __restrict__ sig = ar.sig;
  const float* __restrict__ xf = ar.xf;
  const int xfs = ar.xf_stride;
  const PairLaneF L{xi.x, xi.y, xi.z, (float)cx, (float)g.nc[0], active ? ((sc << 8) | entry_bits(0, 0, 0)) : -1, sc,
                    LB ? sig[sc] : 0.0f, xf[sc]};
  __shared__ double sums[kSumSlots];
  for (int k = 0; k < kSumSlots / kWaveQ; ++k) sums[k * kWaveQ + lane] = 0.0;
  PairAccM A{LaneSums{sums + lane}, 0, 0};
  RepAcc B{{0.0, 0.0, 0.0, 0.0}};
  const PairRep& rp = ar.rep;
  // Rows are chosen and trimmed in the target's cell-relative FP32
  // coordinates.  The gaps are shrunk and the reach grown by margins (1e-5 of
  // a cell, 2e-5 of the cutoff) far above their FP32 rounding (~1e-7), so no
  // cell that holds a source inside the cutoff is ever skipped.
  const float a2m = pc.a2 * (1.0f + 2e-5f);
  const float reach = 1.0f + 2e-5f;
  const float inv_wx = 1.0f / pc.w[0];
  // the skin margin of neighbour reuse (atoms may sit that far outside their
  // cells): shrinks the gaps and grows the reach
  const float mg = (float)g.margin;
  const int nc0 = g.nc[0], nc1 = g.nc[1], nc2 = g.nc[2];
  // the candidate registers of the scans, carried from run to run
  float4 X = make_float4(0.0f, 0.0f, 0.0f, 0.0f), Y = X, Z = X;
  for (int dz = -2; dz <= 2; ++dz) {
    const int uz = cz + dz;
    const int tz = uz < 0 ? uz + nc2 : (uz >= nc2 ? uz - nc2 : uz);
    const float gz = dz == 0 ? 0.0f
                             : fmaxf(0.0f, (dz > 0 ? fmaf((float)dz, pc.w[2], -xi.z)
                                                   : fmaf((float)(-dz - 1), pc.w[2], xi.z)) - 1e-5f * pc.w[2] - mg);
    const float rem_z = a2m - gz * gz;
    const int rowz = tz * nc1;
    int ty = cy - 2 < 0 ? cy - 2 + nc1 : cy - 2;
    for (int dy = -2; dy <= 2; ++dy) {
      const float gy = dy == 0 ? 0.0f
                               : fmaxf(0.0f, (dy > 0 ? fmaf((float)dy, pc.w[1], -xi.y)
                                                     : fmaf((float)(-dy - 1), pc.w[1], xi.y)) - 1e-5f * pc.w[1] - mg);
      const float rem = rem_z - gy * gy;
      int clo = 0, chi = -1;
      if (active && rem > 0.0f) {
        // hardware square root (about 1 ulp): far inside the margin
        const float rx = fmaf(__builtin_amdgcn_sqrtf(rem), reach, 1e-5f * pc.w[0] + mg);
        clo = cx + max(-2, (int)floorf((xi.x - rx) * inv_wx));
        chi = cx + min(2, (int)floorf((xi.x + rx) * inv_wx));
      }
      int lo1 = clo, hi1 = chi, ix1 = 0, lo2 = 0, hi2 = -1, ix2 = 0;
      if (clo < 0) {
        lo1 = clo + nc0; hi1 = nc0 - 1; ix1 = -1;
        lo2 = 0; hi2 = chi; ix2 = 0;
      } else if (chi >= nc0) {
        lo1 = clo; hi1 = nc0 - 1; ix1 = 0;
        lo2 = 0; hi2 = chi - nc0; ix2 = 1;
      }
      const int row = (rowz + ty) * nc0;
      ty = ty + 1 == nc1 ? 0 : ty + 1;
      int j0 = 0, j1 = 0;
      if (lo1 <= hi1) {
        j0 = at32(cstart, row + lo1);
        j1 = at32(cstart, row + hi1 + 1);
      }
      int k0 = 0, k1 = 0;
      if (lo2 <= hi2) {
        k0 = at32(cstart, row + lo2);
        k1 = at32(cstart, row + hi2 + 1);
      }
      // the second run (across the periodic edge) is empty for most waves:
      // its set-up is skipped unless some lane has one
      if (__any(j0 < j1))
        pair_scan_f32<K, R, LB>(j0, j1, ix1, dy, dz, queue, lane, L, xr, xf, xfs, xif, sig, pc, A, rp, B, X, Y, Z);
      if (__any(k0 < k1))
        pair_scan_f32<K, R, LB>(k0, k1, ix2, dy, dz, queue, lane, L, xr, xf, xfs, xif, sig, pc, A, rp, B, X, Y, Z);
    }
  }
  pair_drain_f32<K, R, LB>(queue, kQueueF, lane, L, xr, xif, sig, pc, A, rp, B);
  if (active) {
    const double wi = (double)xif[sc];
    ar.e0[sc] = A.a[0];
    ar.floc[3 * (size_t)sc + 0] = wi * A.a[1];
    ar.floc[3 * (size_t)sc + 1] = wi * A.a[2];
    ar.floc[3 * (size_t)sc + 2] = wi * A.a[3];
  }
  if constexpr (R) store_rep(rp, active, sc, lane, blk, B);
  }
};

}  // namespace

// Threshold of the FP32 candidate filters: the filter's |dx| is within ex of
// the exact value (absolute coordinates and the image shift rounded to FP32,
// at most a few ulp of L + a; neighbour reuse lets atoms sit skin/2 outside
// the box), so r^2 < a^2 + 2 a ex + ex^2, plus FP32 rounding of the sum,
// keeps every pair inside the cutoff.
float filter_a2(const mls_plan_s* P) {
  const double a = std::sqrt(P->a2);
  const double ex = 4.0 * (P->cg.L[0] + P->cg.margin + a) * std::ldexp(1.0, -24);
  return std::nextafter((float)(P->a2 * (1.0 + 4.0 * std::ldexp(1.0, -23)) + 2.0 * a * ex + ex * ex), INFINITY);
}

PairConst pair_const(const mls_plan_s* P) {
  PairConst pc{P->a2, P->inv_a2, P->inv_a6, P->inv_a8, {}, {}, filter_a2(P), {}, {}};
  for (int j = 0; j < 5; ++j) pc.gc[j] = P->gamma_c[j];
  for (int j = 0; j < 4; ++j) pc.gq[j] = 12.0 * (j + 1) * P->gamma_c[j + 1];
  for (int d = 0; d < 3; ++d) {
    pc.wf[d] = (float)P->cg.w[d];
    pc.Lf[d] = (float)P->cg.L[d];
  }
  return pc;
}

PairConstF pair_const_f(const mls_plan_s* P) {
  const PairConst pc = pair_const(P);
  PairConstF pf{(float)pc.a2, (float)pc.inv_a2, (float)pc.inv_a6, (float)pc.inv_a8,
                {(float)P->cg.w[0], (float)P->cg.w[1], (float)P->cg.w[2]}, {}, {}};
  for (int j = 0; j < 5; ++j) pf.gc[j] = (float)pc.gc[j];
  for (int j = 0; j < 4; ++j) pf.gq[j] = (float)pc.gq[j];
  for (int d = 0; d < 3; ++d) pf.L[d] = (float)P->cg.L[d];
  pf.a2f = pc.a2f;
  return pf;
}

int pair_variant(const mls_plan_s* P) { return P->continuity == 2 ? 2 : 0; }

template <int K>
hipError_t launch_pair_k(mls_plan_s* P, int n, hipStream_t s, const PairRep* rep, bool* fused) {
  const CellGeom& g = P->cg;
  const int waves = (n + kWaveQ - 1) / kWaveQ;
  if (P->precision == MLS_MIXED && P->pair_fast && n < (1 << 24)) {
    PairArgsF a{P->d_xr, P->d_xif, P->d_xs, P->d_cell_s, P->d_cell_start, n, g, pair_const_f(P), P->d_e0,
                P->d_floc};
    a.xf = P->d_xf;
    a.xf_stride = P->xf_stride;
    if (!rep) return launch_persist<PairTrimF32<K>>(a, waves, P->pair_blocks, s);
    a.rep = *rep;
    *fused = true;
    P->rep_nb = waves;
    return launch_persist<PairTrimF32<K, true>>(a, waves, P->pair_blocks, s);
  }
  PairArgs a{P->d_xs, P->d_cell_s, P->d_cell_start, n, g, pair_const(P), P->d_e0, P->d_floc, nullptr};
  a.xf = P->d_xf;
  a.xf_stride = P->xf_stride;
  if (P->pair_fast && n < (1 << 25)) {
    if (!rep) return launch_persist<PairTrimF64<K>>(a, waves, P->pair_blocks, s);
    a.rep = *rep;
    *fused = true;
    P->rep_nb = waves;
    return launch_persist<PairTrimF64<K, false, true>>(a, waves, P->pair_blocks, s);
  }
  if (!P->pair_fast) return launch_one<PairWave<K>>(a, n, s);
  return launch_one<PairGeneric<K>>(a, (n + kBlock - 1) / kBlock, s);
}

// Lorentz-Berthelot: the same kernels with the LB source weight.
template <int K>
hipError_t launch_pair_lb_k(mls_plan_s* P, int n, hipStream_t s) {
  if (P->precision == MLS_MIXED && P->pair_fast && n < (1 << 24)) {
    PairArgsF a{P->d_xr, P->d_xif, P->d_xs, P->d_cell_s, P->d_cell_start, n, P->cg, pair_const_f(P), P->d_e0,
                P->d_floc};
    a.sig = P->d_sigf;
    a.xf = P->d_xf;
    a.xf_stride = P->xf_stride;
    return launch_one<PairTrimF32<K, false, true>>(a, (n + kWaveQ - 1) / kWaveQ, s);
  }
  PairArgs a{P->d_xs, P->d_cell_s, P->d_cell_start, n, P->cg, pair_const(P), P->d_e0, P->d_floc, P->d_sig};
  a.xf = P->d_xf;
  a.xf_stride = P->xf_stride;
  if (P->pair_fast && n < (1 << 25)) return launch_one<PairTrimF64<K, true>>(a, (n + kWaveQ - 1) / kWaveQ, s);
  if (!P->pair_fast) return launch_one<PairWave<K, true>>(a, n, s);
  return launch_one<PairGeneric<K, true>>(a, (n + kBlock - 1) / kBlock, s);
}

hipError_t launch_pair_lb(mls_plan_s* P, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return pair_variant(P) == 2 ? launch_pair_lb_k<2>(P, n, s) : launch_pair_lb_k<0>(P, n, s);
}

hipError_t launch_pair(mls_plan_s* P, int n, hipStream_t s, const PairRep* rep, bool* fused) {
  bool f = false;
  if (!fused) fused = &f;
  *fused = false;
  if (n == 0) return hipSuccess;
  return pair_variant(P) == 2 ? launch_pair_k<2>(P, n, s, rep, fused) : launch_pair_k<0>(P, n, s, rep, fused);
}

template <int K>
hipError_t launch_batched_pair_k(const BatchPhase& ph, hipStream_t s, bool lb) {
  switch (ph.kernel) {
    case BK_PAIR_GENERIC:
      return lb ? launch_batched_phase<PairGeneric<K, true>>(ph, s) : launch_batched_phase<PairGeneric<K>>(ph, s);
    case BK_PAIR_WAVE:
      return lb ? launch_batched_phase<PairWave<K, true>>(ph, s) : launch_batched_phase<PairWave<K>>(ph, s);
    case BK_PAIR_TRIM_F64:
      return lb ? launch_batched_phase<PairTrimF64<K, true>>(ph, s) : launch_batched_phase<PairTrimF64<K>>(ph, s);
    case BK_PAIR_TRIM_F32:
      return lb ? launch_batched_phase<PairTrimF32<K, false, true>>(ph, s)
                : launch_batched_phase<PairTrimF32<K>>(ph, s);
    default: return hipErrorInvalidValue;
  }
}

// Batched phases of this file; variant = the pair_variant of its boxes, | 0x10
// under Lorentz-Berthelot mixing.
hipError_t launch_batched_pair(const BatchPhase& ph, hipStream_t s) {
  const bool lb = (ph.variant & 0x10) != 0;
  return (ph.variant & 0xf) == 2 ? launch_batched_pair_k<2>(ph, s, lb) : launch_batched_pair_k<0>(ph, s, lb);
}

}  // namespace mls
