// Device-side closed forms of the method: the nodal basis Phi (and its
// derivative) evaluated for the p grid points a particle touches, the wrap of
// a coordinate into the box, and small helpers.
#pragma once

#include <hip/hip_runtime.h>

namespace mls {

// Coordinate wrapped into [0, L) with every step a single rounded IEEE
// operation (no contraction), so host references can reproduce the cell and
// grid indices it decides exactly.
__device__ __forceinline__ double wrap_coord(double x, double L, double invL) {
#pragma clang fp contract(off)
  double f = floor(x * invL);
  double xw = x - f * L;
  if (xw >= L) xw -= L;
  if (xw < 0.0) xw += L;
  return xw;
}

__device__ __forceinline__ int floordiv(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

__device__ __forceinline__ int wrapi(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Exclusive scan of one value per thread over a block of T threads (a
// multiple of 64); ws holds T / 64 ints.
template <int T>
__device__ __forceinline__ int block_scan_excl(int v, int* ws, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) ws[w] = x;
  __syncthreads();
  if (w == 0) {
    int t = lane < T / 64 ? ws[lane] : 0;
#pragma unroll
    for (int off = 1; off < T / 64; off <<= 1) {
      const int y = __shfl_up(t, off);
      if (lane >= off) t += y;
    }
    if (lane < T / 64) ws[lane] = t;
  }
  __syncthreads();
  total = ws[T / 64 - 1];
  const int before = w > 0 ? ws[w - 1] : 0;
  __syncthreads();
  return before + x - v;
}

// a mod n for a in [-n, 2n): one conditional add or subtract, no division
__device__ __forceinline__ int wrap_near(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Coordinates (x, y, z) of element i of an x-fastest box len[0] x len[1] x
// len[2], advanced by a fixed stride without divisions: the stride is split
// once into (sx, sy, sz) with sx < len[0], sy < len[1], so each step carries
// at most once per dimension.
struct BoxWalk {
  int x, y, z, sx, sy, sz;
  __device__ __forceinline__ BoxWalk(int i, int stride, const int len[3]) {
    x = i % len[0];
    y = (i / len[0]) % len[1];
    z = i / (len[0] * len[1]);
    sx = stride % len[0];
    sy = (stride / len[0]) % len[1];
    sz = stride / (len[0] * len[1]);
  }
  __device__ __forceinline__ void step(const int len[3]) {
    x += sx;
    int c = x >= len[0] ? 1 : 0;
    x -= c * len[0];
    y += sy + c;
    c = y >= len[1] ? 1 : 0;
    y -= c * len[1];
    z += sz + c;
  }
};

// ---------------------------------------------------------------------------
// Basis weights.  For fractional offset f = t - floor(t) in [0,1) the touched
// points are m = floor(t) - (P/2 - 1) + j, j = 0..P-1, at distances
// t - m = f + P/2 - 1 - j.  w[j] = Phi(t - m), dw[j] = dPhi/dt (t - m).
//
// Cubic Hermite (eq:Phi-Hermite), expanded:
//   |t| <= 1:  1 - 5/2 t^2 + 3/2 t^3          derivative  -5 t + 9/2 t^2
//   1..2:      2 - 4 t + 5/2 t^2 - 1/2 t^3    derivative  -4 + 5 t - 3/2 t^2
// Quintic C1 Hermite, expanded (|t| in [0,1], [1,2], [2,3]):
//   (12 - 25 t^2 + 5 t^3 + 13 t^4 - 5 t^5) / 12
//   (24 + 10 t - 105 t^2 + 105 t^3 - 39 t^4 + 5 t^5) / 24
//   (72 - 174 t + 155 t^2 - 65 t^3 + 13 t^4 - t^5) / 24
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T cub_in(T t) { return T(1) + t * t * (T(-2.5) + T(1.5) * t); }
template <class T>
__device__ __forceinline__ T cub_out(T t) { return T(2) + t * (T(-4) + t * (T(2.5) - T(0.5) * t)); }
template <class T>
__device__ __forceinline__ T dcub_in(T t) { return t * (T(-5) + T(4.5) * t); }
template <class T>
__device__ __forceinline__ T dcub_out(T t) { return T(-4) + t * (T(5) - T(1.5) * t); }

template <class T>
__device__ __forceinline__ T qui_1(T t) {
  return T(1) + t * t * (T(-25.0 / 12.0) + t * (T(5.0 / 12.0) + t * (T(13.0 / 12.0) - T(5.0 / 12.0) * t)));
}
template <class T>
__device__ __forceinline__ T qui_2(T t) {
  return (T(24) + t * (T(10) + t * (T(-105) + t * (T(105) + t * (T(-39) + T(5) * t))))) * T(1.0 / 24.0);
}
template <class T>
__device__ __forceinline__ T qui_3(T t) {
  return (T(72) + t * (T(-174) + t * (T(155) + t * (T(-65) + t * (T(13) - t))))) * T(1.0 / 24.0);
}
template <class T>
__device__ __forceinline__ T dqui_1(T t) {
  return t * (T(-50.0 / 12.0) + t * (T(15.0 / 12.0) + t * (T(52.0 / 12.0) - T(25.0 / 12.0) * t)));
}
template <class T>
__device__ __forceinline__ T dqui_2(T t) {
  return (T(10) + t * (T(-210) + t * (T(315) + t * (T(-156) + T(25) * t)))) * T(1.0 / 24.0);
}
template <class T>
__device__ __forceinline__ T dqui_3(T t) {
  return (T(-174) + t * (T(310) + t * (T(-195) + t * (T(52) - T(5) * t)))) * T(1.0 / 24.0);
}

template <int P, class T>
__device__ __forceinline__ void basis_weights(T f, T* w) {
  if constexpr (P == 4) {
    w[0] = cub_out(T(1) + f);
    w[1] = cub_in(f);
    w[2] = cub_in(T(1) - f);
    w[3] = cub_out(T(2) - f);
  } else {
    w[0] = qui_3(T(2) + f);
    w[1] = qui_2(T(1) + f);
    w[2] = qui_1(f);
    w[3] = qui_1(T(1) - f);
    w[4] = qui_2(T(2) - f);
    w[5] = qui_3(T(3) - f);
  }
}

template <int P, class T>
__device__ __forceinline__ void basis_weights_d(T f, T* w, T* dw) {
  basis_weights<P, T>(f, w);
  if constexpr (P == 4) {
    dw[0] = dcub_out(T(1) + f);
    dw[1] = dcub_in(f);
    dw[2] = -dcub_in(T(1) - f);
    dw[3] = -dcub_out(T(2) - f);
  } else {
    dw[0] = dqui_3(T(2) + f);
    dw[1] = dqui_2(T(1) + f);
    dw[2] = dqui_1(f);
    dw[3] = -dqui_1(T(1) - f);
    dw[4] = -dqui_2(T(2) - f);
    dw[5] = -dqui_3(T(3) - f);
  }
}

// Restriction / prolongation weights c_o = Phi(o/2) at odd o > 0 (c_0 = 1 and
// c at even o != 0 vanish): the 4-point (cubic) and 6-point (quintic)
// midpoint interpolation rules.
template <int P>
__device__ __forceinline__ double rp_weight_odd(int k) {  // k = 0 -> o = 1, 1 -> o = 3, 2 -> o = 5
  if constexpr (P == 4) return k == 0 ? 9.0 / 16.0 : -1.0 / 16.0;
  else return k == 0 ? 75.0 / 128.0 : (k == 1 ? -25.0 / 256.0 : 3.0 / 256.0);
}

}  // namespace mls
