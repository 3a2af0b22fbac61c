// Evaluation on the grids (eq:evaluation, k = 1..l):
//   levels k < l:  e^k[mu] = 2^(-6(k-1)) sum_{delta: |delta o h_1| < 2a} g_1(|delta o h_1|) q^k[(mu - delta) mod n_k]
//                  (the cutoff 2^k a and spacing 2^(k-1) h_1 give the same offsets on every level and
//                  g_k(2^(k-1) s) = 2^(-6(k-1)) g_1(s), Sec. II.A.4)
//   level l:       e^l[mu] = sum_nu K_l[(mu - nu) mod n_l] q^l[nu]   with the pre-summed periodic kernel of
//                  eq:last-grid-periodic-transformed (all-to-all, FP64).
#include <algorithm>

#include "device_math.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

// Reference-structured stencil: one thread per output point, taps from the
// level-1 table.
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

__global__ void __launch_bounds__(kBlock) k_coarsest_f64(const double* __restrict__ q, GridDims g,
                                                         const double* __restrict__ K, double* __restrict__ e) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= g.size) return;
  const int x = mu % g.n[0], y = (mu / g.n[0]) % g.n[1], z = mu / (g.n[0] * g.n[1]);
  double acc = 0.0;
  for (int nz = 0; nz < g.n[2]; ++nz) {
    const int dz = wrapi(z - nz, g.n[2]);
    for (int ny = 0; ny < g.n[1]; ++ny) {
      const int dy = wrapi(y - ny, g.n[1]);
      const double* qrow = q + ((size_t)nz * g.n[1] + ny) * g.n[0];
      const double* krow = K + ((size_t)dz * g.n[1] + dy) * g.n[0];
      for (int nx = 0; nx < g.n[0]; ++nx) acc += krow[wrapi(x - nx, g.n[0])] * qrow[nx];
    }
  }
  e[mu] = acc;
}

inline int nblocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_stencils(mls_plan_s* P, hipStream_t s) {
  const int ntaps = (int)P->taps.size();
  for (int k = 1; k < P->levels; ++k) {
    Level& L = P->lv[k - 1];
    const double scale = std::ldexp(1.0, -6 * (k - 1));
    k_stencil_taps_f64<<<nblocks(L.g.size, kBlock), kBlock, 0, s>>>(L.q, L.g, P->d_taps, ntaps, scale, L.e);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_coarsest(mls_plan_s* P, hipStream_t s) {
  Level& L = P->lv[P->levels - 1];
  k_coarsest_f64<<<nblocks(L.g.size, kBlock), kBlock, 0, s>>>(L.q, L.g, P->d_Kl, L.e);
  return hipGetLastError();
}

}  // namespace mls
