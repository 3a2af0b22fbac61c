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

struct PairConst {
  double a2, inv_a2, inv_a6, inv_a8;
};

// g_0(r) and g_0'(r)/r from s = r^2 (caller guarantees 0 < s < a^2).
template <class T>
__device__ __forceinline__ void g0_pair(T s, T inv_a2, T inv_a6, T inv_a8, T& g, T& fr) {
  T ir2 = T(1) / s;
  T ir6 = ir2 * ir2 * ir2;
  T u = s * inv_a2;            // rho^2
  T u2 = u * u;
  T u4 = u2 * u2;
  T u5 = u4 * u;
  T u6 = u4 * u2;
  T u11 = u6 * u5;
  T u12 = u6 * u6;
  g = ir6 - inv_a6 * (T(15.0 / 8.0) + u6 * (T(-5.0 / 4.0) + T(3.0 / 8.0) * u6));
  fr = T(-6) * ir6 * ir2 + inv_a8 * (T(15) * u5 - T(9) * u11);
  (void)u12;
}

// FP64: one thread per cell-sorted target atom.
__global__ void __launch_bounds__(kBlock) k_pair_f64(const double4* __restrict__ xs, const int* __restrict__ cell_s,
                                                     const int* __restrict__ cstart, int n, CellGeom g, PairConst pc,
                                                     double* __restrict__ e0, double* __restrict__ floc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double4 xi = xs[s];
  const int c = cell_s[s];
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
        const int j0 = cstart[t], j1 = cstart[t + 1];
        for (int j = j0; j < j1; ++j) {
          const double4 xj = xs[j];
          const double dx = xi.x - (xj.x + sx);
          const double dy = xi.y - (xj.y + sy);
          const double dz = xi.z - (xj.z + sz);
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 < pc.a2 && !(home && j == s)) {
            double gg, fr;
            g0_pair<double>(r2, pc.inv_a2, pc.inv_a6, pc.inv_a8, gg, fr);
            e += xj.w * gg;
            const double f = xj.w * fr;
            fx += f * dx;
            fy += f * dy;
            fz += f * dz;
          }
        }
      }
    }
  }
  e0[s] = e;
  floc[3 * (size_t)s + 0] = xi.w * fx;
  floc[3 * (size_t)s + 1] = xi.w * fy;
  floc[3 * (size_t)s + 2] = xi.w * fz;
}

}  // namespace

hipError_t launch_pair(mls_plan_s* P, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  PairConst pc{P->a2, P->inv_a2, P->inv_a6, P->inv_a8};
  k_pair_f64<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(P->d_xs, P->d_cell_s, P->d_cell_start, n, P->cg, pc,
                                                          P->d_e0, P->d_floc);
  return hipGetLastError();
}

}  // namespace mls
