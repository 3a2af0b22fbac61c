// Molecular dynamics around the MLS dispersion (Sec. II.D, eq:disp-pair-pot;
// the MD runs of Sec. III.A): the short-ranged repulsive term C^rep_ij r^-12
// with geometric mixing C^rep_ij = sqrt(C12_i C12_j), summed over every
// periodic image closer than a cutoff r_c <= a; the velocity-Verlet
// integrator; and the pieces of multiple time stepping on the MLS split (the
// local part's forces and energy alone, the slow half-kicks, the final force
// sum).
//
// The repulsion reuses the cell-sorted atoms of the evaluation it belongs to
// (binning's wrapped positions, cell starts and permutation).  The half-cell
// pair kernels (pair.hip) evaluate it on the pairs they already queue for
// the local dispersion part (rc <= a); for the other cell layouts RepPair
// below runs on the caller's stream right after the local part, overlapping
// the grid chain on the plan's second stream.  Either writes cell-sorted
// forces and per-block energy sums; the interpolation adds the forces to the
// dispersion forces it writes (no second scatter into the caller's array)
// and the energy reduction adds the sums.
#include <algorithm>
#include <cmath>

#include "device_math.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kBlock = 256;

// sorted sqrt(C12): one random read per atom instead of one per neighbour
struct RepGather {
  using Args = RepGatherArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int s = blk * kBlock + threadIdx.x;
    if (s >= a.n + kSortedPad) return;
    double x = 0.0;
    if (s < a.n) {
      const double c = a.c12[a.perm[s]];
      if (isfinite(c) && c >= 0.0) {
        x = sqrt(c);
      } else {
        atomicOr(a.flags, 8);
      }
    }
    a.x12s[s] = x;
    if (a.x12f) a.x12f[s] = (float)x;
  }
};

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  return sh[0];
}

// This thread's share of sum_{i < n} p[i] over a kBlock-thread block: eight
// independent loads in flight per step (the one-block reductions below sum up
// to n / 64 block sums of the pair kernel).
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int n) {
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 7 * kBlock < n; i += 8 * kBlock)
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += p[i + u * kBlock];
  for (; i < n; i += kBlock) v[0] += p[i];
  return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// One thread per cell-sorted atom.  The neighbour cells of one (dy, dz) pair
// form a run of consecutive cells in x, hence one contiguous range of sorted
// atoms per periodic image in x: the loop walks (dz, dy, image in x, atom).
// Each row is trimmed to the cells that the cutoff sphere reaches: rows whose
// y-z slab lies beyond rc are skipped, and the x run is cut to the chord
// [x - s, x + s], s = sqrt(rc^2 - gy^2 - gz^2), with gy, gz the distances to
// the row's slab.  Distances to slabs are shrunk and the chord widened by a
// margin far above the rounding of the cell assignment, so no pair closer
// than rc is ever left out; the r^2 < rc^2 test decides the rest.
struct RepPair {
  using Args = RepPairArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    __shared__ double sh[kBlock];
    const int s = blk * kBlock + threadIdx.x;
    const CellGeom& g = a.g;
    double e = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    if (s < a.n) {
      const double4 p = a.xs[s];
      const double ci = a.x12s[s];
      const int c = a.cell_s[s];
      const int cx = c % g.nc[0];
      const int cy = (c / g.nc[0]) % g.nc[1];
      const int cz = c / (g.nc[0] * g.nc[1]);
      // margins above the cell rounding, plus how far atoms may sit outside
      // their cells (the skin margin of neighbour reuse)
      const double my = 1e-6 * g.w[1] + g.margin, mz = 1e-6 * g.w[2] + g.margin, mx = 1e-6 * g.w[0] + g.margin;
      for (int dz = -a.nr[2]; dz <= a.nr[2]; ++dz) {
        const int uz = cz + dz;  // unwrapped cell index
        const double gz = fmax(0.0, fmax(uz * g.w[2] - p.z, p.z - (uz + 1) * g.w[2]) - mz);
        const double rz = a.rc2 - gz * gz;
        if (rz <= 0.0) continue;
        const int qz = floor_div(uz, g.nc[2]);
        const int zc = uz - qz * g.nc[2];
        const double sz = qz * g.L[2];
        for (int dy = -a.nr[1]; dy <= a.nr[1]; ++dy) {
          const int uy = cy + dy;
          const double gy = fmax(0.0, fmax(uy * g.w[1] - p.y, p.y - (uy + 1) * g.w[1]) - my);
          const double rem = rz - gy * gy;
          if (rem <= 0.0) continue;
          const int qy = floor_div(uy, g.nc[1]);
          const int yc = uy - qy * g.nc[1];
          const double sy = qy * g.L[1];
          const int row = (zc * g.nc[1] + yc) * g.nc[0];
          const double chord = sqrt(rem) + mx;
          const int ulo = max(cx - a.nr[0], (int)floor((p.x - chord) * g.inv_w[0]));
          const int uhi = min(cx + a.nr[0], (int)floor((p.x + chord) * g.inv_w[0]));
          const int q0 = floor_div(ulo, g.nc[0]);
          const int q1 = floor_div(uhi, g.nc[0]);
          for (int qx = q0; qx <= q1; ++qx) {
            const int lo = max(ulo - qx * g.nc[0], 0);
            const int hi = min(uhi - qx * g.nc[0], g.nc[0] - 1);
            const int j0 = a.cell_start[row + lo], j1 = a.cell_start[row + hi + 1];
            const double sx = qx * g.L[0];
            const bool home = qx == 0 && qy == 0 && qz == 0;
            for (int j = j0; j < j1; ++j) {
              const double4 pj = a.xs[j];
              const double dx = p.x - (pj.x + sx);
              const double dyy = p.y - (pj.y + sy);
              const double dzz = p.z - (pj.z + sz);
              const double r2 = dx * dx + dyy * dyy + dzz * dzz;
              if (r2 < a.rc2 && !(home && j == s)) {
                const double ir2 = 1.0 / r2;
                const double ir6 = ir2 * ir2 * ir2;
                const double v = a.x12s[j] * ir6 * ir6;
                const double f = 12.0 * v * ir2;
                e += v;
                fx += f * dx;
                fy += f * dyy;
                fz += f * dzz;
              }
            }
          }
        }
      }
      e *= ci;
      a.frep[3 * (size_t)s + 0] = ci * fx;
      a.frep[3 * (size_t)s + 1] = ci * fy;
      a.frep[3 * (size_t)s + 2] = ci * fz;
    }
    const double t = block_sum(e, sh);
    if (threadIdx.x == 0) a.partial[blk] = t;
  }
};

// Velocity Verlet, one thread per atom (original order).  With END the
// second half-kick of the previous step, v += dt/2 F/m, is applied; the
// kinetic energy of the resulting v is summed per block; with START the
// first half-kick of the next step and the drift x += dt v follow.  Multiple
// time stepping adds the slow force's half-kicks of its outer step, after the
// fast END kick (SLOW_END) and before the fast START kick (SLOW_START), and
// with three time scales the mid force's half-kicks of its middle step
// (MID_END, MID_START) between them.
struct MdStep {
  using Args = MdStepArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    __shared__ double sh[kBlock];
    const int i = blk * kBlock + threadIdx.x;
    double k = 0.0;
    if (i < a.n) {
      const double im = a.inv_mass[i];
      double v[3], f[3];
      bool bad = !(isfinite(im) && im > 0.0);
      for (int d = 0; d < 3; ++d) {
        v[d] = a.vel[3 * (size_t)i + d];
        f[d] = a.forces[3 * (size_t)i + d];
        bad |= !isfinite(v[d]);
      }
      if (bad) atomicOr(a.flags, 8);
      if (a.mode & kMdEnd)
        for (int d = 0; d < 3; ++d) v[d] = v[d] + a.hdt * f[d] * im;
      if (a.mode & kMdMidEnd)
        for (int d = 0; d < 3; ++d) v[d] = v[d] + a.hmid * a.fmid[3 * (size_t)i + d] * im;
      if (a.mode & kMdSlowEnd)
        for (int d = 0; d < 3; ++d) v[d] = v[d] + a.hslow * a.fslow[3 * (size_t)i + d] * im;
      k = (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / im;
      if (a.mode & kMdSlowStart)
        for (int d = 0; d < 3; ++d) v[d] = v[d] + a.hslow * a.fslow[3 * (size_t)i + d] * im;
      if (a.mode & kMdMidStart)
        for (int d = 0; d < 3; ++d) v[d] = v[d] + a.hmid * a.fmid[3 * (size_t)i + d] * im;
      if (a.mode & kMdStart) {
        for (int d = 0; d < 3; ++d) {
          v[d] = v[d] + a.hdt * f[d] * im;
          a.pos[3 * (size_t)i + d] = a.pos[3 * (size_t)i + d] + a.dt * v[d];
        }
      }
      if (a.mode & (kMdEnd | kMdStart | kMdSlowEnd | kMdSlowStart | kMdMidEnd | kMdMidStart))
        for (int d = 0; d < 3; ++d) a.vel[3 * (size_t)i + d] = v[d];
    }
    const double t = block_sum(k, sh);
    if (threadIdx.x == 0) a.partial[blk] = t;
  }
};

// *out = 1/2 sum of the per-block kinetic sums (fixed order)
struct MdKinetic {
  using Args = MdKineticArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int) {
    __shared__ double sh[kBlock];
    const double t = block_sum(strided_sum(a.partial, a.npartial), sh);
    if (threadIdx.x == 0) *a.out = 0.5 * t;
  }
};

// The local part alone (multiple time stepping's fast force): forces[perm[s]]
// = local + repulsive force of sorted atom s, block sums of xi_s e0_s.
struct LocalOut {
  using Args = LocalOutArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    __shared__ double sh[kBlock];
    const int s = blk * kBlock + threadIdx.x;
    double u = 0.0;
    if (s < a.n) {
      const int i = a.perm[s];
      double f[3];
      for (int d = 0; d < 3; ++d) f[d] = a.floc[3 * (size_t)s + d] + a.frep[3 * (size_t)s + d];
      for (int d = 0; d < 3; ++d) a.forces[3 * (size_t)i + d] = f[d];
      u = a.xs[s].w * a.e0[s];
    }
    const double t = block_sum(u, sh);
    if (threadIdx.x == 0) a.partial[blk] = t;
  }
};

// E_local + E_rep = -1/2 sum_i xi_i e0_i + 1/2 (the repulsion's block sums)
struct LocalEnergy {
  using Args = LocalEnergyArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int) {
    __shared__ double sh[kBlock];
    const double u = strided_sum(a.partial, a.nb);
    const double r = strided_sum(a.rep_partial, a.rep_nb);
    const double tu = block_sum(u, sh);
    __syncthreads();
    const double tr = block_sum(r, sh);
    if (threadIdx.x == 0) *a.energy = -0.5 * tu + 0.5 * tr;
  }
};

struct AddForces {
  using Args = AddForcesArgs;
  static constexpr int kThreads = kBlock;
  static __device__ void run(const Args& a, int blk) {
    const int i = blk * kBlock + threadIdx.x;
    if (i < a.n3) a.forces[i] += a.add[i];
  }
};

inline int nblocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_rep_gather(mls_plan_s* P, int n, const double* c12, hipStream_t s) {
  return launch_one<RepGather>(RepGatherArgs{P->d_perm, c12, n, P->d_x12s, P->d_x12f, P->d_flags},
                               nblocks(n + kSortedPad, kBlock), s);
}

hipError_t launch_repulsion(mls_plan_s* P, int n, double rc, hipStream_t s) {
  RepPairArgs ra{};
  ra.xs = P->d_xs;
  ra.x12s = P->d_x12s;
  ra.cell_s = P->d_cell_s;
  ra.cell_start = P->d_cell_start;
  ra.g = P->cg;
  for (int d = 0; d < 3; ++d) ra.nr[d] = (int)std::ceil((rc + 2.0 * P->cg.margin) * P->cg.inv_w[d]);
  ra.rc2 = rc * rc;
  ra.n = n;
  ra.frep = P->d_frep;
  ra.partial = P->d_md_partial;
  P->rep_nb = nblocks(n, kBlock);
  return launch_one<RepPair>(ra, nblocks(n, kBlock), s);
}

hipError_t launch_md_step(mls_plan_s* P, int n, double* pos, double* vel, const double* forces,
                          const double* inv_mass, double dt, int mode, double* kinetic, hipStream_t s,
                          const double* fslow, double hslow, const double* fmid, double hmid) {
  double* part = P->d_md_partial + P->rep_cap;
  if (n > 0) {
    MdStepArgs ma{pos, vel, forces, inv_mass, n, 0.5 * dt, dt, mode, part, P->d_flags, fslow, hslow, fmid, hmid};
    hipError_t e = launch_one<MdStep>(ma, nblocks(n, kBlock), s);
    if (e != hipSuccess) return e;
  }
  if (!kinetic) return hipSuccess;
  return launch_one<MdKinetic>(MdKineticArgs{part, nblocks(n, kBlock), kinetic}, 1, s);
}

hipError_t launch_local_out(mls_plan_s* P, int n, double* energy, double* forces, hipStream_t s) {
  double* part = P->d_md_partial + P->rep_cap + P->n_partial;
  const int nb = nblocks(n, kBlock);
  if (n > 0) {
    LocalOutArgs la{P->d_xs, P->d_perm, n, P->d_e0, P->d_floc, P->d_frep, forces, part};
    hipError_t e = launch_one<LocalOut>(la, nb, s);
    if (e != hipSuccess) return e;
  }
  return launch_one<LocalEnergy>(LocalEnergyArgs{part, nb, P->d_md_partial, n > 0 ? P->rep_nb : 0, energy}, 1, s);
}

hipError_t launch_add_forces(double* forces, const double* add, int n, hipStream_t s) {
  return launch_one<AddForces>(AddForcesArgs{forces, add, 3 * n}, nblocks(3 * (int64_t)n, kBlock), s);
}

}  // namespace mls
