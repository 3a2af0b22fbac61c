// Host-side plan construction: parameter checks, grid hierarchy, linked cells,
// the level-1 stencil table and the pre-summed coarsest-grid kernel, and the
// device workspace.  Everything here runs once per plan (the paper notes the
// g_k tables and operator maps are constant for fixed grids and can be
// precomputed, Sec. II.A.4, and that the coarsest image sum is
// time-independent, Sec. II.C).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include "mls_internal.h"

namespace mls {
namespace {

// binom(-1/2, m): coefficient m of the series of (1 + u)^(-1/2).
double binom_half(int m) {
  double c = 1.0;
  for (int j = 0; j < m; ++j) c *= (-0.5 - j) / (j + 1);
  return c;
}

// Smoothing function gamma_k: rho^-6 from rho = 1 on; inside, the order-k
// Taylor polynomial of (1 + u)^(-1/2) in u = rho^12 - 1 (C^k at rho = 1, the
// family of Sec. III.B); k = 2 is eq:gamma, evaluated as printed.
double gamma_s(double rho, int k) {
  if (rho >= 1.0) return std::pow(rho, -6);
  const double v = std::pow(rho, 12);
  if (k == 2) return 15.0 / 8.0 + v * (-5.0 / 4.0 + v * (3.0 / 8.0));
  double sum = 0.0, um = 1.0;
  for (int m = 0; m <= k; ++m, um *= v - 1.0) sum += binom_half(m) * um;
  return sum;
}

// gamma_k inside the unit ball as a polynomial in v = rho^12:
// c_j = sum_{m >= j} binom(-1/2, m) C(m, j) (-1)^(m - j).
void gamma_coeffs(int k, double* c) {
  for (int j = 0; j <= 4; ++j) c[j] = 0.0;
  for (int m = 0; m <= k; ++m) {
    double cmj = 1.0;   // C(m, j)
    for (int j = 0; j <= m; ++j) {
      c[j] += binom_half(m) * cmj * (((m - j) & 1) ? -1.0 : 1.0);
      cmj = cmj * (m - j) / (j + 1);
    }
  }
}

// Level-1 kernel of eq:g_k (k = 1): a^-6 gamma(s/a) - (2a)^-6 gamma(s/2a),
// zero from 2a on.
double g_level1(double s, double a, int k) {
  if (s >= 2.0 * a) return 0.0;
  return std::pow(a, -6) * gamma_s(s / a, k) - std::pow(2.0 * a, -6) * gamma_s(s / (2.0 * a), k);
}

// Coarsest kernel eq:g_l with A = 2^(l-1) a.
double g_coarsest(double r, double A, int k) { return std::pow(A, -6) * gamma_s(r / A, k); }

// ---------------------------------------------------------------------------
// Periodic r^-6 lattice sum  S(v) = sum_{n: v + nL != 0} |v + n o L|^-6.
//
// Screened split of r^-6 = (1/2) int_0^inf t^2 e^{-r^2 t} dt at t = b^2:
//   near part  r^-6 e^{-y}(1 + y + y^2/2),    y = b^2 r^2
//   far part   smooth, summed in Fourier space with
//              F(k) = pi^{3/2} b^3 / 3 * [(1 - 2c^2) e^{-c^2} + 2 sqrt(pi) c^3 erfc(c)],
//              c = |k| / (2b), and value b^6/6 at r = 0.
// ---------------------------------------------------------------------------
class LatticeR6 {
 public:
  LatticeR6(const double L[3]) {
    for (int d = 0; d < 3; ++d) L_[d] = L[d];
    double Lmin = std::min(L[0], std::min(L[1], L[2]));
    b_ = 2.5 / Lmin;
    const double lnTol = 40.0;  // e^-40 ~ 4e-18
    rcut_ = std::sqrt(lnTol) / b_;
    double kcut = 2.0 * b_ * std::sqrt(lnTol);
    vol_ = L[0] * L[1] * L[2];
    int m[3];
    for (int d = 0; d < 3; ++d) m[d] = (int)std::ceil(kcut * L[d] / (2.0 * M_PI));
    // half space of k (k and -k contribute equally to a cosine sum)
    for (int mz = 0; mz <= m[2]; ++mz)
      for (int my = (mz == 0 ? 0 : -m[1]); my <= m[1]; ++my)
        for (int mx = ((mz == 0 && my == 0) ? 0 : -m[0]); mx <= m[0]; ++mx) {
          double kx = 2.0 * M_PI * mx / L[0], ky = 2.0 * M_PI * my / L[1], kz = 2.0 * M_PI * mz / L[2];
          double k = std::sqrt(kx * kx + ky * ky + kz * kz);
          if (k > kcut) continue;
          double c = k / (2.0 * b_);
          double F = std::pow(M_PI, 1.5) * b_ * b_ * b_ / 3.0 *
                     ((1.0 - 2.0 * c * c) * std::exp(-c * c) +
                      2.0 * std::sqrt(M_PI) * c * c * c * std::erfc(c));
          double mult = (mx == 0 && my == 0 && mz == 0) ? 1.0 : 2.0;
          kv_.push_back({kx, ky, kz, mult * F / vol_});
        }
  }

  double operator()(const double v[3]) const {
    double near = 0.0;
    int nr[3];
    for (int d = 0; d < 3; ++d) nr[d] = (int)std::ceil((rcut_ + L_[d]) / L_[d]);
    for (int iz = -nr[2]; iz <= nr[2]; ++iz)
      for (int iy = -nr[1]; iy <= nr[1]; ++iy)
        for (int ix = -nr[0]; ix <= nr[0]; ++ix) {
          double x = v[0] + ix * L_[0], y = v[1] + iy * L_[1], z = v[2] + iz * L_[2];
          double r2 = x * x + y * y + z * z;
          if (r2 == 0.0 || r2 > rcut_ * rcut_) continue;
          double yb = b_ * b_ * r2;
          near += std::exp(-yb) * (1.0 + yb + 0.5 * yb * yb) / (r2 * r2 * r2);
        }
    double far = 0.0;
    for (const auto& k : kv_) far += k[3] * std::cos(k[0] * v[0] + k[1] * v[1] + k[2] * v[2]);
    bool on_lattice = true;
    for (int d = 0; d < 3; ++d) {
      double f = v[d] / L_[d];
      if (f != std::round(f)) on_lattice = false;
    }
    double self = on_lattice ? std::pow(b_, 6) / 6.0 : 0.0;
    return near + far - self;
  }

 private:
  double L_[3];
  double b_, rcut_, vol_;
  std::vector<std::array<double, 4>> kv_;
};

template <class T>
mls_status dalloc(mls_plan_s* P, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  size_t bytes = count * sizeof(T);
  if (P->arena) {
    // carve from the caller-provided arena (no allocation)
    const size_t off = (P->arena_used + 255) & ~(size_t)255;
    if (off > P->arena_cap || bytes > P->arena_cap - off) {
      set_error("workspace exceeds the static scratch of " + std::to_string(P->arena_cap) + " bytes");
      return MLS_ERR_UNSUPPORTED;
    }
    *p = (T*)(P->arena + off);
    P->arena_used = off + bytes;
    P->bytes += (int64_t)bytes;
    return MLS_OK;
  }
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    return MLS_ERR_OOM;
  }
  P->allocations.push_back((void*)*p);
  P->bytes += (int64_t)bytes;
  return MLS_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

mls_status build_plan(const mls_params& p, int64_t n_max, mls_plan_s* P) {
  // ---------------------------------------------------------------- checks
  for (int d = 0; d < 3; ++d)
    if (!finite_pos(p.box[d])) { set_error("box lengths must be finite and > 0"); return MLS_ERR_INVALID_ARG; }
  if (!finite_pos(p.cutoff)) { set_error("cutoff a must be finite and > 0"); return MLS_ERR_INVALID_ARG; }
  bool explicit_grid = p.grid[0] > 0 || p.grid[1] > 0 || p.grid[2] > 0;
  if (!explicit_grid && !finite_pos(p.h)) { set_error("spacing h must be finite and > 0"); return MLS_ERR_INVALID_ARG; }
  if (p.order != 4 && p.order != 6) { set_error("order must be 4 (cubic) or 6 (quintic)"); return MLS_ERR_INVALID_ARG; }
  if (p.levels < 0 || p.levels > 16) { set_error("levels must be in [0, 16]"); return MLS_ERR_INVALID_ARG; }
  if (p.precision != MLS_FP64 && p.precision != MLS_MIXED) { set_error("precision must be MLS_FP64 or MLS_MIXED"); return MLS_ERR_INVALID_ARG; }
  if (n_max < 0 || n_max > (int64_t)1 << 30) { set_error("n_max must be in [0, 2^30]"); return MLS_ERR_INVALID_ARG; }
  const int cont = p.continuity == 0 ? 2 : p.continuity;
  if (cont < 1 || cont > 4) { set_error("continuity must be 1..4 (0 means 2)"); return MLS_ERR_INVALID_ARG; }
  if (p.mixing != MLS_GEOMETRIC && p.mixing != MLS_LORENTZ_BERTHELOT) {
    set_error("mixing must be MLS_GEOMETRIC or MLS_LORENTZ_BERTHELOT");
    return MLS_ERR_INVALID_ARG;
  }
  P->mixing = p.mixing;
  if (!(std::isfinite(p.skin) && p.skin >= 0.0 && p.skin < p.cutoff)) {
    set_error("skin must be finite with 0 <= skin < a");
    return MLS_ERR_INVALID_ARG;
  }
  if (p.skin > 0.0 && p.mixing != MLS_GEOMETRIC) {
    set_error("a skin (neighbour reuse in molecular dynamics) needs geometric mixing");
    return MLS_ERR_UNSUPPORTED;
  }
  P->skin = p.skin;

  P->params = p;
  P->order = p.order;
  P->precision = p.precision;
  P->n_max = n_max;
  P->a = p.cutoff;
  P->a2 = p.cutoff * p.cutoff;
  P->inv_a2 = 1.0 / P->a2;
  P->inv_a6 = std::pow(p.cutoff, -6);
  P->inv_a8 = std::pow(p.cutoff, -8);
  P->continuity = cont;
  gamma_coeffs(cont, P->gamma_c);
  P->cself = gamma_s(0.0, cont) * P->inv_a6;  // eq:self-interaction-energy
  hipGetDevice(&P->device);
  if (const char* env = std::getenv("MLS_PAIR_AFTER")) P->pair_after = std::min(5, std::max(0, std::atoi(env)));
  if (const char* env = std::getenv("MLS_SPLIT_RESTRICT")) P->split_restrict = std::atoi(env);
  if (const char* env = std::getenv("MLS_SPLIT_PROLONG")) P->split_prolong = std::atoi(env);
  if (const char* env = std::getenv("MLS_PAIR_WAVES_CU")) {
    // persistent pair kernel: this many single-wave blocks per CU
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && ncu > 0)
      P->pair_blocks = std::max(0, std::atoi(env)) * ncu;
  }

  // ---------------------------------------------------------------- levels
  int l = p.levels;
  if (l == 0) {
    if (explicit_grid) { set_error("levels = 0 needs a spacing h, not an explicit grid"); return MLS_ERR_INVALID_ARG; }
    // largest l whose coarsest grid keeps >= p points per dimension
    int k = 0;
    while (true) {
      double mn = 1e300;
      for (int d = 0; d < 3; ++d) mn = std::min(mn, std::floor(p.box[d] / (std::ldexp(p.h, k + 1)) + 0.5));
      if (mn >= p.order && k < 15) ++k; else break;
    }
    l = k + 1;
  }
  P->levels = l;
  const int m = 1 << (l - 1);
  int n1[3];
  for (int d = 0; d < 3; ++d) {
    if (explicit_grid) {
      n1[d] = p.grid[d];
      if (n1[d] <= 0 || n1[d] % m) { set_error("grid dims must be > 0 and divisible by 2^(levels-1)"); return MLS_ERR_INVALID_ARG; }
    } else {
      double c = std::floor(p.box[d] / (m * p.h) + 0.5);
      if (c > 4096.0) { set_error("finest grid too large"); return MLS_ERR_INVALID_ARG; }
      n1[d] = m * (int)std::max(1.0, c);
    }
  }
  if ((double)n1[0] * n1[1] * n1[2] > 1.0e9) { set_error("finest grid exceeds 1e9 points"); return MLS_ERR_INVALID_ARG; }
  P->lv.resize(l);
  for (int k = 1; k <= l; ++k) {
    Level& L = P->lv[k - 1];
    for (int d = 0; d < 3; ++d) {
      L.g.n[d] = n1[d] >> (k - 1);
      L.h[d] = p.box[d] / L.g.n[d];
    }
    L.g.size = L.g.n[0] * L.g.n[1] * L.g.n[2];
  }
  for (int d = 0; d < 3; ++d) P->invh1[d] = (double)n1[d] / p.box[d];

  // ---------------------------------------------------------------- cells
  // Linked cells (Sec. III.D use the smallest width >= a dividing the box).
  // When the box spans at least five half-cutoff cells per dimension the
  // cells are made half as wide (the smallest width >= a/2 dividing the box):
  // the pair kernel then trims each neighbour row to the cutoff sphere, which
  // examines far fewer candidates.  The pairs found are the same.
  // With a skin s (neighbour reuse) every width is taken for a + s, so that
  // atoms up to s/2 outside their cells are still found by the same window.
  CellGeom& cg = P->cg;
  const double reach = p.cutoff + P->skin;
  bool fast = true;
  for (int d = 0; d < 3; ++d)
    if (std::floor(p.box[d] / (0.5 * reach * (1.0 + 1e-12))) < 5.0) fast = false;
  P->pair_fast = fast;
  const double cw = fast ? 0.5 * reach : reach;
  cg.margin = 0.5 * P->skin;
  cg.ncell = 1;
  for (int d = 0; d < 3; ++d) {
    cg.L[d] = p.box[d];
    cg.invL[d] = 1.0 / p.box[d];
    double c = std::floor(p.box[d] / (cw * (1.0 + 1e-12)));
    cg.nc[d] = (int)std::max(1.0, std::min(c, 2048.0));
    cg.inv_w[d] = (double)cg.nc[d] / p.box[d];
    cg.w[d] = p.box[d] / cg.nc[d];
    cg.noff[d] = std::max(1, (int)std::ceil(reach / cg.w[d] - 1e-12));
    if ((double)cg.ncell * cg.nc[d] > 2.0e8) { set_error("too many linked cells"); return MLS_ERR_INVALID_ARG; }
    cg.ncell *= cg.nc[d];
  }

  // ---------------------------------------------------------------- stencil
  // offsets delta with |delta o h_1| < 2a; g_1 weights (Sec. II.A.4: the same
  // table serves level k with spacing 2^(k-1) h_1, scaled by 2^(-6(k-1)))
  const double* h1 = P->lv[0].h;
  int R[3];
  for (int d = 0; d < 3; ++d) R[d] = (int)std::ceil(2.0 * p.cutoff / h1[d]);
  P->taps.clear();
  P->rows.clear();
  P->row_w.clear();
  P->taps_wsum = 0.0;
  for (int d = 0; d < 3; ++d) P->stencil_R[d] = 0;
  if (l > 1) {
    const double lim = 4.0 * p.cutoff * p.cutoff;
    for (int dz = -R[2]; dz <= R[2]; ++dz)
      for (int dy = -R[1]; dy <= R[1]; ++dy)
        for (int dx = -R[0]; dx <= R[0]; ++dx) {
          double sx = dx * h1[0], sy = dy * h1[1], sz = dz * h1[2];
          double s2 = sx * sx + sy * sy + sz * sz;
          if (s2 >= lim) continue;
          Tap t{dx, dy, dz, 0, g_level1(std::sqrt(s2), p.cutoff, cont)};
          P->taps.push_back(t);
          P->taps_wsum += t.w;
          P->stencil_R[0] = std::max(P->stencil_R[0], std::abs(dx));
          P->stencil_R[1] = std::max(P->stencil_R[1], std::abs(dy));
          P->stencil_R[2] = std::max(P->stencil_R[2], std::abs(dz));
        }
    for (int dy = 0; dy <= R[1]; ++dy)
      for (int dx = 0; dx <= R[0]; ++dx) {
        double base = std::pow(dx * h1[0], 2) + std::pow(dy * h1[1], 2);
        if (base >= lim) continue;
        int hz = 0;
        while (std::pow((hz + 1) * h1[2], 2) + base < lim) ++hz;
        StencilRow r{dx, dy, hz, (int)P->row_w.size()};
        for (int dz = 0; dz <= hz; ++dz)
          P->row_w.push_back(g_level1(std::sqrt(std::pow(dz * h1[2], 2) + base), p.cutoff, cont));
        P->rows.push_back(r);
      }
  }

  // contiguous, cost-balanced split of the tap columns over the waves of a
  // stencil block (cost: mirror loads plus the 2 hz + 1 column updates)
  std::vector<int> wave_rows(kStencilWaves + 1, (int)P->rows.size());
  {
    double total = 0.0;
    std::vector<double> cost;
    for (const auto& r : P->rows) {
      double m = (r.dx ? 2 : 1) * (r.dy ? 2 : 1);
      cost.push_back(m + 2 * r.hz + 1);
      total += cost.back();
    }
    wave_rows[0] = 0;
    double run = 0.0;
    int w = 1;
    for (size_t i = 0; i < cost.size() && w < kStencilWaves; ++i) {
      run += cost[i];
      if (run >= total * w / kStencilWaves) wave_rows[w++] = (int)i + 1;
    }
    for (; w < kStencilWaves; ++w) wave_rows[w] = (int)P->rows.size();
  }

  // tiled stencil: weights compensating the duplicated mirror images on the
  // axes, and the table of (level, tile) blocks of one launch
  std::vector<double> row_w_tile(P->row_w);
  for (const auto& r : P->rows) {
    const double mult = (r.dx == 0 ? 2.0 : 1.0) * (r.dy == 0 ? 2.0 : 1.0);
    for (int d = 0; d <= r.hz; ++d) row_w_tile[r.woff + d] /= mult;
  }
  std::vector<int4> tiles;
  if (const char* env = std::getenv("MLS_STENCIL_KERNEL")) P->stencil_kernel = std::atoi(env) == 0 ? 0 : 1;
  // MFMA recast of the FP32 tile (windows up to 6, z tiles of 16): for tap
  // column c and chunk s of four input planes, lane i + 16 k of the A operand
  // holds the weight of dz = 4 s + k - hz - i (zero outside [-hz, hz]): output
  // plane i of the tile, input plane 4 s + k counted from hz below it
  std::vector<float> mfma_a;
  std::vector<StencilRow> rows_mfma;
  {
    const char* env = std::getenv("MLS_STENCIL_MFMA");
    P->stencil_mfma = env && std::atoi(env) != 0 && P->precision == MLS_MIXED && P->stencil_kernel == 1 && l > 1 &&
                      stencil_window(P) >= 1 && stencil_window(P) <= 6;
  }
  if (P->stencil_mfma) {
    for (const auto& r : P->rows) {
      StencilRow m = r;
      m.woff = (int)mfma_a.size();
      const int S = (16 + 2 * r.hz + 3) / 4;
      for (int sc = 0; sc < S; ++sc)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, k = lane >> 4;
          const int dz = 4 * sc + k - r.hz - i;
          mfma_a.push_back(std::abs(dz) <= r.hz ? (float)row_w_tile[r.woff + std::abs(dz)] : 0.0f);
        }
      rows_mfma.push_back(m);
    }
  }
  if (l > 1) {
    const int Rw = stencil_window(P);
    const int zc = stencil_tile_zc(Rw, P->precision != MLS_MIXED);
    for (int k = 1; k < l; ++k) {
      const GridDims& g = P->lv[k - 1].g;
      const int tx = (g.n[0] + 7) / 8, ty = (g.n[1] + 7) / 8, tz = (g.n[2] + zc - 1) / zc;
      for (int z = 0; z < tz; ++z)
        for (int y = 0; y < ty; ++y)
          for (int x = 0; x < tx; ++x) tiles.push_back(make_int4(k - 1, x, y, z));
    }
  }
  P->ntiles = (int)tiles.size();

  // ---------------------------------------------------------------- coarsest kernel
  {
    const Level& C = P->lv[l - 1];
    const double A = std::ldexp(p.cutoff, l - 1);
    LatticeR6 lat(p.box);
    P->Kl.assign(C.g.size, 0.0);
    int nimg[3];
    for (int d = 0; d < 3; ++d) nimg[d] = (int)std::ceil(A / p.box[d]) + 1;
    for (int z = 0; z < C.g.n[2]; ++z)
      for (int y = 0; y < C.g.n[1]; ++y)
        for (int x = 0; x < C.g.n[0]; ++x) {
          double v[3] = {x * C.h[0], y * C.h[1], z * C.h[2]};
          double K = lat(v);
          // images inside A: replace r^-6 by g_l(r); the r = 0 image carries g_l(0)
          for (int iz = -nimg[2]; iz <= nimg[2]; ++iz)
            for (int iy = -nimg[1]; iy <= nimg[1]; ++iy)
              for (int ix = -nimg[0]; ix <= nimg[0]; ++ix) {
                double rx = v[0] + ix * p.box[0], ry = v[1] + iy * p.box[1], rz = v[2] + iz * p.box[2];
                double r = std::sqrt(rx * rx + ry * ry + rz * rz);
                if (r == 0.0) K += g_coarsest(0.0, A, cont);
                else if (r < A) K += g_coarsest(r, A, cont) - std::pow(r, -6);
              }
          P->Kl[(size_t)(z * C.g.n[1] + y) * C.g.n[0] + x] = K;
        }
  }

  // ---------------------------------------------------------------- two-phase anterpolation tables
  std::vector<int> ant_tab;
  size_t ant_scratch = 0;
  P->ant_tiles = false;
  {
    const char* env = std::getenv("MLS_ANTERP_TILES");
    if (!(env && std::atoi(env) == 0)) {
      for (int cap : {kAntTileSmall, kAntTileMax}) {
        if (cap == kAntTileSmall && P->ant_large_tiles) continue;
        P->ant_tiles = ant_tiles_build(P, P->ant, ant_tab, ant_scratch, cap);
        if (P->ant_tiles) {
          P->ant_cap = cap;
          break;
        }
      }
    }
  }

  // ---------------------------------------------------------------- device memory
  mls_status st;
#define ALLOC(ptr, cnt)                                                  \
  do {                                                                   \
    if ((st = dalloc(P, &(ptr), (size_t)(cnt))) != MLS_OK) return st;    \
  } while (0)
  const size_t N = (size_t)std::max<int64_t>(n_max, 1);
  ALLOC(P->d_count, cg.ncell);
  ALLOC(P->d_cell_start, cg.ncell + 1);
  ALLOC(P->d_slot, N);
  {
    // bucketed binning unless MLS_BIN_BUCKETS=0 or the cells are too many
    const char* env = std::getenv("MLS_BIN_BUCKETS");
    int shift = 0, nb = 0;
    if (!(env && std::atoi(env) == 0) && bin_buckets(cg.ncell, (int64_t)N, shift, nb)) {
      P->bin_shift = shift;
      P->bin_nbucket = nb;
    }
  }
  int64_t scan_len = cg.ncell;
  if (P->bin_nbucket) {
    const int64_t hist = (int64_t)P->bin_nbucket * ((N + bin_block_items() - 1) / bin_block_items());
    ALLOC(P->d_bin_hist, hist + 1);
    ALLOC(P->d_perm_tmp2, N);
    scan_len = std::max<int64_t>(scan_len, hist);
  }
  ALLOC(P->d_bsum, scan_blocks((int)scan_len) + 1);
  ALLOC(P->d_bmax, scan_blocks((int)scan_len) + 1);
  ALLOC(P->d_cid, N);
  ALLOC(P->d_xw, N);
  ALLOC(P->d_perm_tmp, N);
  ALLOC(P->d_perm, N);
  ALLOC(P->d_cell_s, N);
  ALLOC(P->d_xs, N + kSortedPad);
  ALLOC(P->d_e0, N);
  ALLOC(P->d_floc, 3 * N);
  if (P->precision == MLS_MIXED) {
    ALLOC(P->d_xr, N + kSortedPad);
    ALLOC(P->d_xif, N + kSortedPad);
  }
  // filter coordinates of the pair kernels (both precisions)
  P->xf_stride = (int)(N + kSortedPad);
  ALLOC(P->d_xf, 3 * (size_t)P->xf_stride);
  P->n_partial = (int)((N + 255) / 256);
  ALLOC(P->d_partial, 2 * (size_t)P->n_partial + 2);
  ALLOC(P->d_scratch, 64);
  ALLOC(P->d_flags, 4);
  ALLOC(P->d_ncell_max, 4);
  for (int k = 1; k <= l; ++k) {
    Level& L = P->lv[k - 1];
    ALLOC(L.q, L.g.size);
    ALLOC(L.e, L.g.size);
    if (k < l) {
      ALLOC(L.E, L.g.size);
    } else {
      L.E = L.e;  // the coarsest level has nothing to prolongate into it
    }
  }
  if (P->mixing == MLS_GEOMETRIC) {
    // molecular dynamics: repulsive term and integrator (mls_evaluate_md, mls_md_run)
    ALLOC(P->d_x12s, N + kSortedPad);
    if (P->precision == MLS_MIXED) ALLOC(P->d_x12f, N + kSortedPad);
    ALLOC(P->d_frep, 3 * N);
    P->rep_cap = (int)((N + 63) / 64);   // one sum per wave of the pair kernels
    ALLOC(P->d_md_partial, (size_t)P->rep_cap + 2 * (size_t)P->n_partial);
    ALLOC(P->d_fslow, 3 * N);
    ALLOC(P->d_fmid, 3 * N);
    if (P->skin > 0.0) {
      ALLOC(P->d_xref, 3 * N);
      ALLOC(P->d_rebin, 1);
    }
    ALLOC(P->d_efast, 1);
  }
  if (P->mixing == MLS_LORENTZ_BERTHELOT) {
    // seven charge vectors: one set of grids each (Sec. II.D)
    ALLOC(P->d_sig, N + kSortedPad);
    const int slots = P->lb_slots > 1 ? 7 : 1;
    P->lb_slots = slots;
    P->lb_stride = N + kSortedPad;
    ALLOC(P->d_charge, (size_t)slots * P->lb_stride);
    if (P->precision == MLS_MIXED) {
      ALLOC(P->d_sigf, N + kSortedPad);
      P->lb_npart = (int)((P->lb_stride + 255) / 256);
      ALLOC(P->d_lb_partial, (size_t)slots * P->lb_npart);
    }
    for (int r = 0; r < 7; ++r) {
      P->lb_lv[r] = P->lv;
      for (int k = 1; k <= l; ++k) {
        Level& L = P->lb_lv[r][k - 1];
        ALLOC(L.q, L.g.size);
        ALLOC(L.e, L.g.size);
        if (k < l) {
          ALLOC(L.E, L.g.size);
        } else {
          L.E = L.e;
        }
      }
    }
  }
  ALLOC(P->d_taps, P->taps.size());
  ALLOC(P->d_rows, P->rows.size());
  ALLOC(P->d_wave_rows, kStencilWaves + 1);
  ALLOC(P->d_row_w_tile, P->row_w.size());
  ALLOC(P->d_row_wf_tile, P->row_w.size());
  ALLOC(P->d_tiles, tiles.size());
  ALLOC(P->d_row_w, P->row_w.size());
  ALLOC(P->d_row_wf, P->row_w.size());
  ALLOC(P->d_Kl, P->Kl.size());
  if (P->stencil_mfma) {
    ALLOC(P->d_mfma_a, mfma_a.size());
    ALLOC(P->d_rows_mfma, rows_mfma.size());
  }
  if (P->ant_tiles) {
    ALLOC(P->d_ant_tab, ant_tab.size());
    P->ant_scratch_n = ant_scratch;
    ALLOC(P->d_ant_scratch, ant_scratch * (P->mixing == MLS_LORENTZ_BERTHELOT ? P->lb_slots : 1));
  }
#undef ALLOC
  hipError_t e;
  if (!P->taps.empty()) {
    if ((e = hipMemcpy(P->d_taps, P->taps.data(), P->taps.size() * sizeof(Tap), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy stencil taps");
    if ((e = hipMemcpy(P->d_rows, P->rows.data(), P->rows.size() * sizeof(StencilRow), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy stencil rows");
    if ((e = hipMemcpy(P->d_row_w, P->row_w.data(), P->row_w.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy stencil weights");
    std::vector<float> wf(P->row_w.begin(), P->row_w.end());
    if ((e = hipMemcpy(P->d_row_wf, wf.data(), wf.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy stencil weights (fp32)");
  }
  if (!tiles.empty()) {
    if ((e = hipMemcpy(P->d_tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy stencil tiles");
    if ((e = hipMemcpy(P->d_row_w_tile, row_w_tile.data(), row_w_tile.size() * sizeof(double),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy stencil tile weights");
    std::vector<float> wtf(row_w_tile.begin(), row_w_tile.end());
    if ((e = hipMemcpy(P->d_row_wf_tile, wtf.data(), wtf.size() * sizeof(float), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return hip_fail(e, "copy stencil tile weights (fp32)");
  }
  if ((e = hipMemcpy(P->d_wave_rows, wave_rows.data(), wave_rows.size() * sizeof(int), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return hip_fail(e, "copy stencil wave split");
  if (P->stencil_mfma) {
    if ((e = hipMemcpy(P->d_mfma_a, mfma_a.data(), mfma_a.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy MFMA stencil operands");
    if ((e = hipMemcpy(P->d_rows_mfma, rows_mfma.data(), rows_mfma.size() * sizeof(StencilRow),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "copy MFMA stencil columns");
  }
  if ((e = hipMemcpy(P->d_Kl, P->Kl.data(), P->Kl.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "copy coarsest kernel");
  if (P->ant_tiles &&
      (e = hipMemcpy(P->d_ant_tab, ant_tab.data(), ant_tab.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "copy anterpolation tables");
  if ((e = hipMemset(P->d_flags, 0, 4 * sizeof(int))) != hipSuccess) return hip_fail(e, "clear flags");
  // the binning's cell counts: zero here, and zero again after every scan
  if ((e = hipMemset(P->d_count, 0, (size_t)cg.ncell * sizeof(int))) != hipSuccess)
    return hip_fail(e, "clear cell counts");
  if ((e = hipMemset(P->d_scratch, 0, 64 * sizeof(double))) != hipSuccess) return hip_fail(e, "clear scratch");
  return MLS_OK;
}

void free_plan(mls_plan_s* P) {
  for (void* p : P->allocations) (void)hipFree(p);
  P->allocations.clear();
}

}  // namespace mls
