// extern "C" entry points of the MLS dispersion library (include/mlsdisp.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>

#include "mls_internal.h"

namespace mls {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

mls_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return MLS_ERR_HIP;
}

}  // namespace mls

using namespace mls;

static constexpr int kTimingSlots = 256;

#define HIP_TRY(call, what)                    \
  do {                                         \
    hipError_t _e = (call);                    \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

extern "C" {

const char* mls_status_string(int status) {
  switch (status) {
    case MLS_OK: return "success";
    case MLS_ERR_INVALID_ARG: return "invalid argument";
    case MLS_ERR_UNSUPPORTED: return "unsupported request";
    case MLS_ERR_HIP: return "HIP runtime error";
    case MLS_ERR_OOM: return "device out of memory";
    case MLS_ERR_NONFINITE: return "non-finite or negative input data";
    default: return "unknown status";
  }
}

const char* mls_last_error(void) { return g_last_error.c_str(); }

mls_status mls_plan_create(const mls_params* params, int64_t n_max, mls_plan_t* out) {
  g_last_error.clear();
  if (!params || !out) { set_error("mls_plan_create: null params or out"); return MLS_ERR_INVALID_ARG; }
  *out = nullptr;
  mls_plan_s* P = new (std::nothrow) mls_plan_s();
  if (!P) { set_error("host allocation failed"); return MLS_ERR_OOM; }
  mls_status st = build_plan(*params, n_max, P);
  if (st != MLS_OK) {
    free_plan(P);
    delete P;
    return st;
  }
  *out = P;
  return MLS_OK;
}

mls_status mls_plan_get_info(mls_plan_t P, mls_plan_info* info) {
  if (!P || !info) { set_error("mls_plan_get_info: null argument"); return MLS_ERR_INVALID_ARG; }
  std::memset(info, 0, sizeof(*info));
  info->levels = P->levels;
  for (int d = 0; d < 3; ++d) {
    info->grid[d] = P->lv[0].g.n[d];
    info->coarsest[d] = P->lv[P->levels - 1].g.n[d];
    info->cells[d] = P->cg.nc[d];
    info->h_eff[d] = P->lv[0].h[d];
    info->cell_width[d] = P->cg.w[d];
  }
  info->taps = (int64_t)P->taps.size();
  info->n_max = P->n_max;
  info->workspace_bytes = P->bytes;
  info->precision = P->precision;
  info->order = P->order;
  info->continuity = P->continuity;
  info->mixing = P->mixing;
  info->stencil_path = stencil_path(P);
  return MLS_OK;
}

}  // extern "C"

namespace {

// The repulsive term of the MD entry points: sqrt(C12) per atom and its cutoff.
struct Repulsion {
  const double* c12;
  double rc;
};

// mls_evaluate, optionally with the repulsion (rep non-null) run after the
// local part on the caller's stream and added in the interpolation.
// binning of an evaluation: a fresh one, one that records the positions
// (first step of an MD run with neighbour reuse), or the reuse check
enum { kBinFresh = 0, kBinRecord = 1, kBinReuse = 2 };

mls_status evaluate_geometric(mls_plan_t P, int64_t n, const double* pos, const double* c6, double* energy,
                              double* forces, double* potential, double* dE_dc6, void* stream,
                              const Repulsion* rep, int binmode = kBinFresh) {
  if (!P) { set_error("mls_evaluate: null plan"); return MLS_ERR_INVALID_ARG; }
  if (n < 0 || n > P->n_max) {
    set_error("mls_evaluate: n = " + std::to_string(n) + " outside [0, n_max = " + std::to_string(P->n_max) + "]");
    return MLS_ERR_INVALID_ARG;
  }
  if (!energy) { set_error("mls_evaluate: energy pointer is required"); return MLS_ERR_INVALID_ARG; }
  if (n > 0 && (!pos || !c6)) { set_error("mls_evaluate: null pos or c6"); return MLS_ERR_INVALID_ARG; }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != P->device) {
    set_error("mls_evaluate: current device differs from the plan's device");
    return MLS_ERR_INVALID_ARG;
  }
  if (P->mixing != MLS_GEOMETRIC) {
    set_error("mls_evaluate: the plan uses Lorentz-Berthelot mixing (call mls_evaluate_lb)");
    return MLS_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  P->last_stream = s;
  P->last_n = n;
  const int ni = (int)n;
  hipEvent_t* ev = nullptr;
  if (P->timing && P->timing_slots < kTimingSlots) {
    ev = &P->events[(size_t)P->timing_slots * (MLS_NUM_STAGES + 1)];
    ++P->timing_slots;
  }
  auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord(ev[k], s) : hipSuccess; };
  // with per-stage timing every stage runs in order on the caller's stream;
  // otherwise the grid chain runs on the plan's second stream, concurrently
  // with the local part
  const bool fork = !ev && !P->serial;
  if (fork && !P->side) {
    HIP_TRY(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    HIP_TRY(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming), "hipEventCreateWithFlags");
    HIP_TRY(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming), "hipEventCreateWithFlags");
  }
  const hipStream_t g = fork ? P->side : s;
  HIP_TRY(mark(0), "timing event");
  if (binmode == kBinRecord) {
    HIP_TRY(launch_binning_ref(P, ni, pos, c6, s), "binning");
  } else if (binmode == kBinReuse) {
    HIP_TRY(launch_binning_reuse(P, ni, pos, c6, s), "binning");
  } else {
    HIP_TRY(launch_binning(P, ni, pos, c6, s), "binning");
  }
  HIP_TRY(mark(1 + MLS_T_BINNING), "timing event");
  if (fork) {
    HIP_TRY(hipEventRecord(P->ev_fork, s), "fork");
    HIP_TRY(hipStreamWaitEvent(g, P->ev_fork, 0), "fork");
  }
  // In concurrent mode the local part is submitted after the grid chain's
  // first `pair_after` stages (default 1: the anterpolation, whose blocks need
  // 35 KB of LDS each and are otherwise held back until the pair kernel has
  // filled and drained every CU; measured with graph replays at 10^6 atoms:
  // 0.835 ms per evaluation against 0.877 ms with the pair kernel first).
  const int after = fork ? P->pair_after : 0;
  // the repulsion rides on the pair kernel where that kernel supports it,
  // else runs as its own kernel right after it
  const PairRep prep{P->d_x12s, P->d_x12f, rep ? rep->rc * rep->rc : 0.0, P->d_frep, P->d_md_partial};
  auto pair = [&]() -> mls_status {
    if (rep) HIP_TRY(launch_rep_gather(P, ni, rep->c12, s), "repulsion");
    bool fused = false;
    HIP_TRY(launch_pair(P, ni, s, rep ? &prep : nullptr, &fused), "pair kernel");
    if (rep && !fused) HIP_TRY(launch_repulsion(P, ni, rep->rc, s), "repulsion");
    HIP_TRY(mark(1 + MLS_T_PAIR), "timing event");
    return MLS_OK;
  };
  mls_status st;
  if (after == 0 && (st = pair()) != MLS_OK) return st;
  // the sum of xi is needed first by the stencils: launched after the
  // anterpolation, whose tiles then start as soon as the binning ends
  HIP_TRY(launch_anterpolate(P, ni, g), "anterpolation");
  HIP_TRY(launch_sum_xi(P, ni, g), "sum of xi");
  HIP_TRY(mark(1 + MLS_T_ANTERP), "timing event");
  if (after == 1 && (st = pair()) != MLS_OK) return st;
  HIP_TRY(launch_restrictions(P, g), "restriction");
  HIP_TRY(mark(1 + MLS_T_RESTRICT), "timing event");
  if (after == 2 && (st = pair()) != MLS_OK) return st;
  HIP_TRY(launch_stencils(P, g), "level stencils");
  HIP_TRY(mark(1 + MLS_T_STENCIL), "timing event");
  if (after == 3 && (st = pair()) != MLS_OK) return st;
  HIP_TRY(launch_coarsest(P, g), "coarsest grid");
  HIP_TRY(mark(1 + MLS_T_COARSEST), "timing event");
  if (after == 4 && (st = pair()) != MLS_OK) return st;
  HIP_TRY(launch_prolongations(P, g), "prolongation");
  HIP_TRY(mark(1 + MLS_T_PROLONG), "timing event");
  if (fork) HIP_TRY(hipEventRecord(P->ev_join, g), "join");
  if (after == 5 && (st = pair()) != MLS_OK) return st;
  if (fork) HIP_TRY(hipStreamWaitEvent(s, P->ev_join, 0), "join");
  HIP_TRY(launch_interpolate(P, ni, energy, forces, potential, dE_dc6, s, rep ? kInterpRep : 0), "interpolation");
  HIP_TRY(mark(1 + MLS_T_INTERP), "timing event");
  return MLS_OK;
}

// Multiple time stepping: the fast force alone (local part of eq:evaluation
// with k = 0 plus the repulsion), all on stream s.
hipError_t evaluate_fast(mls_plan_t P, int n, const double* pos, const double* c6, const Repulsion& rep,
                         double* energy, double* forces, hipStream_t s) {
  hipError_t e = launch_binning(P, n, pos, c6, s);
  if (e == hipSuccess) e = launch_rep_gather(P, n, rep.c12, s);
  const PairRep prep{P->d_x12s, P->d_x12f, rep.rc * rep.rc, P->d_frep, P->d_md_partial};
  bool fused = false;
  if (e == hipSuccess) e = launch_pair(P, n, s, &prep, &fused);
  if (e == hipSuccess && !fused) e = launch_repulsion(P, n, rep.rc, s);
  if (e == hipSuccess) e = launch_local_out(P, n, energy, forces, s);
  return e;
}

// Both forces at the same positions from one binning: the grid chain on the
// plan's second stream, concurrently with the local part (as in
// mls_evaluate), then the fast outputs and the grid-only interpolation.
// *energy = E_fast + E_slow.
hipError_t evaluate_split(mls_plan_t P, int n, const double* pos, const double* c6, const Repulsion& rep,
                          double* energy, double* forces, double* fslow, hipStream_t s) {
  hipError_t e;
  if (!P->side) {
    if ((e = hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming)) != hipSuccess) return e;
  }
  const hipStream_t g = P->side;
  if ((e = launch_binning(P, n, pos, c6, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(P->ev_fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(g, P->ev_fork, 0)) != hipSuccess) return e;
  if ((e = launch_sum_xi(P, n, g)) != hipSuccess) return e;
  if ((e = launch_anterpolate(P, n, g)) != hipSuccess) return e;
  if ((e = launch_rep_gather(P, n, rep.c12, s)) != hipSuccess) return e;
  const PairRep prep{P->d_x12s, P->d_x12f, rep.rc * rep.rc, P->d_frep, P->d_md_partial};
  bool fused = false;
  if ((e = launch_pair(P, n, s, &prep, &fused)) != hipSuccess) return e;
  if (!fused && (e = launch_repulsion(P, n, rep.rc, s)) != hipSuccess) return e;
  if ((e = launch_restrictions(P, g)) != hipSuccess) return e;
  if ((e = launch_stencils(P, g)) != hipSuccess) return e;
  if ((e = launch_coarsest(P, g)) != hipSuccess) return e;
  if ((e = launch_prolongations(P, g)) != hipSuccess) return e;
  if ((e = hipEventRecord(P->ev_join, g)) != hipSuccess) return e;
  if ((e = launch_local_out(P, n, energy, forces, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(s, P->ev_join, 0)) != hipSuccess) return e;
  return launch_interpolate(P, n, energy, fslow, nullptr, nullptr, s, kInterpGridOnly);
}

hipError_t ensure_side(mls_plan_s* P) {
  hipError_t e = hipSuccess;
  if (!P->side) {
    if ((e = hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming)) != hipSuccess) return e;
    e = hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming);
  }
  return e;
}

// Multiple time stepping per level, fast and mid forces at the same
// positions from one binning: the local part (and repulsion) on stream s, the
// level-1 grid part (anterpolation and the level-1 stencil; none with one
// level) on the second stream; *energy = E_fast + E_mid, fmid = the
// interpolated e^1 forces.
hipError_t evaluate_fast_mid(mls_plan_s* P, int n, const double* pos, const double* c6, const Repulsion& rep,
                             double* energy, double* forces, double* fmid, hipStream_t s) {
  hipError_t e;
  if (P->levels < 2) {
    if ((e = evaluate_fast(P, n, pos, c6, rep, energy, forces, s)) != hipSuccess) return e;
    return launch_zero(fmid, 3 * (int64_t)n, s);
  }
  if ((e = ensure_side(P)) != hipSuccess) return e;
  const hipStream_t g = P->side;
  if ((e = launch_binning(P, n, pos, c6, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(P->ev_fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(g, P->ev_fork, 0)) != hipSuccess) return e;
  if ((e = launch_sum_xi(P, n, g)) != hipSuccess) return e;
  if ((e = launch_anterpolate(P, n, g)) != hipSuccess) return e;
  if ((e = launch_rep_gather(P, n, rep.c12, s)) != hipSuccess) return e;
  const PairRep prep{P->d_x12s, P->d_x12f, rep.rc * rep.rc, P->d_frep, P->d_md_partial};
  bool fused = false;
  if ((e = launch_pair(P, n, s, &prep, &fused)) != hipSuccess) return e;
  if (!fused && (e = launch_repulsion(P, n, rep.rc, s)) != hipSuccess) return e;
  if ((e = launch_stencils(P, g, 1)) != hipSuccess) return e;
  if ((e = hipEventRecord(P->ev_join, g)) != hipSuccess) return e;
  if ((e = launch_local_out(P, n, energy, forces, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(s, P->ev_join, 0)) != hipSuccess) return e;
  return launch_interpolate(P, n, energy, fmid, nullptr, nullptr, s, kInterpGridOnly | kInterpLevel1 | kInterpNoSelf);
}

// All three classes at the same positions: fast as above; mid = the
// interpolated e^1 (l >= 2, else zero); slow = the interpolated prolongation
// of E^2 without e^1 (l = 1: the coarsest level, which is level 1) with the
// self-energy term.  *energy = E_fast + E_mid + E_slow.
hipError_t evaluate_split3(mls_plan_s* P, int n, const double* pos, const double* c6, const Repulsion& rep,
                           double* energy, double* forces, double* fmid, double* fslow, hipStream_t s) {
  hipError_t e;
  if ((e = ensure_side(P)) != hipSuccess) return e;
  const hipStream_t g = P->side;
  const bool two = P->levels >= 2;
  if ((e = launch_binning(P, n, pos, c6, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(P->ev_fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(g, P->ev_fork, 0)) != hipSuccess) return e;
  if ((e = launch_sum_xi(P, n, g)) != hipSuccess) return e;
  if ((e = launch_anterpolate(P, n, g)) != hipSuccess) return e;
  if ((e = launch_rep_gather(P, n, rep.c12, s)) != hipSuccess) return e;
  const PairRep prep{P->d_x12s, P->d_x12f, rep.rc * rep.rc, P->d_frep, P->d_md_partial};
  bool fused = false;
  if ((e = launch_pair(P, n, s, &prep, &fused)) != hipSuccess) return e;
  if (!fused && (e = launch_repulsion(P, n, rep.rc, s)) != hipSuccess) return e;
  if ((e = launch_restrictions(P, g)) != hipSuccess) return e;
  if ((e = launch_stencils(P, g)) != hipSuccess) return e;
  if ((e = launch_coarsest(P, g)) != hipSuccess) return e;
  if ((e = launch_prolongations(P, g, two)) != hipSuccess) return e;
  if ((e = hipEventRecord(P->ev_join, g)) != hipSuccess) return e;
  if ((e = launch_local_out(P, n, energy, forces, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(s, P->ev_join, 0)) != hipSuccess) return e;
  if (two) {
    e = launch_interpolate(P, n, energy, fmid, nullptr, nullptr, s, kInterpGridOnly | kInterpLevel1 | kInterpNoSelf);
  } else {
    e = launch_zero(fmid, 3 * (int64_t)n, s);
  }
  if (e != hipSuccess) return e;
  return launch_interpolate(P, n, energy, fslow, nullptr, nullptr, s, kInterpGridOnly);
}

}  // namespace

namespace mls {
mls_status evaluate_plan(mls_plan_s* P, int64_t n, const double* pos, const double* c6, double* energy,
                         double* forces, double* potential, double* dE_dc6, void* stream) {
  return evaluate_geometric(P, n, pos, c6, energy, forces, potential, dE_dc6, stream, nullptr);
}
}  // namespace mls

extern "C" {

mls_status mls_evaluate(mls_plan_t P, int64_t n, const double* pos, const double* c6, double* energy,
                        double* forces, double* potential, double* dE_dc6, void* stream) {
  return evaluate_geometric(P, n, pos, c6, energy, forces, potential, dE_dc6, stream, nullptr);
}

static mls_status check_rep(mls_plan_t P, int64_t n, const double* c12, double rc, const char* who) {
  if (!P) { set_error(std::string(who) + ": null plan"); return MLS_ERR_INVALID_ARG; }
  if (n > 0 && !c12) { set_error(std::string(who) + ": null c12"); return MLS_ERR_INVALID_ARG; }
  if (!(rc > 0.0 && rc <= P->a)) {
    set_error(std::string(who) + ": repulsion cutoff must satisfy 0 < rc <= a");
    return MLS_ERR_INVALID_ARG;
  }
  return MLS_OK;
}

mls_status mls_evaluate_md(mls_plan_t P, int64_t n, const double* pos, const double* c6, const double* c12,
                           double rc, double* energy, double* forces, void* stream) {
  mls_status st = check_rep(P, n, c12, rc, "mls_evaluate_md");
  if (st != MLS_OK) return st;
  const Repulsion rep{c12, rc};
  return evaluate_geometric(P, n, pos, c6, energy, forces, nullptr, nullptr, stream, &rep);
}

mls_status mls_md_run(mls_plan_t P, int64_t n, double* pos, double* vel, const double* c6, const double* c12,
                      double rc, const double* inv_mass, double dt, int nsteps, double* forces, double* epot,
                      double* ekin, void* stream) {
  mls_status st = check_rep(P, n, c12, rc, "mls_md_run");
  if (st != MLS_OK) return st;
  if (nsteps < 0 || !(std::isfinite(dt))) { set_error("mls_md_run: nsteps < 0 or non-finite dt"); return MLS_ERR_INVALID_ARG; }
  if (!epot || !ekin || (n > 0 && (!pos || !vel || !inv_mass || !forces))) {
    set_error("mls_md_run: null pos, vel, inv_mass, forces, epot or ekin");
    return MLS_ERR_INVALID_ARG;
  }
  const Repulsion rep{c12, rc};
  const hipStream_t s = (hipStream_t)stream;
  const int ni = (int)std::min<int64_t>(std::max<int64_t>(n, 0), P->n_max);
  // with a skin the binning of the first evaluation is kept while no atom
  // has moved more than skin/2 since (checked on the device every step)
  const bool reuse = P->skin > 0.0;
  if ((st = evaluate_geometric(P, n, pos, c6, epot, forces, nullptr, nullptr, stream, &rep,
                               reuse ? kBinRecord : kBinFresh)) != MLS_OK)
    return st;
  for (int k = 1; k <= nsteps; ++k) {
    // end of step k-1 (k > 1): second half-kick, E_kin(k-1); step k: first
    // half-kick and drift
    const int mode = (k > 1 ? kMdEnd : 0) | kMdStart;
    HIP_TRY(launch_md_step(P, ni, pos, vel, forces, inv_mass, dt, mode, ekin + (k - 1), s), "integrator");
    if ((st = evaluate_geometric(P, n, pos, c6, epot + k, forces, nullptr, nullptr, stream, &rep,
                                 reuse ? kBinReuse : kBinFresh)) != MLS_OK)
      return st;
  }
  HIP_TRY(launch_md_step(P, ni, pos, vel, forces, inv_mass, dt, nsteps > 0 ? kMdEnd : 0, ekin + nsteps, s),
          "integrator");
  return MLS_OK;
}

mls_status mls_md_run_mts(mls_plan_t P, int64_t n, double* pos, double* vel, const double* c6, const double* c12,
                          double rc, const double* inv_mass, double dt, int nsteps, int k_slow, double* forces,
                          double* epot, double* ekin, void* stream) {
  mls_status st = check_rep(P, n, c12, rc, "mls_md_run_mts");
  if (st != MLS_OK) return st;
  if (k_slow < 1 || nsteps < 0 || nsteps % k_slow != 0 || !(std::isfinite(dt))) {
    set_error("mls_md_run_mts: need k_slow >= 1, nsteps >= 0 a multiple of k_slow, finite dt");
    return MLS_ERR_INVALID_ARG;
  }
  if (!epot || !ekin || (n > 0 && (!pos || !vel || !inv_mass || !forces || !c6))) {
    set_error("mls_md_run_mts: null pos, vel, c6, inv_mass, forces, epot or ekin");
    return MLS_ERR_INVALID_ARG;
  }
  if (n > P->n_max) {
    set_error("mls_md_run_mts: n = " + std::to_string(n) + " above n_max = " + std::to_string(P->n_max));
    return MLS_ERR_INVALID_ARG;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != P->device) {
    set_error("mls_md_run_mts: current device differs from the plan's device");
    return MLS_ERR_INVALID_ARG;
  }
  if (P->mixing != MLS_GEOMETRIC) {
    set_error("mls_md_run_mts: the plan uses Lorentz-Berthelot mixing");
    return MLS_ERR_INVALID_ARG;
  }
  const hipStream_t s = (hipStream_t)stream;
  P->last_stream = s;
  P->last_n = n;
  const int ni = (int)std::max<int64_t>(n, 0);
  const Repulsion rep{c12, rc};
  const double hslow = 0.5 * k_slow * dt;
  double* fs = P->d_fslow;
  // outer step o: slow half-kick, k_slow inner velocity-Verlet steps with the
  // fast force, slow force at the new positions, slow half-kick
  HIP_TRY(evaluate_split(P, ni, pos, c6, rep, epot, forces, fs, s), "forces");
  const int nout = nsteps / k_slow;
  for (int o = 1; o <= nout; ++o) {
    for (int i = 1; i <= k_slow; ++i) {
      int mode = kMdStart;
      double* kin = nullptr;
      if (i == 1) {
        // end of outer step o-1 (o > 1): its last fast and slow half-kicks and
        // E_kin; then the slow half-kick of outer step o
        mode |= kMdSlowStart;
        if (o > 1) mode |= kMdEnd | kMdSlowEnd;
        kin = ekin + (o - 1);
      } else {
        mode |= kMdEnd;
      }
      HIP_TRY(launch_md_step(P, ni, pos, vel, forces, inv_mass, dt, mode, kin, s, fs, hslow), "integrator");
      if (i < k_slow) {
        HIP_TRY(evaluate_fast(P, ni, pos, c6, rep, P->d_efast, forces, s), "fast force");
      } else {
        HIP_TRY(evaluate_split(P, ni, pos, c6, rep, epot + o, forces, fs, s), "forces");
      }
    }
  }
  HIP_TRY(launch_md_step(P, ni, pos, vel, forces, inv_mass, dt, nout > 0 ? (kMdEnd | kMdSlowEnd) : 0, ekin + nout, s,
                         fs, hslow),
          "integrator");
  // the total force at the final positions
  if (ni > 0) HIP_TRY(launch_add_forces(forces, fs, ni, s), "forces");
  return MLS_OK;
}

mls_status mls_md_run_mts_levels(mls_plan_t P, int64_t n, double* pos, double* vel, const double* c6,
                                 const double* c12, double rc, const double* inv_mass, double dt, int nsteps, int k_mid,
                                 int k_slow, double* forces, double* epot, double* ekin, void* stream) {
  mls_status st = check_rep(P, n, c12, rc, "mls_md_run_mts_levels");
  if (st != MLS_OK) return st;
  if (k_mid < 1 || k_slow < 1 || nsteps < 0 || (int64_t)k_mid * k_slow > (1 << 20) ||
      nsteps % (k_mid * k_slow) != 0 || !(std::isfinite(dt))) {
    set_error("mls_md_run_mts_levels: need k_mid, k_slow >= 1, nsteps >= 0 a multiple of k_mid k_slow, finite dt");
    return MLS_ERR_INVALID_ARG;
  }
  if (!epot || !ekin || (n > 0 && (!pos || !vel || !inv_mass || !forces || !c6))) {
    set_error("mls_md_run_mts_levels: null pos, vel, c6, inv_mass, forces, epot or ekin");
    return MLS_ERR_INVALID_ARG;
  }
  if (n > P->n_max) {
    set_error("mls_md_run_mts_levels: n = " + std::to_string(n) + " above n_max = " + std::to_string(P->n_max));
    return MLS_ERR_INVALID_ARG;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != P->device) {
    set_error("mls_md_run_mts_levels: current device differs from the plan's device");
    return MLS_ERR_INVALID_ARG;
  }
  if (P->mixing != MLS_GEOMETRIC) {
    set_error("mls_md_run_mts_levels: the plan uses Lorentz-Berthelot mixing");
    return MLS_ERR_INVALID_ARG;
  }
  const hipStream_t s = (hipStream_t)stream;
  P->last_stream = s;
  P->last_n = n;
  const int ni = (int)std::max<int64_t>(n, 0);
  const Repulsion rep{c12, rc};
  const double hslow = 0.5 * k_mid * k_slow * dt, hmid = 0.5 * k_mid * dt;
  double* fs = P->d_fslow;
  double* fm = P->d_fmid;
  HIP_TRY(evaluate_split3(P, ni, pos, c6, rep, epot, forces, fm, fs, s), "forces");
  const int nout = nsteps / (k_mid * k_slow);
  for (int o = 1; o <= nout; ++o) {
    for (int m = 1; m <= k_slow; ++m) {
      for (int i = 1; i <= k_mid; ++i) {
        int mode = kMdStart;
        double* kin = nullptr;
        if (i == 1) {
          // a middle step begins: the end of the previous one (and at an
          // outer boundary the previous outer step's end, E_kin, and the
          // slow half-kick of outer step o), then its mid half-kick
          mode |= kMdMidStart;
          if (m == 1) {
            mode |= kMdSlowStart;
            if (o > 1) mode |= kMdEnd | kMdMidEnd | kMdSlowEnd;
            kin = ekin + (o - 1);
          } else {
            mode |= kMdEnd | kMdMidEnd;
          }
        } else {
          mode |= kMdEnd;
        }
        HIP_TRY(launch_md_step(P, ni, pos, vel, forces, inv_mass, dt, mode, kin, s, fs, hslow, fm, hmid),
                "integrator");
        hipError_t e;
        if (i < k_mid) {
          e = evaluate_fast(P, ni, pos, c6, rep, P->d_efast, forces, s);
        } else if (m < k_slow) {
          e = evaluate_fast_mid(P, ni, pos, c6, rep, P->d_efast, forces, fm, s);
        } else {
          e = evaluate_split3(P, ni, pos, c6, rep, epot + o, forces, fm, fs, s);
        }
        if (e != hipSuccess) return hip_fail(e, "forces");
      }
    }
  }
  HIP_TRY(launch_md_step(P, ni, pos, vel, forces, inv_mass, dt, nout > 0 ? (kMdEnd | kMdMidEnd | kMdSlowEnd) : 0,
                         ekin + nout, s, fs, hslow, fm, hmid),
          "integrator");
  // the total force at the final positions
  if (ni > 0) {
    HIP_TRY(launch_add_forces(forces, fm, ni, s), "forces");
    HIP_TRY(launch_add_forces(forces, fs, ni, s), "forces");
  }
  return MLS_OK;
}

mls_status mls_evaluate_lb(mls_plan_t P, int64_t n, const double* pos, const double* eps, const double* sigma,
                           double* energy, double* forces, void* stream) {
  if (!P) { set_error("mls_evaluate_lb: null plan"); return MLS_ERR_INVALID_ARG; }
  if (P->mixing != MLS_LORENTZ_BERTHELOT) {
    set_error("mls_evaluate_lb: the plan was not created with Lorentz-Berthelot mixing");
    return MLS_ERR_INVALID_ARG;
  }
  if (n < 0 || n > P->n_max) {
    set_error("mls_evaluate_lb: n = " + std::to_string(n) + " outside [0, n_max = " + std::to_string(P->n_max) + "]");
    return MLS_ERR_INVALID_ARG;
  }
  if (!energy) { set_error("mls_evaluate_lb: energy pointer is required"); return MLS_ERR_INVALID_ARG; }
  if (n > 0 && (!pos || !eps || !sigma)) { set_error("mls_evaluate_lb: null pos, eps or sigma"); return MLS_ERR_INVALID_ARG; }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != P->device) {
    set_error("mls_evaluate_lb: current device differs from the plan's device");
    return MLS_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  P->last_stream = s;
  P->last_n = n;
  const int ni = (int)n;
  if (!P->side) {
    HIP_TRY(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    HIP_TRY(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming), "hipEventCreateWithFlags");
    HIP_TRY(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming), "hipEventCreateWithFlags");
  }
  const hipStream_t g = P->side;
  // binning with xi = sqrt(2 eps) (the e_i of the pair coefficient) and the
  // sorted sigma
  HIP_TRY(launch_binning_scaled(P, ni, pos, eps, 2.0, s), "binning");
  HIP_TRY(launch_lb_gather(P, ni, sigma, s), "sigma gather");
  // the seven grid chains run on the plan's second stream, concurrently with
  // the local part, and meet it at interpolation
  HIP_TRY(hipEventRecord(P->ev_fork, s), "fork");
  HIP_TRY(hipStreamWaitEvent(g, P->ev_fork, 0), "fork");
  HIP_TRY(launch_pair_lb(P, ni, s), "pair kernel");
  // grid part once per charge vector (their grids in turn become the plan's
  // working levels; the vectors share one charge buffer, in stream order)
  for (int k = 0; k < 7; ++k) {
    HIP_TRY(launch_lb_charge(P, ni, k, g), "charges");
    std::swap(P->lv, P->lb_lv[k]);
    P->charge = lb_charge_buf(P, k);
    P->ant_scratch = lb_ant_scratch(P, k);
    if (P->precision == MLS_MIXED) P->sum_q = lb_sum_buf(P, k);
    hipError_t e = launch_anterpolate(P, ni, g);
    if (e == hipSuccess) e = launch_restrictions(P, g);
    if (e == hipSuccess) e = launch_stencils(P, g);
    if (e == hipSuccess) e = launch_coarsest(P, g);
    if (e == hipSuccess) e = launch_prolongations(P, g);
    P->charge = nullptr;
    P->ant_scratch = nullptr;
    P->sum_q = nullptr;
    std::swap(P->lv, P->lb_lv[k]);
    if (e != hipSuccess) return hip_fail(e, "grid part");
  }
  HIP_TRY(hipEventRecord(P->ev_join, g), "join");
  HIP_TRY(hipStreamWaitEvent(s, P->ev_join, 0), "join");
  HIP_TRY(launch_interpolate_lb(P, ni, energy, forces, s), "interpolation");
  return MLS_OK;
}

mls_status mls_plan_set_timing(mls_plan_t P, int enable) {
  if (!P) { set_error("mls_plan_set_timing: null plan"); return MLS_ERR_INVALID_ARG; }
  if (enable && P->events.empty()) {
    P->events.resize((size_t)kTimingSlots * (MLS_NUM_STAGES + 1));
    for (auto& e : P->events) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
  }
  P->timing = enable != 0;
  P->timing_slots = 0;
  return MLS_OK;
}

mls_status mls_plan_read_timing(mls_plan_t P, double* ms, int* count) {
  if (!P || !ms || !count) { set_error("mls_plan_read_timing: null argument"); return MLS_ERR_INVALID_ARG; }
  for (int k = 0; k < MLS_NUM_STAGES; ++k) ms[k] = 0.0;
  *count = P->timing_slots;
  for (int sl = 0; sl < P->timing_slots; ++sl) {
    hipEvent_t* ev = &P->events[(size_t)sl * (MLS_NUM_STAGES + 1)];
    HIP_TRY(hipEventSynchronize(ev[MLS_NUM_STAGES]), "hipEventSynchronize");
    for (int k = 0; k < MLS_NUM_STAGES; ++k) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, ev[k], ev[k + 1]), "hipEventElapsedTime");
      ms[k] += t;
    }
  }
  P->timing_slots = 0;
  return MLS_OK;
}

mls_status mls_plan_copy_stage(mls_plan_t P, int what, int level, void* dst, int64_t capacity, void* stream) {
  if (!P || !dst) { set_error("mls_plan_copy_stage: null argument"); return MLS_ERR_INVALID_ARG; }
  int64_t need = 0;
  const int64_t n = P->last_n < 0 ? 0 : P->last_n;
  switch (what) {
    case MLS_STAGE_PERM: need = 4 * n; break;
    case MLS_STAGE_CELL_START: need = 4 * ((int64_t)P->cg.ncell + 1); break;
    case MLS_STAGE_E0: need = 8 * n; break;
    case MLS_STAGE_FLOC: need = 24 * n; break;
    case MLS_STAGE_Q:
    case MLS_STAGE_E_LEVEL:
    case MLS_STAGE_E_TOTAL:
      if (level < 1 || level > P->levels) { set_error("mls_plan_copy_stage: level out of range"); return MLS_ERR_INVALID_ARG; }
      need = 8 * (int64_t)P->lv[level - 1].g.size;
      break;
    default: set_error("mls_plan_copy_stage: unknown stage"); return MLS_ERR_INVALID_ARG;
  }
  if (capacity < need) { set_error("mls_plan_copy_stage: destination too small"); return MLS_ERR_INVALID_ARG; }
  HIP_TRY(launch_copy_stage(P, what, level, dst, (hipStream_t)stream), "copy stage");
  return MLS_OK;
}

mls_status mls_plan_status(mls_plan_t P, int* flags) {
  if (!P || !flags) { set_error("mls_plan_status: null argument"); return MLS_ERR_INVALID_ARG; }
  HIP_TRY(hipStreamSynchronize(P->last_stream), "synchronise");
  int h[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpy(h, P->d_flags, sizeof(h), hipMemcpyDeviceToHost), "read flags");
  HIP_TRY(hipMemset(P->d_flags, 0, sizeof(h)), "clear flags");
  *flags = h[0];
  if (h[0] & 11) {
    set_error("input data contained non-finite positions, non-finite/negative C6 or C12, "
              "non-finite velocities or non-positive inverse masses");
    return MLS_ERR_NONFINITE;
  }
  if (h[0]) { set_error("internal error: an atom fell outside its anterpolation block"); return MLS_ERR_HIP; }
  return MLS_OK;
}

mls_status mls_plan_destroy(mls_plan_t P) {
  if (!P) return MLS_OK;
  for (auto& e : P->events) (void)hipEventDestroy(e);
  P->events.clear();
  if (P->side) {
    (void)hipStreamSynchronize(P->side);
    (void)hipStreamDestroy(P->side);
    (void)hipEventDestroy(P->ev_fork);
    (void)hipEventDestroy(P->ev_join);
  }
  free_plan(P);
  delete P;
  return MLS_OK;
}

}  // extern "C"
