// Batched evaluation of many independent periodic boxes.
//
// Every box gets its own plan (grids, cells, stencil tables, coarsest kernel,
// workspace), built exactly as for a single evaluation.  An evaluation of the
// batch is one fixed sequence of phases, one launch each, in the order of the
// steps of Sec. II.B (binning, local part, anterpolation, restrictions,
// level stencils, coarsest level, prolongations, interpolation): each launch
// covers every box that has work in that phase through a device array of
// per-box kernel arguments and a (box, block) work list, largest boxes first,
// walked by a persistent grid whose size per stage is chosen by the
// autotuner.  The sequence is captured once into a hipGraph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mls_internal.h"

using namespace mls;

namespace {

constexpr int kCandidateGrids[] = {0, 512, 1024, 2048, 4096};
constexpr int kTuneReps = 3;

inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

struct mls_batch_s {
  int nbox = 0;
  int device = 0;
  int precision = 0;
  int order = 4;
  int mixing = 0;                    // mls_mixing, shared by every box
  std::vector<mls_plan_s*> plans;
  std::vector<int64_t> off;          // nbox + 1 atom offsets

  // phases of one evaluation, in launch order, and their device arena
  std::vector<BatchPhase> phases;
  void* arena = nullptr;
  bool built = false;

  // caller buffers the phases were built for
  const double* pos = nullptr;
  const double* c6 = nullptr;        // C6, or epsilon under Lorentz-Berthelot mixing
  const double* sigma = nullptr;     // Lorentz-Berthelot: sigma
  double* energies = nullptr;
  double* forces = nullptr;
  double* dE_dc6 = nullptr;

  mls_batch_tuning tune{};
  bool tune_pending = false;

  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  hipStream_t side = nullptr;        // grid chain, concurrent with the local part
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last_stream = nullptr;
  std::vector<hipEvent_t> events;    // MLS_NUM_STAGES + 1, for the autotuner
};

namespace {

#define HIP_TRY(call, what)                            \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return hip_fail(_e, what);   \
  } while (0)

void drop_graph(mls_batch_s* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
}

void drop_phases(mls_batch_s* B) {
  drop_graph(B);
  if (B->arena) (void)hipFree(B->arena);
  B->arena = nullptr;
  B->phases.clear();
  B->built = false;
}

// Host image of one phase before upload.
struct HostPhase {
  BatchPhase ph;
  std::vector<char> args;            // nbox * sizeof(Args)
  std::vector<int2> work;
  std::vector<int4> tiles;           // BK_STENCIL
};

template <class A>
HostPhase make_phase(int kernel, int stage, int variant, int nbox) {
  HostPhase h;
  h.ph.kernel = kernel;
  h.ph.stage = stage;
  h.ph.variant = variant;
  h.args.assign(sizeof(A) * (size_t)std::max(nbox, 1), 0);
  return h;
}

template <class A>
void set_box(HostPhase& h, int b, const A& a, int blocks) {
  std::memcpy(h.args.data() + sizeof(A) * (size_t)b, &a, sizeof(A));
  for (int k = 0; k < blocks; ++k) h.work.push_back(make_int2(b, k));
}

GridGeom finest(const mls_plan_s* P) {
  GridGeom g;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = P->lv[0].g.n[d];
    g.invh[d] = P->invh1[d];
  }
  return g;
}

int stencil_template(int R) { return R <= 4 ? 4 : (R <= 6 ? 6 : 8); }

// One grid chain (anterpolation .. prolongation) of the batch: per box under
// geometric mixing, per box and charge vector under Lorentz-Berthelot mixing
// (Sec. II.D), each vector with its own slot of buffers.  `id` indexes the
// chain phases' argument arrays.
struct Chain {
  int id;
  mls_plan_s* P;
  std::vector<Level>* lv;
  const double* charge;   // null: the xi of the binning
  double* scratch;        // expanded anterpolation grid
  const double* sum;      // mixed precision: sum of the charges
};

// Build the phase list of one evaluation for the current caller buffers and
// tuning, and upload it (one arena).  Boxes are visited largest first so the
// work lists start with the longest items.
mls_status build_phases(mls_batch_s* B) {
  drop_phases(B);
  const int nb = B->nbox;
  const bool mixed = B->precision == MLS_MIXED;
  std::vector<int> order(nb);
  for (int b = 0; b < nb; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return B->off[x + 1] - B->off[x] > B->off[y + 1] - B->off[y];
  });
  int max_levels = 1;
  for (auto* P : B->plans) max_levels = std::max(max_levels, P->levels);

  std::vector<HostPhase> hp;
  auto n_of = [&](int b) { return (int)(B->off[b + 1] - B->off[b]); };
  const bool lb = B->mixing == MLS_LORENTZ_BERTHELOT;
  std::vector<Chain> chains;
  for (int b : order) {
    mls_plan_s* P = B->plans[b];
    if (!lb) {
      chains.push_back(Chain{b, P, &P->lv, nullptr, P->d_ant_scratch, P->d_scratch});
      continue;
    }
    for (int k = 0; k < 7; ++k)
      chains.push_back(Chain{7 * b + k, P, &P->lb_lv[k], lb_charge_buf(P, k), lb_ant_scratch(P, k), lb_sum_buf(P, k)});
  }
  const int nchain = lb ? 7 * nb : nb;   // entries of the chain phases' argument arrays

  // ------------------------------------------------ binning (Sec. III.D)
  {
    HostPhase fill = make_phase<FillArgs>(BK_FILL_I, MLS_T_BINNING, 0, nb);
    HostPhase cnt = make_phase<BinCountArgs>(BK_BIN_COUNT, MLS_T_BINNING, 0, nb);
    HostPhase s1 = make_phase<ScanArgs>(BK_SCAN_BLOCKS, MLS_T_BINNING, 0, nb);
    HostPhase s2 = make_phase<ScanArgs>(BK_SCAN_SUMS, MLS_T_BINNING, 0, nb);
    HostPhase s3 = make_phase<ScanArgs>(BK_SCAN_ADD, MLS_T_BINNING, 0, nb);
    HostPhase sc = make_phase<ScatterArgs>(BK_SCATTER, MLS_T_BINNING, 0, nb);
    HostPhase rk = make_phase<RankArgs>(BK_RANK, MLS_T_BINNING, 0, nb);
    HostPhase ga = make_phase<GatherArgs>(BK_GATHER, MLS_T_BINNING, 0, nb);
    HostPhase x2 = make_phase<SumXiArgs>(BK_SUM_XI_FINAL, MLS_T_BINNING, 0, nb);
    HostPhase sg = make_phase<LbGatherArgs>(BK_LB_GATHER, MLS_T_BINNING, 0, nb);
    for (int b : order) {
      mls_plan_s* P = B->plans[b];
      const int n = n_of(b);
      const int nc = P->cg.ncell;
      const int64_t o = B->off[b];
      set_box(fill, b, FillArgs{P->d_count, nc}, nblk(nc, 256));
      // xi = sqrt(C6), or e = sqrt(2 eps) under Lorentz-Berthelot mixing
      set_box(cnt, b, BinCountArgs{B->pos + 3 * o, B->c6 + o, n, P->cg, P->d_cid, P->d_slot, P->d_count, P->d_xw,
                                   P->d_flags, lb ? 2.0 : 1.0}, nblk(n, 256));
      ScanArgs sa{P->d_count, nc, P->d_cell_start, P->d_bsum, P->d_bmax, P->d_ncell_max};
      set_box(s1, b, sa, scan_blocks(nc));
      set_box(s2, b, sa, 1);
      set_box(s3, b, sa, nblk(nc, 256));
      set_box(sc, b, ScatterArgs{P->d_cid, P->d_slot, n, P->d_cell_start, P->d_perm_tmp}, nblk(n, 256));
      set_box(rk, b, RankArgs{P->d_cell_start, P->d_perm_tmp, n, P->d_perm}, nblk(n, 256));
      const bool xi_sum = mixed && !lb;
      set_box(ga, b, GatherArgs{P->d_perm, n, P->d_xw, P->d_xs, P->d_cell_s, P->d_xr, P->d_xif, P->cg,
                                xi_sum ? P->d_partial : nullptr, P->d_xf, P->xf_stride},
              nblk(n + kSortedPad, 256));
      if (xi_sum) set_box(x2, b, SumXiArgs{n + kSortedPad, P->d_partial, P->d_scratch}, 1);
      if (lb)
        set_box(sg, b, LbGatherArgs{P->d_perm, n, B->sigma + o, P->d_sig, P->d_flags, P->d_sigf},
                nblk(n + kSortedPad, 256));
    }
    for (HostPhase* h : {&fill, &cnt, &s1, &s2, &s3, &sc, &rk, &ga, &x2, &sg})
      hp.push_back(std::move(*h));
  }

  // ------------------------------------------------ local part (eq:g_0)
  {
    // boxes share the smoothing function; 0x10 selects the LB source weight
    const int pv = pair_variant(B->plans[0]) | (lb ? 0x10 : 0);
    HostPhase f32 = make_phase<PairArgsF>(BK_PAIR_TRIM_F32, MLS_T_PAIR, pv, nb);
    HostPhase f64 = make_phase<PairArgs>(BK_PAIR_TRIM_F64, MLS_T_PAIR, pv, nb);
    HostPhase gen = make_phase<PairArgs>(BK_PAIR_GENERIC, MLS_T_PAIR, pv, nb);
    HostPhase wav = make_phase<PairArgs>(BK_PAIR_WAVE, MLS_T_PAIR, pv, nb);
    for (int b : order) {
      mls_plan_s* P = B->plans[b];
      const int n = n_of(b);
      if (n == 0) continue;
      const CellGeom& g = P->cg;
      PairArgs a{P->d_xs, P->d_cell_s, P->d_cell_start, n, g, pair_const(P), P->d_e0, P->d_floc,
                 lb ? P->d_sig : nullptr};
      a.xf = P->d_xf;
      a.xf_stride = P->xf_stride;
      if (mixed && P->pair_fast && n < (1 << 24)) {
        PairArgsF af{P->d_xr, P->d_xif, P->d_xs, P->d_cell_s, P->d_cell_start, n, g, pair_const_f(P), P->d_e0,
                     P->d_floc};
        af.sig = lb ? P->d_sigf : nullptr;
        af.xf = P->d_xf;
        af.xf_stride = P->xf_stride;
        set_box(f32, b, af, nblk(n, 64));
      } else if (P->pair_fast && n < (1 << 25)) {
        set_box(f64, b, a, nblk(n, 64));
      } else if (!P->pair_fast) {
        set_box(wav, b, a, n);
      } else {
        set_box(gen, b, a, nblk(n, 128));
      }
    }
    hp.push_back(std::move(f32));
    hp.push_back(std::move(f64));
    hp.push_back(std::move(wav));
    hp.push_back(std::move(gen));
  }

  const int gvar = B->order | (mixed ? 0x100 : 0);
  // ------------------------------------------------ Lorentz-Berthelot charge vectors (Sec. II.D)
  if (lb) {
    HostPhase chg = make_phase<LbChargeArgs>(BK_LB_CHARGE, MLS_T_ANTERP, 0, nchain);
    HostPhase sq = make_phase<SumXiArgs>(BK_SUM_XI_FINAL, MLS_T_ANTERP, 0, nchain);
    for (const Chain& c : chains) {
      const int b = c.id / 7, k = c.id % 7, n = n_of(b);
      mls_plan_s* P = c.P;
      double* part = mixed ? lb_partial_buf(P, k) : nullptr;
      if (n > 0) set_box(chg, c.id, LbChargeArgs{P->d_xs, P->d_sig, n, k, lb_charge_buf(P, k), part}, nblk(n + kSortedPad, 256));
      // mixed precision: the mean the stencils subtract (0 without atoms)
      if (mixed) set_box(sq, c.id, SumXiArgs{n > 0 ? n + kSortedPad : 0, part, lb_sum_buf(P, k)}, 1);
    }
    hp.push_back(std::move(chg));
    hp.push_back(std::move(sq));
  }

  // ------------------------------------------------ anterpolation (eq:anterpolation)
  {
    HostPhase tile = make_phase<AnterpTileArgs>(BK_ANT_TILE, MLS_T_ANTERP, gvar, nchain);
    HostPhase coll = make_phase<AnterpCollectArgs>(BK_ANT_COLLECT, MLS_T_ANTERP, gvar, nchain);
    HostPhase own = make_phase<AnterpArgs>(BK_ANT_OWNED, MLS_T_ANTERP, gvar, nchain);
    HostPhase zero = make_phase<FillDArgs>(BK_FILL_D, MLS_T_ANTERP, 0, nchain);
    HostPhase atom = make_phase<AnterpArgs>(BK_ANT_ATOMIC, MLS_T_ANTERP, gvar, nchain);
    for (const Chain& c : chains) {
      mls_plan_s* P = c.P;
      const int n = n_of(lb ? c.id / 7 : c.id);
      Level& L1 = (*c.lv)[0];
      AnterpArgs a{P->d_xs, P->d_cell_start, n, P->cg, finest(P), AntGeom{}, L1.q, c.charge};
      if (P->ant_tiles) {
        // two phases: per cell block into the expanded grid, then per point
        set_box(tile, c.id, AnterpTileArgs{P->d_xs, P->d_cell_start, P->cg, finest(P), P->ant, P->d_ant_tab,
                                           c.scratch, c.charge, P->d_flags},
                P->ant.nb[0] * P->ant.nb[1] * P->ant.nb[2]);
        set_box(coll, c.id, AnterpCollectArgs{P->ant, P->d_ant_tab, c.scratch, L1.q, L1.g}, nblk(L1.g.size, 256));
      } else if (anterp_owned_geom(P, a.ag)) {
        set_box(own, c.id, a, a.ag.nb[0] * a.ag.nb[1] * a.ag.nb[2]);
      } else {
        set_box(zero, c.id, FillDArgs{L1.q, L1.g.size}, nblk(L1.g.size, 256));
        set_box(atom, c.id, a, nblk(n, 256));
      }
    }
    hp.push_back(std::move(tile));
    hp.push_back(std::move(coll));
    hp.push_back(std::move(own));
    hp.push_back(std::move(zero));
    hp.push_back(std::move(atom));
  }

  // ------------------------------------------------ restrictions, level by level
  for (int k = 1; k < max_levels; ++k) {
    HostPhase r = make_phase<TransferArgs>(BK_RESTRICT, MLS_T_RESTRICT, gvar, nchain);
    for (const Chain& c : chains) {
      if (c.P->levels <= k) continue;
      Level& F = (*c.lv)[k - 1];
      Level& C = (*c.lv)[k];
      set_box(r, c.id, TransferArgs{F.q, F.g, nullptr, C.q, C.g}, nblk(C.g.size, 256));
    }
    hp.push_back(std::move(r));
  }

  // ------------------------------------------------ level stencils (all levels < l of all chains)
  for (int Rt : {8, 6, 4}) {
    int zc = B->tune.stencil_zc;
    if (!stencil_tile_ok(Rt, zc)) zc = 8;
    const int var = Rt | (zc << 8) | (mixed ? 0x10000 : 0);
    HostPhase st;
    st.ph.kernel = BK_STENCIL;
    st.ph.stage = MLS_T_STENCIL;
    st.ph.variant = var;
    std::vector<StencilLevel> desc;
    for (const Chain& c : chains) {
      mls_plan_s* P = c.P;
      if (P->levels < 2) continue;
      if (stencil_template(stencil_window(P)) != Rt) continue;
      for (int k = 1; k < P->levels; ++k) {
        Level& Lv = (*c.lv)[k - 1];
        StencilLevel V{};
        V.q = Lv.q;
        V.e = Lv.e;
        for (int d = 0; d < 3; ++d) V.n[d] = Lv.g.n[d];
        V.tiles_z = nblk(Lv.g.n[2], zc);
        V.tile0 = (int)st.tiles.size();
        V.scale = std::ldexp(1.0, -6 * (k - 1));
        V.inv_size = 1.0 / (double)Lv.g.size;
        V.rows = P->d_rows;
        V.wave_rows = P->d_wave_rows;
        V.wts = mixed ? (const void*)P->d_row_wf_tile : (const void*)P->d_row_w_tile;
        V.sum_xi = c.sum;
        V.wsum = P->taps_wsum;
        const int id = (int)desc.size();
        desc.push_back(V);
        for (int z = 0; z < V.tiles_z; ++z)
          for (int y = 0; y < nblk(Lv.g.n[1], 8); ++y)
            for (int x = 0; x < nblk(Lv.g.n[0], 8); ++x) st.tiles.push_back(make_int4(id, x, y, z));
      }
    }
    st.args.resize(sizeof(StencilLevel) * std::max<size_t>(desc.size(), 1));
    if (!desc.empty()) std::memcpy(st.args.data(), desc.data(), sizeof(StencilLevel) * desc.size());
    hp.push_back(std::move(st));
  }

  // ------------------------------------------------ coarsest level (eq:last-grid-periodic-transformed)
  {
    HostPhase c = make_phase<CoarsestArgs>(BK_COARSEST, MLS_T_COARSEST, 0, nchain);
    for (const Chain& ch : chains) {
      Level& L = (*ch.lv)[ch.P->levels - 1];
      // the register-row form where the level allows it (each K value read
      // serves a row of FMAs), else four output points per wave of the
      // wave-per-point form: the boxes fill the chip, and each block's
      // staging of q and K serves more outputs
      const int rows = coarsest_rows_form(L.g);
      set_box(c, ch.id, CoarsestArgs{L.q, L.g, ch.P->d_Kl, L.e, 4, rows}, coarsest_blocks(L.g, 4, rows));
    }
    hp.push_back(std::move(c));
  }

  // ------------------------------------------------ prolongations: step s brings level l-s+1 to l-s
  for (int s = 1; s < max_levels; ++s) {
    HostPhase p = make_phase<TransferArgs>(BK_PROLONG, MLS_T_PROLONG, gvar, nchain);
    for (const Chain& c : chains) {
      const int k = c.P->levels - s;   // fine level
      if (k < 1) continue;
      Level& F = (*c.lv)[k - 1];
      Level& C = (*c.lv)[k];
      set_box(p, c.id, TransferArgs{C.E, C.g, F.e, F.E, F.g}, nblk(C.g.size, 256));
    }
    hp.push_back(std::move(p));
  }

  // ------------------------------------------------ interpolation, outputs, energies (eq:interpolation)
  {
    HostPhase in = make_phase<InterpArgs>(BK_INTERP, MLS_T_INTERP, gvar, nb);
    HostPhase il = make_phase<InterpLbArgs>(BK_INTERP_LB, MLS_T_INTERP, gvar, nb);
    HostPhase en = make_phase<EnergyArgs>(BK_ENERGY, MLS_T_INTERP, 0, nb);
    for (int b : order) {
      mls_plan_s* P = B->plans[b];
      const int n = n_of(b);
      const int64_t o = B->off[b];
      if (lb) {
        InterpLbArgs a{P->d_xs, P->d_sig, P->d_perm, n, finest(P), {}, P->d_e0, P->d_floc,
                       B->forces ? B->forces + 3 * o : nullptr, P->d_partial};
        for (int k = 0; k < 7; ++k) a.E1[k] = P->lb_lv[k][0].E;
        set_box(il, b, a, nblk(n, 256));
      } else {
        OutPtrs out{B->forces ? B->forces + 3 * o : nullptr, nullptr, B->dE_dc6 ? B->dE_dc6 + o : nullptr};
        set_box(in, b, InterpArgs{P->d_xs, P->d_perm, n, finest(P), P->lv[0].E, P->d_e0, P->d_floc, P->cself, out,
                                  P->d_partial}, nblk(n, 256));
      }
      set_box(en, b, EnergyArgs{P->d_partial, nblk(n, 256), P->cself, B->energies + b}, 1);
    }
    hp.push_back(std::move(in));
    hp.push_back(std::move(il));
    hp.push_back(std::move(en));
  }

  // ------------------------------------------------ upload
  size_t total = 0;
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  std::vector<HostPhase*> keep;
  for (auto& h : hp) {
    const size_t nw = h.ph.kernel == BK_STENCIL ? h.tiles.size() : h.work.size();
    if (nw == 0) continue;
    keep.push_back(&h);
    total += align(h.args.size());
    total += align(h.ph.kernel == BK_STENCIL ? nw * sizeof(int4) : nw * sizeof(int2));
  }
  std::vector<char> host(total);
  char* dev = nullptr;
  if (total > 0) {
    hipError_t e = hipMalloc((void**)&dev, total);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("batch: allocation of the phase tables failed");
      return MLS_ERR_OOM;
    }
  }
  B->arena = dev;
  size_t at = 0;
  for (HostPhase* h : keep) {
    BatchPhase ph = h->ph;
    std::memcpy(host.data() + at, h->args.data(), h->args.size());
    ph.args = dev + at;
    at += align(h->args.size());
    if (ph.kernel == BK_STENCIL) {
      std::memcpy(host.data() + at, h->tiles.data(), h->tiles.size() * sizeof(int4));
      ph.nwork = (int)h->tiles.size();
      ph.work = dev + at;
      at += align(h->tiles.size() * sizeof(int4));
    } else {
      std::memcpy(host.data() + at, h->work.data(), h->work.size() * sizeof(int2));
      ph.nwork = (int)h->work.size();
      ph.work = dev + at;
      at += align(h->work.size() * sizeof(int2));
    }
    ph.grid = B->tune.blocks[ph.stage];
    B->phases.push_back(ph);
  }
  if (total > 0) HIP_TRY(hipMemcpy(dev, host.data(), total, hipMemcpyHostToDevice), "batch: upload phase tables");
  B->built = true;
  return MLS_OK;
}

hipError_t launch_phase(const BatchPhase& ph, hipStream_t s) {
  switch (ph.kernel) {
    case BK_PAIR_GENERIC:
    case BK_PAIR_WAVE:
    case BK_PAIR_TRIM_F64:
    case BK_PAIR_TRIM_F32: return launch_batched_pair(ph, s);
    case BK_ANT_ATOMIC:
    case BK_ANT_OWNED:
    case BK_ANT_TILE:
    case BK_ANT_COLLECT:
    case BK_RESTRICT:
    case BK_PROLONG:
    case BK_INTERP:
    case BK_INTERP_LB:
    case BK_ENERGY: return launch_batched_grid(ph, s);
    case BK_STENCIL:
    case BK_COARSEST: return launch_batched_stencil(ph, s);
    default: return launch_batched_binning(ph, s);
  }
}

// Enqueue every phase; with `ev`, record an event at each stage boundary
// (ev[k] before stage k, ev[MLS_NUM_STAGES] at the end) and keep every phase
// on `s`.  Without, the grid chain (anterpolation .. prolongation) runs on the
// batch's second stream, forked after binning and joined before
// interpolation, concurrently with the local part.
mls_status run_phases(mls_batch_s* B, hipStream_t s, hipEvent_t* ev) {
  const bool fork = !ev;
  bool forked = false, joined = false;
  int stage = -1;
  // concurrent mode: the local part's phases are submitted after the
  // anterpolation phases, whose LDS-heavy blocks then get their CUs first
  std::vector<const BatchPhase*> local;
  auto flush_local = [&]() -> mls_status {
    for (const BatchPhase* q : local) HIP_TRY(launch_phase(*q, s), "batch: launch");
    local.clear();
    return MLS_OK;
  };
  mls_status st;
  for (const BatchPhase& ph : B->phases) {
    while (ev && stage < ph.stage) HIP_TRY(hipEventRecord(ev[++stage], s), "batch: timing event");
    if (fork && !forked && ph.stage > MLS_T_BINNING) {
      HIP_TRY(hipEventRecord(B->ev_fork, s), "batch: fork");
      HIP_TRY(hipStreamWaitEvent(B->side, B->ev_fork, 0), "batch: fork");
      forked = true;
    }
    if (forked && ph.stage == MLS_T_PAIR) {
      local.push_back(&ph);
      continue;
    }
    if (forked && ph.stage > MLS_T_ANTERP && (st = flush_local()) != MLS_OK) return st;
    if (forked && !joined && ph.stage > MLS_T_PROLONG) {
      HIP_TRY(hipEventRecord(B->ev_join, B->side), "batch: join");
      HIP_TRY(hipStreamWaitEvent(s, B->ev_join, 0), "batch: join");
      joined = true;
    }
    const bool chain = forked && ph.stage >= MLS_T_ANTERP && ph.stage <= MLS_T_PROLONG;
    HIP_TRY(launch_phase(ph, chain ? B->side : s), "batch: launch");
  }
  if ((st = flush_local()) != MLS_OK) return st;
  if (forked && !joined) {
    HIP_TRY(hipEventRecord(B->ev_join, B->side), "batch: join");
    HIP_TRY(hipStreamWaitEvent(s, B->ev_join, 0), "batch: join");
  }
  while (ev && stage < MLS_NUM_STAGES) HIP_TRY(hipEventRecord(ev[++stage], s), "batch: timing event");
  return MLS_OK;
}

void apply_grids(mls_batch_s* B) {
  for (BatchPhase& ph : B->phases) ph.grid = B->tune.blocks[ph.stage];
  drop_graph(B);
}

// Per-stage times (ms) of `reps` eager evaluations, minimum over the reps.
mls_status time_stages(mls_batch_s* B, hipStream_t s, int reps, double* stage_ms, double* total_ms) {
  for (int k = 0; k < MLS_NUM_STAGES; ++k) stage_ms[k] = 1e30;
  *total_ms = 1e30;
  mls_status st;
  if ((st = run_phases(B, s, nullptr)) != MLS_OK) return st;   // warm-up
  for (int r = 0; r < reps; ++r) {
    if ((st = run_phases(B, s, B->events.data())) != MLS_OK) return st;
    HIP_TRY(hipEventSynchronize(B->events[MLS_NUM_STAGES]), "batch: timing");
    for (int k = 0; k < MLS_NUM_STAGES; ++k) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, B->events[k], B->events[k + 1]), "batch: timing");
      stage_ms[k] = std::min(stage_ms[k], (double)t);
    }
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, B->events[0], B->events[MLS_NUM_STAGES]), "batch: timing");
    *total_ms = std::min(*total_ms, (double)t);
  }
  return MLS_OK;
}

// Autotuner: every stage's persistent grid over kCandidateGrids and the
// stencil tile depth over {16, 8}, timed on the caller's data; per stage the
// fastest candidate is kept.
mls_status autotune(mls_batch_s* B, hipStream_t s) {
  if (B->events.empty()) {
    B->events.resize(MLS_NUM_STAGES + 1);
    for (auto& e : B->events) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
  }
  double best[MLS_NUM_STAGES];
  int best_grid[MLS_NUM_STAGES];
  int best_zc = 16;
  for (int k = 0; k < MLS_NUM_STAGES; ++k) {
    best[k] = 1e30;
    best_grid[k] = 0;
  }
  mls_status st;
  for (int zc : {16, 8}) {
    B->tune.stencil_zc = zc;
    if ((st = build_phases(B)) != MLS_OK) return st;
    for (int g : kCandidateGrids) {
      for (int k = 0; k < MLS_NUM_STAGES; ++k) B->tune.blocks[k] = g;
      apply_grids(B);
      double ms[MLS_NUM_STAGES], tot;
      if ((st = time_stages(B, s, kTuneReps, ms, &tot)) != MLS_OK) return st;
      for (int k = 0; k < MLS_NUM_STAGES; ++k) {
        // the tile depth only matters to the stencil stage; other stages are
        // compared on the first depth only
        if (k != MLS_T_STENCIL && zc != 16) continue;
        if (ms[k] < best[k]) {
          best[k] = ms[k];
          best_grid[k] = g;
          if (k == MLS_T_STENCIL) best_zc = zc;
        }
      }
    }
  }
  for (int k = 0; k < MLS_NUM_STAGES; ++k) B->tune.blocks[k] = best_grid[k];
  B->tune.stencil_zc = best_zc;
  if ((st = build_phases(B)) != MLS_OK) return st;
  double ms[MLS_NUM_STAGES], tot;
  if ((st = time_stages(B, s, kTuneReps, ms, &tot)) != MLS_OK) return st;
  B->tune.tuned_ms = tot;
  for (int k = 0; k < MLS_NUM_STAGES; ++k) B->tune.stage_ms[k] = ms[k];
  return MLS_OK;
}

}  // namespace

extern "C" {

mls_status mls_batch_create(int nbox, const mls_params* per_box, const int64_t* n_per_box, int autotune_flag,
                            mls_batch_t* out) {
  if (!out) { set_error("mls_batch_create: null out"); return MLS_ERR_INVALID_ARG; }
  *out = nullptr;
  if (nbox < 1 || nbox > (1 << 20) || !per_box || !n_per_box) {
    set_error("mls_batch_create: need 1 <= nbox <= 2^20 and non-null per_box, n_per_box");
    return MLS_ERR_INVALID_ARG;
  }
  int64_t total = 0;
  for (int b = 0; b < nbox; ++b) {
    if (n_per_box[b] < 0 || n_per_box[b] > ((int64_t)1 << 30)) {
      set_error("mls_batch_create: box " + std::to_string(b) + " atom count outside [0, 2^30]");
      return MLS_ERR_INVALID_ARG;
    }
    if (per_box[b].precision != per_box[0].precision || per_box[b].order != per_box[0].order ||
        (per_box[b].continuity == 0 ? 2 : per_box[b].continuity) !=
            (per_box[0].continuity == 0 ? 2 : per_box[0].continuity)) {
      set_error("mls_batch_create: all boxes must share precision, order and continuity");
      return MLS_ERR_INVALID_ARG;
    }
    if (per_box[b].mixing != per_box[0].mixing) {
      set_error("mls_batch_create: all boxes must share the mixing rule");
      return MLS_ERR_INVALID_ARG;
    }

    total += n_per_box[b];
  }
  if (total > ((int64_t)1 << 31) - 1) { set_error("mls_batch_create: more than 2^31 - 1 atoms"); return MLS_ERR_INVALID_ARG; }
  mls_batch_s* B = new (std::nothrow) mls_batch_s();
  if (!B) { set_error("host allocation failed"); return MLS_ERR_OOM; }
  B->nbox = nbox;
  B->precision = per_box[0].precision;
  B->order = per_box[0].order;
  B->mixing = per_box[0].mixing;
  (void)hipGetDevice(&B->device);
  B->off.assign(nbox + 1, 0);
  for (int b = 0; b < nbox; ++b) B->off[b + 1] = B->off[b] + n_per_box[b];
  B->plans.assign(nbox, nullptr);
  auto fail = [&](mls_status st) {
    mls_batch_destroy(B);
    return st;
  };
  for (int b = 0; b < nbox; ++b) {
    mls_plan_s* P = new (std::nothrow) mls_plan_s();
    if (!P) { set_error("host allocation failed"); return fail(MLS_ERR_OOM); }
    B->plans[b] = P;
    // Lorentz-Berthelot: one buffer slot per charge vector, so each chain
    // phase runs the seven vectors of every box in one launch
    P->lb_slots = 7;
    P->ant_large_tiles = true;
    mls_status st = build_plan(per_box[b], n_per_box[b], P);
    if (st != MLS_OK) {
      set_error("box " + std::to_string(b) + ": " + mls_last_error());
      return fail(st);
    }
    if (P->levels > 1 && (P->stencil_kernel != 1 || !stencil_tile_ok(stencil_window(P), 8))) {
      set_error("box " + std::to_string(b) + ": batched level stencils need a window of at most 8 grid points "
                "(2a / h <= 8)");
      return fail(MLS_ERR_UNSUPPORTED);
    }
  }
  for (int k = 0; k < MLS_NUM_STAGES; ++k) B->tune.blocks[k] = 0;
  B->tune.stencil_zc = 16;
  B->tune.tuned_ms = 0.0;
  for (int k = 0; k < MLS_NUM_STAGES; ++k) B->tune.stage_ms[k] = 0.0;
  B->tune_pending = autotune_flag != 0;
  hipError_t e = hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) return fail(hip_fail(e, "batch: streams and events"));
  *out = B;
  return MLS_OK;
}

}  // extern "C"

namespace {

mls_status batch_evaluate(mls_batch_t B, const double* pos, const double* c6, const double* sigma, double* energies,
                          double* forces, double* dE_dc6, void* stream, const char* who) {
  const std::string w(who);
  if (!energies) { set_error(w + ": energies pointer is required"); return MLS_ERR_INVALID_ARG; }
  const bool lb = B->mixing == MLS_LORENTZ_BERTHELOT;
  if (B->off[B->nbox] > 0 && (!pos || !c6 || (lb && !sigma))) {
    set_error(w + (lb ? ": null pos, eps or sigma" : ": null pos or c6"));
    return MLS_ERR_INVALID_ARG;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != B->device) { set_error(w + ": current device differs from the batch's device"); return MLS_ERR_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  mls_status st;
  const bool same_io = B->built && pos == B->pos && c6 == B->c6 && sigma == B->sigma && energies == B->energies &&
                       forces == B->forces && dE_dc6 == B->dE_dc6;
  if (!same_io) {
    // the phase tables hold the caller's pointers: wait for work that may
    // still read the old tables before replacing them
    if (B->built) HIP_TRY(hipDeviceSynchronize(), "batch: synchronise");
    B->pos = pos;
    B->c6 = c6;
    B->sigma = sigma;
    B->energies = energies;
    B->forces = forces;
    B->dE_dc6 = dE_dc6;
    if ((st = build_phases(B)) != MLS_OK) return st;
  }
  if (B->tune_pending) {
    B->tune_pending = false;
    if ((st = autotune(B, s)) != MLS_OK) return st;
  }
  B->last_stream = s;
  if (!B->use_graph) return run_phases(B, s, nullptr);
  if (!B->exec) {
    HIP_TRY(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeRelaxed), "batch: begin capture");
    st = run_phases(B, B->cap_stream, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (st != MLS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "batch: end capture");
    B->graph = g;
    HIP_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "batch: instantiate graph");
  }
  HIP_TRY(hipGraphLaunch(B->exec, s), "batch: graph launch");
  return MLS_OK;
}

}  // namespace

extern "C" {

mls_status mls_batch_evaluate(mls_batch_t B, const double* pos, const double* c6, double* energies, double* forces,
                              double* dE_dc6, void* stream) {
  if (!B) { set_error("mls_batch_evaluate: null batch"); return MLS_ERR_INVALID_ARG; }
  if (B->mixing != MLS_GEOMETRIC) {
    set_error("mls_batch_evaluate: the batch uses Lorentz-Berthelot mixing (call mls_batch_evaluate_lb)");
    return MLS_ERR_INVALID_ARG;
  }
  return batch_evaluate(B, pos, c6, nullptr, energies, forces, dE_dc6, stream, "mls_batch_evaluate");
}

mls_status mls_batch_evaluate_lb(mls_batch_t B, const double* pos, const double* eps, const double* sigma,
                                 double* energies, double* forces, void* stream) {
  if (!B) { set_error("mls_batch_evaluate_lb: null batch"); return MLS_ERR_INVALID_ARG; }
  if (B->mixing != MLS_LORENTZ_BERTHELOT) {
    set_error("mls_batch_evaluate_lb: the batch was not created with Lorentz-Berthelot mixing");
    return MLS_ERR_INVALID_ARG;
  }
  return batch_evaluate(B, pos, eps, sigma, energies, forces, nullptr, stream, "mls_batch_evaluate_lb");
}

mls_status mls_batch_set_graph(mls_batch_t B, int enable) {
  if (!B) { set_error("mls_batch_set_graph: null batch"); return MLS_ERR_INVALID_ARG; }
  B->use_graph = enable != 0;
  return MLS_OK;
}

mls_status mls_batch_get_tuning(mls_batch_t B, mls_batch_tuning* t) {
  if (!B || !t) { set_error("mls_batch_get_tuning: null argument"); return MLS_ERR_INVALID_ARG; }
  *t = B->tune;
  return MLS_OK;
}

mls_status mls_batch_set_tuning(mls_batch_t B, const mls_batch_tuning* t) {
  if (!B || !t) { set_error("mls_batch_set_tuning: null argument"); return MLS_ERR_INVALID_ARG; }
  for (int k = 0; k < MLS_NUM_STAGES; ++k)
    if (t->blocks[k] < 0) { set_error("mls_batch_set_tuning: negative grid"); return MLS_ERR_INVALID_ARG; }
  if (t->stencil_zc != 8 && t->stencil_zc != 16) {
    set_error("mls_batch_set_tuning: stencil_zc must be 8 or 16");
    return MLS_ERR_INVALID_ARG;
  }
  if (B->built) HIP_TRY(hipDeviceSynchronize(), "batch: synchronise");
  const bool rebuild = B->built && t->stencil_zc != B->tune.stencil_zc;
  B->tune = *t;
  B->tune.tuned_ms = 0.0;
  for (int k = 0; k < MLS_NUM_STAGES; ++k) B->tune.stage_ms[k] = 0.0;
  B->tune_pending = false;
  if (rebuild) return build_phases(B);
  apply_grids(B);
  return MLS_OK;
}

mls_status mls_batch_box_info(mls_batch_t B, int box, mls_plan_info* info) {
  if (!B || !info || box < 0 || box >= B->nbox) { set_error("mls_batch_box_info: bad argument"); return MLS_ERR_INVALID_ARG; }
  return mls_plan_get_info(B->plans[box], info);
}

mls_status mls_batch_status(mls_batch_t B, int* flags) {
  if (!B || !flags) { set_error("mls_batch_status: null argument"); return MLS_ERR_INVALID_ARG; }
  HIP_TRY(hipStreamSynchronize(B->last_stream), "synchronise");
  int any = 0;
  for (auto* P : B->plans) {
    int h[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(h, P->d_flags, sizeof(h), hipMemcpyDeviceToHost), "read flags");
    if (h[0]) HIP_TRY(hipMemset(P->d_flags, 0, sizeof(h)), "clear flags");
    any |= h[0];
  }
  *flags = any;
  if (any) { set_error("input data contained non-finite positions or non-finite/negative C6"); return MLS_ERR_NONFINITE; }
  return MLS_OK;
}

mls_status mls_batch_destroy(mls_batch_t B) {
  if (!B) return MLS_OK;
  if (B->built) (void)hipDeviceSynchronize();
  drop_phases(B);
  for (auto& e : B->events) (void)hipEventDestroy(e);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->side) {
    (void)hipStreamSynchronize(B->side);
    (void)hipStreamDestroy(B->side);
  }
  if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
  if (B->ev_join) (void)hipEventDestroy(B->ev_join);
  for (auto* P : B->plans) {
    if (!P) continue;
    free_plan(P);
    delete P;
  }
  delete B;
  return MLS_OK;
}

}  // extern "C"
