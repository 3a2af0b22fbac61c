// Internal declarations of the MLS dispersion library: plan layout, device
// helpers shared by the kernels, and the host-side launchers each kernel file
// provides.  Not part of the public ABI (see include/mlsdisp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mlsdisp.h"

namespace mls {

// ---------------------------------------------------------------------------
// Geometry passed by value to kernels
// ---------------------------------------------------------------------------
struct CellGeom {
  double L[3];       // box
  double invL[3];    // 1 / L (host division, correctly rounded)
  double inv_w[3];   // nc / L: cell index = trunc(x_w * inv_w)
  double w[3];       // L / nc
  int nc[3];         // cells per dimension
  int noff[3];       // neighbour-cell reach: ceil((a + skin) / w)
  int ncell;
  double margin = 0.0;   // skin / 2: how far an atom may sit outside its cell
};

struct GridDims {
  int n[3];
  int size;          // n0*n1*n2
};

// One stencil offset of the level-1 table.
struct Tap {
  int dx, dy, dz, pad;
  double w;
};

// Column of stencil taps along z sharing |dx|,|dy|: the radial kernel is
// mirror symmetric in x and y, so the up to four columns (+-dx, +-dy) are
// summed before the taps dz in [-hz, hz] with weights w[|dz|] are applied.
struct StencilRow {
  int dx, dy;        // >= 0
  int hz;            // taps dz in [-hz, hz]
  int woff;          // offset of the hz+1 weights w[|dz|] in the weight table
};

// Rows past the end of the cell-sorted atom array, filled with far-away
// positions every evaluation so the pair filter may read ahead freely.
constexpr int kSortedPad = 16;

// Waves per block of the level-stencil kernel; the tap columns are split
// into this many cost-balanced contiguous ranges at plan time.
constexpr int kStencilWaves = 8;

// Per-level bookkeeping of the grid hierarchy.
struct Level {
  GridDims g;
  double h[3];
  double* q = nullptr;   // charges q^k
  double* e = nullptr;   // evaluation e^k
  double* E = nullptr;   // prolongated total E^k (aliases e on the coarsest level)
};

// ---------------------------------------------------------------------------
// Kernel argument sets.  Every kernel body is a functor K with
//   using Args = ...;  static constexpr int kThreads;  static __device__ void run(const Args&, int blk);
// The single-plan path launches k_one<K> (one block per blk, Args by value);
// the batched path launches k_batched<K>, whose blocks walk a list of
// (box, blk) items over a device array of per-box Args.
// ---------------------------------------------------------------------------
struct GridGeom {
  int n[3];
  double invh[3];
};

// owner-computes anterpolation blocking (cells per block, blocks, halo cells)
struct AntGeom {
  int cb[3];
  int nb[3];
  int nh[3];
};

// gc[j]: gamma_k = sum_j gc[j] v^j with v = rho^12 (zero beyond k);
// gq[j] = 12 (j + 1) gc[j + 1]: gamma_k'(rho) / rho = rho^10 sum_j gq[j] v^j.
struct PairConst {
  double a2, inv_a2, inv_a6, inv_a8;
  double gc[5], gq[4];
  // FP32 candidate filter of the FP64 kernel: threshold (a^2 widened by the
  // FP32 rounding of the filter coordinates), cell widths, box
  float a2f, wf[3], Lf[3];
};

struct PairConstF {
  float a2, inv_a2, inv_a6, inv_a8;
  float w[3];
  float gc[5], gq[4];
  float a2f;    // filter threshold: a^2 widened by the FP32 rounding of absolute x
  float L[3];   // box (periodic image shift of the filter's x)
};

struct OutPtrs {
  double* forces;
  double* potential;
  double* dE_dc6;
};

struct FillArgs { int* p; int n; };
struct FillDArgs { double* p; int n; };
struct BinCountArgs {
  const double* pos; const double* c6; int n; CellGeom g;
  int* cid; int* slot; int* count; double4* xw; int* flags;
  double c6_scale;   // xi = sqrt(c6_scale * c6): 1 for C6, 2 for Lorentz-Berthelot epsilon
  double* xi_partial = nullptr;   // per-block sums of xi in original order (single plans, mixed)
  const int* cond = nullptr;      // if set and *cond == 0 the binning is skipped (neighbour reuse)
  double* xref = nullptr;         // if set: the positions of this binning (neighbour reuse)
};
// Neighbour reuse (plans with a skin): after a binning the atoms keep their
// sorted slots and cells; each later evaluation either bins again (*cond set
// by the displacement check) or re-gathers the new positions through perm.
struct DispCheckArgs { const double* pos; const double* xref; int n; double lim2; int* cond; };
struct RegatherArgs {
  const double* pos; const int* perm; const int* cell_s; int n; CellGeom g; const int* cond;
  double4* xs; float4* xr; float* xf; int xf_stride;
};
// molecular dynamics (md.hip): repulsion of eq:disp-pair-pot and velocity Verlet
struct RepGatherArgs { const int* perm; const double* c12; int n; double* x12s; float* x12f; int* flags; };
struct RepPairArgs {
  const double4* xs; const double* x12s; const int* cell_s; const int* cell_start; CellGeom g;
  int nr[3]; double rc2; int n; double* frep; double* partial;
};
constexpr int kMdEnd = 1, kMdStart = 2, kMdSlowEnd = 4, kMdSlowStart = 8, kMdMidEnd = 16, kMdMidStart = 32;
struct MdStepArgs {
  double* pos; double* vel; const double* forces; const double* inv_mass; int n;
  double hdt, dt; int mode; double* partial; int* flags;
  const double* fslow = nullptr;   // multiple time stepping: slow forces and their half-kick factor
  double hslow = 0.0;
  const double* fmid = nullptr;    // three time scales: the level-1 grid forces and their factor
  double hmid = 0.0;
};
struct LocalOutArgs {
  const double4* xs; const int* perm; int n; const double* e0; const double* floc; const double* frep;
  double* forces; double* partial;
};
struct LocalEnergyArgs {
  const double* partial; int nb; const double* rep_partial; int rep_nb; double* energy;
};
struct AddForcesArgs { double* forces; const double* add; int n3; };
struct MdKineticArgs { const double* partial; int npartial; double* out; };
struct LbGatherArgs { const int* perm; int n; const double* sigma; double* sig_s; int* flags; float* sig_f; };
// partial: if set, per-block sums of the charges (the mean the mixed stencil
// subtracts)
struct LbChargeArgs { const double4* xs; const double* sig_s; int n; int k; double* charge; double* partial; };
struct ScanArgs { int* count; int m; int* start; int* bsum; int* bmax; int* max_count; const int* cond = nullptr; };
// Bucketed binning (single plans): a bucket is a run of 2^shift consecutive
// cell ids; hist[bucket * nblk + blk] counts the atoms of block blk in the
// bucket, then (scanned in place, per scan block; bsum: the scan blocks'
// totals) gives where they start in tmp.
struct BinBucketArgs {
  const double* pos; const double* c6; int n; CellGeom g; int* cid; double4* xw; int* flags; double c6_scale;
  double* xi_partial; const int* cond; double* xref;
  int shift; int nbucket; int nblk; int* hist;
};
struct BucketScatterArgs {
  const int* cid; int n; int shift; int nbucket; int nblk; const int* hist; const int* bsum; int2* tmp;
  const int* cond;
};
struct BucketSortArgs {
  const int* hist; const int* bsum; int nblk; int shift; int nbucket; const int2* tmp; int2* tmp2; int n; int* start;
  int* perm; const double4* xw; double4* xs; int* cell_s; float4* xr; float* xif; CellGeom g; const int* cond;
  float* xf; int xf_stride;
};
struct ScatterArgs { const int* cid; const int* slot; int n; const int* start; int2* perm_tmp; const int* cond = nullptr; };
struct RankArgs { const int* start; const int2* perm_tmp; int n; int* perm; };
// Rank of each atom among its cell's atoms by original index, fused with the
// gather of the sorted arrays (single plans).
struct RankGatherArgs {
  const int* start; const int2* perm_tmp; int n; int* perm; const double4* xw;
  double4* xs; int* cell_s; float4* xr; float* xif; CellGeom g;
  const int* cond = nullptr;
  float* xf = nullptr;    // mixed precision: filter coordinates x, y, z (absolute x, cell-relative y, z), SoA
  int xf_stride = 0;      // floats per coordinate array of xf
};
struct GatherArgs {
  const int* perm; int n; const double4* xw;
  double4* xs; int* cell_s; float4* xr; float* xif; CellGeom g;
  double* xi_partial;   // mixed precision: per-block sums of xi (else null)
  float* xf = nullptr;  // mixed precision: filter coordinates, SoA
  int xf_stride = 0;
};
struct SumXiArgs { int rows; const double* partial; double* out; };   // partials of ceil(rows / 256) gather blocks
// The repulsive term of the MD entry points, evaluated by the pair kernels on
// the pairs they already hold (rc <= a): sorted sqrt(C12) in FP64 (and FP32
// for the mixed kernel), the cutoff, the sorted (n,3) forces and one energy
// sum per block.
struct PairRep {
  const double* x12; const float* x12f; double rc2; double* frep; double* partial;
};
struct PairArgs {
  const double4* xs; const int* cell_s; const int* cstart; int n; CellGeom g; PairConst pc;
  double* e0; double* floc;
  const double* sig;      // Lorentz-Berthelot: sorted sigma (source weight e_j s_ij^6)
  PairRep rep{};
  const float* xf = nullptr;   // FP32 filter coordinates (three arrays of xf_stride floats)
  int xf_stride = 0;
};
struct PairArgsF {
  const float4* xr; const float* xif; const double4* xs; const int* cell_s; const int* cstart;
  int n; CellGeom g; PairConstF pc; double* e0; double* floc;
  PairRep rep{};
  const float* sig = nullptr;   // Lorentz-Berthelot: sorted sigma in FP32
  const float* xf = nullptr;    // filter coordinates: x (absolute), y, z (cell-relative) arrays
  int xf_stride = 0;            // floats per array
};
struct AnterpArgs {
  const double4* xs; const int* cstart; int n; CellGeom cg; GridGeom gg; AntGeom ag; double* q;
  const double* charge;   // sorted charges (else the xi in xs.w)
};
// Two-phase anterpolation of single plans: blocks of linked cells, each with
// the range of finest points its atoms reach (unwrapped), laid side by side in
// an expanded grid of NX[0] x NX[1] x NX[2] points; for every finest point the
// expanded coordinates that hold its contributions (up to four per
// dimension).  Integer tables at the offsets below.
// doubles of one block's LDS tile, in two capacities.  Single plans take the
// small one where their tables fit it (14^3: blocks of 6^3 half-cutoff cells
// at a = 3, h = 1; the 22 KB tile lets six blocks share a CU, against four for
// 16^3 tiles: anterpolation and interpolation 5 % faster, the 10^6-atom mixed
// evaluation 0.658 -> 0.645 ms).  The boxes of a batch take the large one:
// their blocks then cover more of a small box, and fewer, fuller blocks made
// the batched evaluation 4 % faster than the small tiles.
constexpr int kAntTileSmall = 2744;
constexpr int kAntTileMax = 4096;
constexpr int kAntTileRows = 256;   // cell rows (y, z) of one block
struct AntTiles {
  int nb[3];        // blocks per dimension
  int NX[3];        // expanded grid size per dimension
  int off_c[3];     // nb + 1 cell boundaries
  int off_e[3];     // nb first reached points (unwrapped)
  int off_len[3];   // nb reached lengths
  int off_x0[3];    // nb offsets into the expanded grid
  int off_cov[3];   // n int4: covering expanded coordinates (-1: none); 16-byte aligned
};
struct AnterpTileArgs {
  const double4* xs; const int* cstart; CellGeom cg; GridGeom gg; AntTiles t; const int* tab;
  double* scratch; const double* charge; int* flags;
};
struct AnterpCollectArgs { AntTiles t; const int* tab; const double* scratch; double* q; GridDims g; };
struct TransferArgs {              // restriction (fine -> coarse) and prolongation (coarse -> fine)
  const double* src; GridDims gs;  // q^{k-1} (restriction) or E^{k+1} (prolongation)
  const double* add;               // prolongation: e^k added to the interpolated values
  double* dst; GridDims gd;
};
struct InterpArgs {
  const double4* xs; const int* perm; int n; GridGeom gg; const double* E1; const double* e0;
  const double* floc; double cself; OutPtrs out; double* partial;
  const double* frep = nullptr;   // sorted (n,3) repulsive forces added to the output, or null
  int grid_only = 0;              // 1: the grid part alone (no e0, no local forces)
};
// Interpolation over the anterpolation's blocks of linked cells: each block
// stages the finest-grid values its atoms reach in LDS.
struct InterpTileArgs {
  InterpArgs a; const int* cstart; CellGeom cg; AntTiles t; const int* tab; int* flags;
};
struct EnergyArgs {
  const double* partial; int nb; double cself; double* energy;
  const double* rep_partial = nullptr;  // block sums of the repulsive energy (twice E_rep), or null
  int rep_nb = 0;
  int add = 0;                          // 1: add to *energy instead of overwriting it
};
struct InterpLbArgs {
  const double4* xs; const double* sig; const int* perm; int n; GridGeom gg; const double* E1[7];
  const double* e0; const double* floc; double* forces; double* partial;
};
// outs: points per wave of the wave-per-point form; rows: the level's x
// extent when the register-row form runs (coarsest_rows_form), else 0
struct CoarsestArgs { const double* q; GridDims g; const double* K; double* e; int outs; int rows; };
constexpr int kCoarsestThreads = 512;   // threads per block of the coarsest-level kernel
constexpr int kCoarsestWaves = kCoarsestThreads / 64;

// One level of the tiled stencil: grids, scale, and the tap tables of its plan.
struct StencilLevel {
  const double* q;
  double* e;
  int n[3];
  int tiles_z;                 // z chunks
  int tile0;                   // first tile index of this level
  double scale;                // 2^(-6(k-1))
  double inv_size;             // 1 / points of the level
  const StencilRow* rows;
  const int* wave_rows;
  const void* wts;             // tile weights (double, or float in mixed precision)
  const double* sum_xi;        // mixed precision: sum of xi (mean of the charges)
  double wsum;                 // sum of the level-1 weights
};

// One phase of a batched evaluation: a kernel, per-box Args in device
// memory, and its (box, blk) work list.  The stencil phase walks int4 tiles
// (StencilLevel index, tile x, y, z) instead.
enum BatchKernel {
  BK_FILL_I, BK_FILL_D, BK_BIN_COUNT, BK_SCAN_BLOCKS, BK_SCAN_SUMS, BK_SCAN_ADD, BK_SCATTER, BK_RANK, BK_GATHER,
  BK_SUM_XI_FINAL,
  BK_PAIR_GENERIC, BK_PAIR_WAVE, BK_PAIR_TRIM_F64, BK_PAIR_TRIM_F32,
  BK_ANT_ATOMIC, BK_ANT_OWNED, BK_ANT_TILE, BK_ANT_COLLECT, BK_RESTRICT, BK_PROLONG, BK_INTERP, BK_ENERGY,
  BK_STENCIL, BK_COARSEST,
  BK_LB_GATHER, BK_LB_CHARGE, BK_INTERP_LB
};

struct BatchPhase {
  int kernel = 0;              // BatchKernel
  int stage = 0;               // MLS_T_* stage it belongs to (timing and tuning)
  int variant = 0;             // order / precision / stencil window, per kernel
  void* args = nullptr;        // device array of the kernel's Args (one per box)
  void* work = nullptr;        // device int2 (box, blk) items, or int4 tiles for BK_STENCIL
  int nwork = 0;
  int grid = 0;                // persistent grid in blocks (0: one block per item)
};

// Workgroups of a launch go to the chip's eight XCDs in turn (hardware block
// b runs on XCD b mod 8), and each XCD has its own L2.  xcd_block maps b to a
// logical block so that every XCD gets one contiguous range of logical blocks
// (XCD x: [x q + min(x, r), ...) for nblk = 8 q + r); data shared by
// neighbouring blocks (nearby atoms, adjacent grid rows) is then fetched into
// one L2 instead of eight.  A bijection on [0, nblk).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int x = b % kXcds, i = b / kXcds;
  const int q = nblk / kXcds, r = nblk % kXcds;
  return x * q + (x < r ? x : r) + i;
}

template <class K>
__global__ void __launch_bounds__(K::kThreads) k_one(typename K::Args a) {
  K::run(a, xcd_block(blockIdx.x, gridDim.x));
}

template <class K>
__global__ void __launch_bounds__(K::kThreads) k_batched(const typename K::Args* __restrict__ args,
                                                         const int2* __restrict__ work, int nwork) {
  // round by round, each XCD takes one contiguous stretch of the work list
  for (int w = xcd_block(blockIdx.x, gridDim.x); w < nwork; w += gridDim.x) {
    const int2 it = work[w];
    K::run(args[it.x], it.y);
    __syncthreads();   // LDS of the item is free before the next one
  }
}

template <class K>
hipError_t launch_one(const typename K::Args& a, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  k_one<K><<<blocks, K::kThreads, 0, s>>>(a);
  return hipGetLastError();
}

// Persistent form of k_one for a kernel that should not fill the chip: the
// grid holds a fixed number of blocks, and block b (on XCD b mod 8) walks the
// items of its XCD's contiguous share of [0, nwork) with the stride of the
// blocks on that XCD.  The wave slots it leaves free on every CU serve the
// kernels of other streams.
template <class K>
__global__ void __launch_bounds__(K::kThreads) k_persist(typename K::Args a, int nwork) {
  const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
  const int q = nwork / kXcds, r = nwork % kXcds;
  const int lo = x * q + (x < r ? x : r), cnt = q + (x < r ? 1 : 0);
  const int nbx = ((int)gridDim.x - x + kXcds - 1) / kXcds;
  for (int w = i; w < cnt; w += nbx) {
    K::run(a, lo + w);
    __syncthreads();   // LDS of the item is free before the next one
  }
}

// blocks <= 0 or >= nwork: the ordinary launch of one block per item
template <class K>
hipError_t launch_persist(const typename K::Args& a, int nwork, int blocks, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (blocks <= 0 || blocks >= nwork) return launch_one<K>(a, nwork, s);
  k_persist<K><<<blocks, K::kThreads, 0, s>>>(a, nwork);
  return hipGetLastError();
}

template <class K>
hipError_t launch_batched_phase(const BatchPhase& ph, hipStream_t s) {
  if (ph.nwork == 0) return hipSuccess;
  const int grid = ph.grid > 0 ? (ph.grid < ph.nwork ? ph.grid : ph.nwork) : ph.nwork;
  k_batched<K><<<grid, K::kThreads, 0, s>>>((const typename K::Args*)ph.args, (const int2*)ph.work, ph.nwork);
  return hipGetLastError();
}

}  // namespace mls

struct mls_plan_s {
  mls_params params{};
  int levels = 0;
  int order = 4;
  int precision = 0;
  double a = 0, a2 = 0, inv_a2 = 0, inv_a6 = 0, inv_a8 = 0, cself = 0;
  int continuity = 2;              // k of the smoothing function gamma_k
  int mixing = 0;                  // mls_mixing
  std::vector<mls::Level> lb_lv[7];  // Lorentz-Berthelot: grids of charge vector k
  double* d_sig = nullptr;         // Lorentz-Berthelot: sorted sigma (n_max + pad)
  float* d_sigf = nullptr;         // Lorentz-Berthelot, mixed precision: the same in FP32
  // Lorentz-Berthelot work slots: the single-plan path runs the seven charge
  // vectors one after another through slot 0; the batched form gives each
  // vector its own slot (charges, partial sums, their sum, expanded
  // anterpolation grid) so one launch covers all seven.
  int lb_slots = 1;
  size_t lb_stride = 0;            // doubles per slot of d_charge (n_max + pad)
  int lb_npart = 0;                // partial sums per slot of d_lb_partial
  size_t ant_scratch_n = 0;        // doubles of one expanded anterpolation grid
  double* d_charge = nullptr;      // Lorentz-Berthelot: sorted charges, lb_slots x lb_stride
  double* d_lb_partial = nullptr;  // Lorentz-Berthelot, mixed: per-block charge sums per slot
  const double* charge = nullptr;  // charges the anterpolation reads (null: xi)
  double* ant_scratch = nullptr;   // expanded grid the anterpolation uses (null: d_ant_scratch)
  const double* sum_q = nullptr;   // mixed: sum of the charges the stencils read (null: Sigma xi)
  double gamma_c[5]{};             // gamma_k inside the unit ball: sum_j gamma_c[j] rho^(12 j)
  mls::CellGeom cg{};
  double invh1[3]{};               // n_1 / L
  std::vector<mls::Level> lv;      // index k-1 for level k
  int64_t n_max = 0;
  int device = 0;

  // stencil tables (levels 1..l-1)
  std::vector<mls::Tap> taps;
  std::vector<mls::StencilRow> rows;
  std::vector<double> row_w;
  int stencil_R[3]{};              // max |dx|, |dy|, |dz|
  mls::Tap* d_taps = nullptr;
  mls::StencilRow* d_rows = nullptr;
  int* d_wave_rows = nullptr;      // kStencilWaves + 1 offsets into rows
  // MFMA level stencil (mixed precision): per tap column and K-chunk the
  // 64-lane A operand of v_mfma_f32_16x16x4_f32 (the z band of the column);
  // the columns again, their woff being the column's offset in that table
  bool stencil_mfma = false;
  float* d_mfma_a = nullptr;
  mls::StencilRow* d_rows_mfma = nullptr;
  double* d_row_w_tile = nullptr;  // weights divided by the mirror duplication on the axes
  float* d_row_wf_tile = nullptr;  // the same in FP32 (mixed precision)
  int4* d_tiles = nullptr;         // (level-1, tile x, tile y, tile z) of the tiled stencil
  int ntiles = 0;
  int stencil_kernel = 1;          // 1: LDS tile kernel, 0: plane-streaming kernel
  int stencil_min_waves = 1536;    // launch-shape knob of the level stencils
  double* d_row_w = nullptr;
  float* d_row_wf = nullptr;
  double taps_wsum = 0;            // sum of level-1 weights (mean term in mixed precision)

  // coarsest kernel K_l, x fastest
  std::vector<double> Kl;
  double* d_Kl = nullptr;

  // atom workspace
  int* d_count = nullptr;          // ncell
  int* d_cell_start = nullptr;     // ncell + 1
  int* d_slot = nullptr;           // n_max: arrival slot of an atom in its cell
  double4* d_xw = nullptr;         // n_max: wrapped x,y,z + xi, original order
  int* d_bsum = nullptr;           // scan block sums
  int* d_bmax = nullptr;           // scan block maxima
  bool pair_fast = false;          // half-cutoff cells with per-atom row trimming
  int pair_after = 1;              // concurrent mode: grid-chain stages submitted before the local part
  int pair_blocks = 0;             // > 0: the trimmed pair kernels run persistent with this many blocks
  // coarse points up to which restriction and prolongation use the forms
  // with a group of lanes per coarse point
  int split_restrict = 65536, split_prolong = 0;
  int* d_cid = nullptr;            // n_max: cell of original atom
  int2* d_perm_tmp = nullptr;      // n_max: (original index, cell) in arrival order
  // bucketed binning (0 buckets: the counting sort with device-wide atomics)
  int bin_shift = 0, bin_nbucket = 0;
  int* d_bin_hist = nullptr;       // bin_nbucket * blocks + 1
  int2* d_perm_tmp2 = nullptr;     // n_max: (original index, cell) in cell order
  int* d_perm = nullptr;           // n_max
  int* d_cell_s = nullptr;         // n_max: cell of sorted atom
  double4* d_xs = nullptr;         // n_max: sorted
  float4* d_xr = nullptr;          // n_max + pad: sorted, cell-relative FP32 x,y,z and cell x index (mixed)
  float* d_xf = nullptr;           // 3 x xf_stride: sorted FP32 filter coordinates, absolute x, cell-relative y, z (mixed)
  int xf_stride = 0;               // floats per coordinate array of d_xf (n_max + pad)
  float* d_xif = nullptr;          // n_max + pad: sorted xi in FP32 (mixed)
  double* d_e0 = nullptr;          // n_max sorted local potential
  double* d_floc = nullptr;        // 3 n_max sorted local force / (xi_i)
  double* d_partial = nullptr;     // energy partial sums
  int n_partial = 0;
  double* d_scratch = nullptr;     // small reductions (grid means)
  int* d_flags = nullptr;          // [0]: input flags (1 position, 2 C6, 4 anterpolation tile overrun,
                                   //      8 C12 / inverse mass / velocity of the MD entry points)
  double* d_x12s = nullptr;        // geometric mixing: sorted sqrt(C12) (n_max + pad)
  float* d_x12f = nullptr;         // the same in FP32 (mixed precision)
  int rep_cap = 0;                 // repulsion energy block sums d_md_partial holds before the kinetic ones
  int rep_nb = 0;                  // block sums written by the last repulsion launch
  double* d_frep = nullptr;        // geometric mixing: sorted repulsive forces (n_max,3)
  double* d_md_partial = nullptr;  // geometric mixing: repulsion energy (rep_cap), kinetic and local-energy
                                   // (n_partial each) block sums
  double* d_fslow = nullptr;       // geometric mixing: grid-part forces of multiple time stepping (n_max,3)
  double* d_fmid = nullptr;        // multiple time stepping per level: the level-1 grid forces (n_max,3)
  double skin = 0.0;               // neighbour reuse: see mls_params.skin
  double* d_xref = nullptr;        // positions of the last binning (n_max,3), plans with a skin
  int* d_rebin = nullptr;          // 1: the next conditional binning runs
  double* d_efast = nullptr;       // geometric mixing: energy of an inner step's fast evaluation
  bool ant_tiles = false;          // two-phase anterpolation tables built
  bool ant_large_tiles = false;    // set before building: tables for kAntTileMax tiles only
  int ant_cap = 0;                 // tile capacity the tables were built for (kAntTileSmall or kAntTileMax)
  mls::AntTiles ant{};
  int* d_ant_tab = nullptr;
  double* d_ant_scratch = nullptr; // the expanded grid
  int* d_ncell_max = nullptr;

  // the grid chain (anterpolation .. prolongation) runs on a second stream,
  // concurrently with the local part: fork after binning, join before
  // interpolation
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // per-stage timing (mls_plan_set_timing)
  bool timing = false;
  int timing_slots = 0;            // evaluations recorded in the window
  std::vector<hipEvent_t> events;  // (MLS_NUM_STAGES + 1) per slot

  int64_t bytes = 0;
  int64_t last_n = -1;
  hipStream_t last_stream = nullptr;
  std::vector<void*> allocations;

  // Workspace placement: with `arena` set, build_plan carves every device
  // buffer out of [arena, arena + arena_cap) (256-byte aligned) instead of
  // calling hipMalloc (mls_evaluate_noalloc); `serial` keeps every stage on
  // the caller's stream (no second stream, no events).
  unsigned char* arena = nullptr;
  size_t arena_cap = 0;
  size_t arena_used = 0;
  bool serial = false;
};

namespace mls {

// error reporting (api.cpp)
void set_error(const std::string& msg);
mls_status hip_fail(hipError_t e, const char* what);

// plan construction (plan.cpp)
mls_status build_plan(const mls_params& p, int64_t n_max, mls_plan_s* plan);
void free_plan(mls_plan_s* plan);

// mls_evaluate on a built plan (api.cpp)
mls_status evaluate_plan(mls_plan_s* P, int64_t n, const double* pos, const double* c6, double* energy,
                         double* forces, double* potential, double* dE_dc6, void* stream);

// number of blocks of the cell-count scan
int scan_blocks(int ncell);
// Bucketed binning: atoms per block of its per-atom kernels, and the bucket
// geometry for ncell cells (false: too many cells for it).
int bin_block_items();
bool bin_buckets(int64_t ncell, int64_t n_max, int& shift, int& nbucket);
// halo window of the level stencil and z extent of its LDS tile
int stencil_window(const mls_plan_s* P);
// blocks of the coarsest-level kernel for a grid, `outs` output points per wave
// The register-row form serves throughput (one block per 64 output rows,
// the source rows split over the block's waves); a lone level is done sooner
// by the wave-per-point form, whose blocks spread over the chip.  Returns
// the rows argument for a batched launch of level g.
int coarsest_rows_form(const GridDims& g);
int coarsest_blocks(const GridDims& g, int outs, int rows);
int stencil_tile_zc(int R, bool f64);

// kernel launchers (one per file); all enqueue on `s` and return the launch status
hipError_t launch_binning(mls_plan_s* P, int n, const double* pos, const double* c6, hipStream_t s);
// Neighbour reuse (plans with a skin): binning that records the positions
// (first evaluation of an MD run), and the per-step alternative: check the
// displacements since then and either bin again or re-gather.
hipError_t launch_binning_ref(mls_plan_s* P, int n, const double* pos, const double* c6, hipStream_t s);
hipError_t launch_binning_reuse(mls_plan_s* P, int n, const double* pos, const double* c6, hipStream_t s);
// mixed precision: sum of xi from binning's block sums, needed by the grid
// part only (launched on the grid chain's stream, after binning)
hipError_t launch_sum_xi(mls_plan_s* P, int n, hipStream_t s);
// With `rep`, the FP32 and FP64 half-cell kernels also evaluate the repulsion
// (*fused set); other kernels leave it to launch_repulsion.
hipError_t launch_pair(mls_plan_s* P, int n, hipStream_t s, const PairRep* rep = nullptr, bool* fused = nullptr);
hipError_t launch_scan(mls_plan_s* P, int* count, int m, int* start, hipStream_t s);
hipError_t launch_anterpolate(mls_plan_s* P, int n, hipStream_t s);
hipError_t launch_restrict(mls_plan_s* P, int k_fine, hipStream_t s);
// Level stencils of levels 1..kmax (kmax = 0: all levels below the coarsest).
hipError_t launch_stencils(mls_plan_s* P, hipStream_t s, int kmax = 0);
int stencil_path(const mls_plan_s* P);   // mls_stencil_path of the plan
hipError_t launch_coarsest(mls_plan_s* P, hipStream_t s);
hipError_t launch_prolong(mls_plan_s* P, int k_fine, hipStream_t s);
// All restrictions (levels 2..l) and all prolongations (l-1..1) of an evaluation.
hipError_t launch_restrictions(mls_plan_s* P, hipStream_t s);
// drop_e1: the last prolongation writes E^1 = prolongated E^2 without e^1
// (the levels 2..l part of multiple time stepping per level)
hipError_t launch_prolongations(mls_plan_s* P, hipStream_t s, bool drop_e1 = false);
// mode: 0 the full evaluation, kInterpRep with the repulsion of the MD entry
// points, kInterpGridOnly the grid part alone (energy added to *energy)
// kInterpLevel1: interpolate e^1 (the level-1 stencil alone) instead of E^1;
// kInterpNoSelf: leave the self-energy term out of the energy
constexpr int kInterpRep = 1, kInterpGridOnly = 2, kInterpLevel1 = 4, kInterpNoSelf = 8;
hipError_t launch_interpolate(mls_plan_s* P, int n, double* energy, double* forces,
                              double* potential, double* dE_dc6, hipStream_t s, int mode = 0);
// Lorentz-Berthelot pieces: sorted sigma and flags, the sorted charges of
// vector k, and the interpolation of all seven vectors with the energy
hipError_t launch_lb_gather(mls_plan_s* P, int n, const double* sigma, hipStream_t s);
hipError_t launch_pair_lb(mls_plan_s* P, int n, hipStream_t s);
hipError_t launch_lb_charge(mls_plan_s* P, int n, int k, hipStream_t s);
hipError_t launch_interpolate_lb(mls_plan_s* P, int n, double* energy, double* forces, hipStream_t s);
hipError_t launch_binning_scaled(mls_plan_s* P, int n, const double* pos, const double* c6, double scale,
                                 hipStream_t s);
hipError_t launch_zero(double* p, int64_t count, hipStream_t s);
hipError_t launch_zero_i(int* p, int64_t count, hipStream_t s);
hipError_t launch_copy_stage(mls_plan_s* P, int what, int level, void* dst, hipStream_t s);
// molecular dynamics (md.hip): repulsion over the sorted atoms of the current
// evaluation (its forces and energy join the outputs in the interpolation,
// launch_interpolate with with_repulsion), and one velocity-Verlet
// kernel (mode kMdEnd / kMdStart) with the kinetic energy written to *kinetic
hipError_t launch_rep_gather(mls_plan_s* P, int n, const double* c12, hipStream_t s);
hipError_t launch_repulsion(mls_plan_s* P, int n, double rc, hipStream_t s);
hipError_t launch_md_step(mls_plan_s* P, int n, double* pos, double* vel, const double* forces,
                          const double* inv_mass, double dt, int mode, double* kinetic, hipStream_t s,
                          const double* fslow = nullptr, double hslow = 0.0, const double* fmid = nullptr,
                          double hmid = 0.0);
// the local part alone as MD's fast force: forces = local + repulsive forces,
// *energy = local + repulsive energy; forces += add
hipError_t launch_local_out(mls_plan_s* P, int n, double* energy, double* forces, hipStream_t s);
hipError_t launch_add_forces(double* forces, const double* add, int n, hipStream_t s);

// owner-computes anterpolation blocking of a plan (false: use the atomic kernel)
bool anterp_owned_geom(const mls_plan_s* P, AntGeom& ag);
// tables of the two-phase anterpolation; false when no blocking fits
bool ant_tiles_build(const mls_plan_s* P, AntTiles& t, std::vector<int>& tab, size_t& scratch, int cap);

// Lorentz-Berthelot slot of charge vector k and its buffers.
inline int lb_slot(const mls_plan_s* P, int k) { return P->lb_slots > 1 ? k : 0; }
inline double* lb_charge_buf(const mls_plan_s* P, int k) { return P->d_charge + (size_t)lb_slot(P, k) * P->lb_stride; }
inline double* lb_partial_buf(const mls_plan_s* P, int k) {
  return P->d_lb_partial ? P->d_lb_partial + (size_t)lb_slot(P, k) * P->lb_npart : nullptr;
}
// the sum of the charges of vector k (mixed precision; after Sigma xi in slot 0)
inline double* lb_sum_buf(const mls_plan_s* P, int k) { return P->d_scratch + 8 + lb_slot(P, k); }
inline double* lb_ant_scratch(const mls_plan_s* P, int k) {
  return P->d_ant_scratch ? P->d_ant_scratch + (size_t)lb_slot(P, k) * P->ant_scratch_n : nullptr;
}
// z extent candidates of a stencil tile for window R
bool stencil_tile_ok(int R, int zc);

// constants of the pair kernels (pair.hip) and their template variant (2:
// eq:gamma folded in, 0: any member of the smoothing family)
PairConst pair_const(const mls_plan_s* P);
PairConstF pair_const_f(const mls_plan_s* P);
int pair_variant(const mls_plan_s* P);

// batched launchers: one phase of a batched evaluation (per kernel file)
hipError_t launch_batched_binning(const BatchPhase& ph, hipStream_t s);
hipError_t launch_batched_pair(const BatchPhase& ph, hipStream_t s);
hipError_t launch_batched_grid(const BatchPhase& ph, hipStream_t s);
hipError_t launch_batched_stencil(const BatchPhase& ph, hipStream_t s);

}  // namespace mls
