// Internal declarations of the nonbonded library: per-system descriptors, the
// workspace layout and the argument block every kernel receives.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "nbhip.h"

namespace nb {

constexpr int kBlock = 256;           // threads per workgroup of the per-atom kernels
constexpr int kWaves = kBlock / 64;   // wave64
constexpr int kPart = 10;             // per-block partial sums: energy + 9 virial entries
constexpr int kWindow = 64;           // exclusion bitmap reach in original index (section 3)
constexpr int kDescChunk = 40;        // system descriptors carried by one launch (packed, 80 bytes each)
constexpr int kXcds = 8;          // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kQueueStride = 16;  // uint32 per work counter (one 64-byte line each)
constexpr uint32_t kBuiltMagic = 0x4E424831u;  // status[1]: written by nb_build_cells
constexpr int kScanTileCells = 16384;  // cells per workgroup of the multi-workgroup cell scan
constexpr int64_t kFuseCells = 16000;  // at most this many cell_start entries: one fused scan-and-scatter launch (LDS)

// Kernel variants that read the column cluster counts built by nb_build_cells.
__host__ __device__ __forceinline__ bool uses_clusters(int kernel) {
  return kernel == NB_KERNEL_CLUSTER || kernel == NB_KERNEL_CLUSTER_HALF;
}

// Workspace header words: status[0] = NB_STATUS_* bits, status[1] = kBuiltMagic,
// status[2] = atom count, status[3] = what was built (kBuiltClusters | kBuiltF64 | kBuiltJacc),
// status[4] = cluster size | work items per cluster << 8 of the cluster arrays (0 without them).
constexpr uint32_t kBuiltClusters = 1u;  // column cluster arrays (cluster kernels)
constexpr uint32_t kBuiltF64 = 2u;       // double-precision sorted positions (FP64 kernels)
constexpr uint32_t kBuiltJacc = 4u;      // zeroed half-shell accumulators
// Words 1-4 are written by the build only, so a later kernel reads them through the
// constant address space: four scalar loads issued together, and no test waits on
// another's load.
__device__ __forceinline__ bool built_for(const uint32_t *status, int64_t n_atoms, bool need_clusters,
                                          bool need_f64, bool need_jacc = false, uint32_t cluster_key = 0u) {
  using ConstU32 = const __attribute__((address_space(4))) uint32_t;
  ConstU32 *w = (ConstU32 *)status;
  const uint32_t magic = w[1], n = w[2], what = w[3], key = w[4];
  const bool ok = (magic == kBuiltMagic) & (n == static_cast<uint32_t>(n_atoms)) &
                  (!need_clusters | ((what & kBuiltClusters) != 0u)) & (!need_f64 | ((what & kBuiltF64) != 0u)) &
                  (!need_jacc | ((what & kBuiltJacc) != 0u)) & ((cluster_key == 0u) | (key == cluster_key));
  return ok;
}

// Cluster kernels: the M work items are cut into kXcds contiguous ranges, range x being
// [xcd_range_lo(M, x), xcd_range_lo(M, x + 1)), and launch slot kXcds k + x takes item k
// of range x (workgroups are dealt to the XCDs round robin, and each XCD has its own L2,
// so that an XCD works on a compact region of space).
__host__ __device__ __forceinline__ int xcd_range_lo(int64_t M, int x) {
  return static_cast<int>((M * x) / kXcds);
}
__host__ __device__ inline int item_slot(int m, int64_t M) {
  int x = kXcds - 1;
  while (x > 0 && xcd_range_lo(M, x) > m) --x;
  return kXcds * (m - xcd_range_lo(M, x)) + x;
}

// The work item of one launch slot of the cluster kernels, written by the build: what a
// wave needs before it loads its atoms and its neighbour columns' windows, in one 64-byte
// scalar load.  count 0: the slot has no item.
struct alignas(64) ItemRec {
  int32_t first, count, item, sys;  // first sorted atom, atoms, item index m, system
  int32_t cx, cy, cz0, cell_begin;  // column, z-cell of the first atom, the system's first cell
  int32_t nx, ny, nz, kx;           // the system's cell grid, stencil reach in x
  int32_t ky, kz, cz1, pad;         // stencil reach in y and z, z-cell of the last atom
};

// Per-system descriptor, resident in the workspace.  Sorted atoms of system b are
// [atom_begin, atom_end) (the sort keeps systems in order), its cells are
// [cell_begin, cell_begin + nx*ny*nz) and its per-atom-kernel blocks
// [blk_begin, blk_begin + ceil(n_b / kBlock)).
struct alignas(16) SysDesc {
  int32_t atom_begin, atom_end, cell_begin, blk_begin;
  int32_t dims[4];    // nx, ny, nz, (unused)
  int32_t reach[4];   // stencil reach in cells per dimension
  int32_t clu_begin, clu_end, col_begin, pad0;  // cluster and column ranges (cluster kernel)
  double box[4];      // L per dimension
  double inv_box[4];  // 1/L
  double scale[4];    // L / 2^32: Angstrom per fixed-point unit
  float scale2f[4];   // (L / 2^32)^2 in float, for squared distances from fixed-point deltas
};

// One entry of the type-pair table: u_LJ = c12/r^12 - c6/r^6 and
// du/dsigma_ij = (12 c12/r^12 - 6 c6/r^6) * inv_sig.
struct alignas(16) TypePair64 { double c6, c12, inv_sig, pad; };
struct alignas(16) TypePair32 { float c6, c12, inv_sig, pad; };

// Byte offsets into the workspace (all 256-aligned).
struct Layout {
  size_t status, desc, tab64, tab32, cell_count, cell_start, atom_cell, atom_slot, atom_fix, tmp, s_range, scan_tiles;
  size_t s_fix, s_pos64, s_q32, s_type, excl_mask, excl_far, partials, adj_partials;
  size_t col_clu_start, part, queue, jacc, p14_mask, rtab, vsort, items, col_info, atom_col;
  size_t total;
};

// Host-side plan derived from (system, params); recomputed by every call.
struct Plan {
  int B = 0;
  int64_t N = 0;
  int T = 0;
  int precision = 0;
  int kernel = 0;
  int div_xy = 2, div_z = 2;
  int split = 1;         // work items per cluster (cluster kernel)
  int cluster_size = 8;  // atoms per cluster (cluster kernel): 4 or 8
  int schedule = 2;      // NB_SCHED_STATIC or NB_SCHED_DYNAMIC (cluster kernel)
  int wg_per_cu = 16;    // resident one-wave workgroups per compute unit (dynamic schedule)
  double cutoff = 0, beta = 0, ke = 0;
  // Force-field options: LJ switch from r_on (0 = none), scaled 1-4 pairs (has14: the
  // system carries 1-4 lists); ff when either is in use (the pair kernels' FF variants).
  double switch_on = 0, s14_lj = 1, s14_c = 1;
  bool has14 = false, ff = false;
  // Tabulated variant: 0 direct, 1 linear, 2 cubic Hermite radial tables of table_n intervals.
  int table = 0, table_n = 0;
  int64_t n_cells = 0, n_blocks = 0, n_clusters_max = 0, n_columns = 0;
  int64_t n_item_slots = 0;  // cluster kernels: launch slots (work items, upper bound, a multiple of 8)
  std::vector<SysDesc> desc;
  Layout lay{};
};

// Pointers into one workspace, passed by value to the kernels.
struct Dev {
  uint32_t *status;
  SysDesc *desc;
  int B;
  TypePair64 *tab64;
  TypePair32 *tab32;
  int T;
  int32_t *cell_count, *cell_start;
  int32_t *scan_tiles;  // per kScanTileCells cells: their count total (multi-workgroup scan)
  int64_t n_cells;
  int32_t *atom_cell, *atom_slot, *tmp;
  int2 *s_range;     // sorted position (arrival order): the [start, end) of its atom's cell (fused build only)
  uint4 *atom_fix;   // original order: fixed-point x, y, z, system index
  uint4 *s_fix;      // sorted: fixed-point x, y, z, original index
  double4 *s_pos64;  // sorted: raw x, y, z (double), charge (double)
  float *s_q32;      // sorted: charge * sqrt(k_e) in float
  int32_t *s_type;   // sorted: type (clamped into range)
  uint4 *excl_mask;  // original order: 128-bit exclusion window
  uint4 *p14_mask;   // original order: 128-bit window of the scaled 1-4 partners (null without 1-4 lists)
  float4 *rtab;      // radial tables of the tabulated variant (null for direct evaluation)
  double4 *vsort;    // force VJP: the caller's vector v in sorted order (mixed path: times L/2^32)
  uint32_t *excl_far;// original order: nonzero if the atom has an exclusion beyond the window
  double *partials;      // [kPart][n_slots]: per-block (or per-wave) energy and virial sums
  double *adj_partials;  // [2 T][n_slots]: per-block (or per-wave) sigma / eps sums by type
  int64_t n_slots;       // max(n_blocks, cluster-kernel waves)
  int64_t N;
  int64_t n_blocks;
  // Cluster kernel: 8 consecutive sorted atoms of one (x, y) column form a cluster.
  int32_t *col_clu_start;  // [n_columns + 1] first cluster of each column (global)
  double4 *part;           // [split][N] per-wave shares of each sorted atom's force and energy (or dE/dq)
  int64_t n_columns;
  int64_t n_clusters_max;
  uint32_t *queue;         // [kXcds * kQueueStride] work counters of the dynamic schedule
  ItemRec *items;          // [n_item_slots] the work item of each launch slot (cluster kernels)
  int64_t n_item_slots;
  // Cluster kernels, for the work-item records: per (x, y) column its first cell, its sorted
  // atoms [first, end) and cx | cy << 16; per atom (original order) its global column.
  int4 *col_info;          // [n_columns]
  int32_t *atom_col;       // [N]
  // Half-shell cluster kernel: per sorted atom, force x, y, z and energy share, as four
  // arrays of N (component-major, so that the atomic additions of consecutive atoms
  // coalesce), added up by atomics; zero outside a force or energy call (the build zeroes
  // them and the finishing pass of every call that used them copies them out and zeroes
  // them again).  64-bit fixed point in units of 2^-32 kJ/mol/A (or kJ/mol), whose sums do
  // not depend on the order of the additions; the FP64 path adds a second limb in units of
  // 2^-64 (the part of each value below 2^-32), summed apart from the first.
  long long *jacc_fix;     // [4][N], null unless the half-shell kernel is selected
  long long *jacc_lo;      // [4][N], the FP64 path's second limbs (null on the mixed path)
};

// Per-call constants and outputs of the pair kernels.
// kVJP: the vector-Jacobian product of the forces with respect to charges, sigma_t and
// eps_t (the force-matching gradient).
enum PairMode : int { kForces = 0, kEnergy = 1, kAdjoint = 2, kVJP = 3 };

struct Consts {
  double rc2, beta, two_beta_sqrtpi, ke, sqrt_ke;
  float rc2f, betaf, two_beta_sqrtpif, mb2l2e, rc2_box;
  int erfc_short;  // beta R within the short FP64 erfc table's range
  // FF variants: 1-4 scale factors and the LJ switch as x = (r^2 - sw_on2) sw_inv, S = 1 for
  // x <= 0 (no switch: sw_on2 = R^2 and sw_inv = 0, so S = 1 for every pair)
  double s14_lj, s14_c, sw_on2, sw_inv;
  float s14_ljf, s14_cf, sw_on2f, sw_invf;
  // tabulated variant: 1/h of the radial tables and the last interval's index n - 1
  float tab_inv_h, tab_last;
};

struct Out {
  double *force;
  double *atom_energy;
  double *grad_pos;
  double *grad_charge;
  const double *grad_energy;
  const double *vjp_v;    // force VJP: v [N*3], caller's order
  const int32_t *excl_off;
  const int32_t *excl_idx;
  int want_part;    // write energy (and, for forces, virial) partials
  int want_virial;
};

// Host helpers (nb_api.cpp).
nb_status make_plan(const nb_system *sys, const nb_params *prm, Plan *plan);
Dev dev_view(const Plan &plan, void *ws);
void set_error(const std::string &msg);

// Optional events around pair-kernel launches (nb_pair_timer_start / _stop).
struct PairTimer {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t used = 0;
};
extern PairTimer g_pair_timer;
inline void timer_before(hipStream_t s) {
  if (g_pair_timer.on && g_pair_timer.used < g_pair_timer.ev.size())
    (void)hipEventRecord(g_pair_timer.ev[g_pair_timer.used].first, s);
}
inline void timer_after(hipStream_t s) {
  if (g_pair_timer.on && g_pair_timer.used < g_pair_timer.ev.size())
    (void)hipEventRecord(g_pair_timer.ev[g_pair_timer.used++].second, s);
}

// Launchers (nb_build.hip / nb_pair.hip); each returns hipSuccess or the first error.
hipError_t launch_build(const Plan &plan, const Dev &d, const nb_system *sys, hipStream_t s);
hipError_t launch_ewald(const Plan &plan, const Dev &d, const nb_system *sys, double *force, double *energy,
                        double *virial, hipStream_t s);
hipError_t launch_forces(const Plan &plan, const Dev &d, const nb_system *sys, double *force,
                         double *energy, double *virial, hipStream_t s);
hipError_t launch_energy(const Plan &plan, const Dev &d, const nb_system *sys, double *energy,
                         double *atom_energy, hipStream_t s);
hipError_t launch_backward(const Plan &plan, const Dev &d, const nb_system *sys,
                           const double *grad_energy, double *grad_pos, double *grad_charge,
                           double *grad_sigma, double *grad_eps, hipStream_t s);
hipError_t launch_force_vjp(const Plan &plan, const Dev &d, const nb_system *sys, const double *v,
                            double *grad_charge, double *grad_sigma, double *grad_eps, hipStream_t s);
// Build and forces on the library's own scratch array (nb_noalloc.hip); `why` receives
// the message of a non-OK return.
nb_status noalloc_forces(const Plan &p, const nb_system *sys, double *force, double *energy, double *virial,
                         hipStream_t stream, std::string *why);
// Cluster pair kernel and its finishing pass (nb_pair_cluster.hip).
void launch_cluster_pair(const Plan &plan, const Dev &d, const Consts &c, const Out &o, int mode, hipStream_t s,
                         double *energy, double *virial, const double *eps, double *grad_sigma, double *grad_eps);

}  // namespace nb
