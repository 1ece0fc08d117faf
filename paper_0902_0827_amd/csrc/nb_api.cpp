// C ABI of the nonbonded library: argument validation, the per-call plan and
// workspace layout, and dispatch to the kernel launchers.  Host code only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "nb_internal.h"
#include "nb_md.h"
#include "nb_pme.h"

namespace nb {

namespace {
thread_local std::string g_last_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

nb_status fail(nb_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

// Cells per dimension: the largest n with L/n >= R/k plus a margin of four
// fixed-point units, so that atoms more than k cells apart (in fixed point) are
// more than R apart in true coordinates.
int64_t grid_dim(double L, double cutoff, int k) {
  const double n = std::floor(k * L / (cutoff + 4.0 * L / 4294967296.0));
  return n < 1.0 ? 1 : static_cast<int64_t>(n);
}
}  // namespace

PairTimer g_pair_timer;

void set_error(const std::string &msg) { g_last_error = msg; }

nb_status make_plan(const nb_system *sys, const nb_params *prm, Plan *plan) {
  if (!sys || !prm || !plan) return fail(NB_ERR_ARG, "null system, params or output pointer");
  if (sys->n_systems < 1) return fail(NB_ERR_ARG, "n_systems must be >= 1");
  if (!sys->atom_offset || !sys->box) return fail(NB_ERR_ARG, "atom_offset and box are required host arrays");
  if (sys->pos_is_f64 != 0 && sys->pos_is_f64 != 1) return fail(NB_ERR_ARG, "pos_is_f64 must be 0 or 1");
  if (sys->n_types < 1 || sys->n_types > NB_MAX_TYPES)
    return fail(NB_ERR_ARG, "n_types must be in [1, NB_MAX_TYPES]");
  if (!(prm->cutoff > 0.0) || !std::isfinite(prm->cutoff)) return fail(NB_ERR_ARG, "cutoff must be positive and finite");
  if (!(prm->ewald_beta >= 0.0) || !std::isfinite(prm->ewald_beta)) return fail(NB_ERR_ARG, "ewald_beta must be >= 0 and finite");
  if (!std::isfinite(prm->coulomb_k)) return fail(NB_ERR_ARG, "coulomb_k must be finite");
  if (prm->precision != NB_FP64 && prm->precision != NB_MIXED) return fail(NB_ERR_ARG, "unknown precision");
  // At most 3 cells per cutoff in x and y: the pair kernel's run table holds the runs of
  // (2k+1)^2 <= 49 neighbour columns in one pass of its scan.
  if (prm->cell_div_xy < 0 || prm->cell_div_xy > 3) return fail(NB_ERR_ARG, "cell_div_xy must be in [0, 3]");
  if (prm->cell_div_z < 0 || prm->cell_div_z > 16) return fail(NB_ERR_ARG, "cell_div_z must be in [0, 16]");
  if (prm->kernel < NB_KERNEL_AUTO || prm->kernel > NB_KERNEL_CLUSTER_HALF) return fail(NB_ERR_ARG, "unknown kernel variant");
  if (prm->split < 0 || prm->split > 8) return fail(NB_ERR_ARG, "split must be in [0, 8]");
  if (prm->schedule < NB_SCHED_AUTO || prm->schedule > NB_SCHED_DYNAMIC) return fail(NB_ERR_ARG, "unknown schedule");
  if (prm->wg_per_cu < 0 || prm->wg_per_cu > 32) return fail(NB_ERR_ARG, "wg_per_cu must be in [0, 32]");
  if (prm->cluster_size != 0 && prm->cluster_size != 4 && prm->cluster_size != 8)
    return fail(NB_ERR_ARG, "cluster_size must be 0, 4 or 8");
  if (!(prm->lj_switch_on >= 0.0) || !(prm->lj_switch_on < prm->cutoff))
    return fail(NB_ERR_ARG, "lj_switch_on must be in [0, cutoff)");
  if (!std::isfinite(prm->scale14_lj) || !std::isfinite(prm->scale14_coul))
    return fail(NB_ERR_ARG, "scale14_lj and scale14_coul must be finite");
  if ((sys->pair14_offset == nullptr) != (sys->pair14_index == nullptr))
    return fail(NB_ERR_ARG, "pair14_offset and pair14_index must both be given or both be NULL");
  if (prm->table < 0 || prm->table > 2) return fail(NB_ERR_ARG, "table must be 0, 1 or 2");
  if (prm->table_size != 0 && (prm->table_size < 16 || prm->table_size > 65536))
    return fail(NB_ERR_ARG, "table_size must be 0 or in [16, 65536]");

  const int B = sys->n_systems;
  if (sys->atom_offset[0] != 0) return fail(NB_ERR_ARG, "atom_offset[0] must be 0");
  for (int b = 0; b < B; ++b)
    if (sys->atom_offset[b + 1] < sys->atom_offset[b]) return fail(NB_ERR_ARG, "atom_offset must be non-decreasing");
  const int64_t N = sys->atom_offset[B];
  if (N > INT32_MAX / 2) return fail(NB_ERR_CAPACITY, "more atoms than 32-bit indexing supports");
  if (N > 0 && (!sys->pos || !sys->charge || !sys->type || !sys->excl_offset || !sys->excl_index))
    return fail(NB_ERR_ARG, "pos, charge, type, excl_offset and excl_index must be device pointers");
  if (!sys->lj_sigma || !sys->lj_eps) return fail(NB_ERR_ARG, "lj_sigma and lj_eps are required");

  Plan p;
  p.B = B;
  p.N = N;
  p.T = sys->n_types;
  p.precision = prm->precision;
  // Default: each pair evaluated once (the half-shell cluster kernel, its per-atom sums in
  // 64-bit fixed point, one limb on the mixed path and two on the FP64 path, so results
  // stay bitwise reproducible).  Measured on the 23.6k-atom box: mixed pair kernel 55
  // against 66 us; FP64 85 against 119 us (measured with FP64 atomics, before the two
  // fixed-point limbs).
  p.kernel = prm->kernel != NB_KERNEL_AUTO ? prm->kernel : NB_KERNEL_CLUSTER_HALF;
  p.split = prm->split;  // 0: chosen below from the cluster count
  p.schedule = prm->schedule == NB_SCHED_DYNAMIC ? NB_SCHED_DYNAMIC : NB_SCHED_STATIC;  // static measured faster
  p.wg_per_cu = prm->wg_per_cu ? prm->wg_per_cu : 16;
  // Measured on the 23.6k-atom box: 8-atom clusters are faster for FP32 pair math and for
  // the half shell (FP64: 89 us against 125 us with 4-atom clusters, whose candidates are
  // staged twice as often), 4-atom clusters (fewer wasted out-of-range pairs per FP64
  // evaluation) for the FP64 full shell.
  p.cluster_size = prm->cluster_size ? prm->cluster_size
                   : (p.precision == NB_MIXED || p.kernel == NB_KERNEL_CLUSTER_HALF) ? 8 : 4;
  p.div_xy = prm->cell_div_xy ? prm->cell_div_xy : 2;
  // The cluster kernel wants thin z-cells, so that a column's atoms come out nearly z-sorted.
  p.div_z = prm->cell_div_z ? prm->cell_div_z : (p.kernel == NB_KERNEL_ATOM ? p.div_xy : 8);
  p.cutoff = prm->cutoff;
  p.beta = prm->ewald_beta;
  p.ke = prm->coulomb_k;
  p.switch_on = prm->lj_switch_on;
  p.has14 = sys->pair14_offset != nullptr;
  p.s14_lj = p.has14 ? prm->scale14_lj : 1.0;
  p.s14_c = p.has14 ? prm->scale14_coul : 1.0;
  p.ff = p.has14 || p.switch_on > 0.0;
  if (p.ff && p.kernel == NB_KERNEL_ATOM)
    return fail(NB_ERR_ARG, "the per-atom kernel supports neither the LJ switch nor 1-4 pairs");
  // the tabulated variant: mixed path, cluster kernels, plain interaction only
  p.table = p.precision == NB_MIXED ? prm->table : 0;
  if (p.table != 0 && (p.ff || p.kernel == NB_KERNEL_ATOM))
    return fail(NB_ERR_ARG, "the tables are not combined with the switch, 1-4 pairs or the per-atom kernel");
  p.table_n = p.table == 0 ? 0 : (prm->table_size ? prm->table_size : (p.table == 1 ? 4096 : 1024));
  p.desc.resize(B);
  int64_t cells = 0, blocks = 0, clusters = 0, columns = 0;
  for (int b = 0; b < B; ++b) {
    SysDesc &d = p.desc[b];
    std::memset(&d, 0, sizeof(d));
    const int div[3] = {p.div_xy, p.div_xy, p.div_z};
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
      const double L = sys->box[3 * b + a];
      if (!(L > 0.0) || !std::isfinite(L))
        return fail(NB_ERR_BOX, "box lengths must be positive and finite (system " + std::to_string(b) + ")");
      if (!(prm->cutoff < 0.5 * L))
        return fail(NB_ERR_BOX, "cutoff must be below half of every box length (system " + std::to_string(b) + ")");
      const int64_t n = grid_dim(L, prm->cutoff, div[a]);
      if (n > (1 << 20)) return fail(NB_ERR_CAPACITY, "cell grid too fine");
      d.dims[a] = static_cast<int32_t>(n);
      d.reach[a] = div[a];
      d.box[a] = L;
      d.inv_box[a] = 1.0 / L;
      d.scale[a] = L / 4294967296.0;
      d.scale2f[a] = static_cast<float>(d.scale[a] * d.scale[a]);
      ncell *= n;
    }
    const int64_t nb = sys->atom_offset[b + 1] - sys->atom_offset[b];
    d.atom_begin = static_cast<int32_t>(sys->atom_offset[b]);
    d.atom_end = static_cast<int32_t>(sys->atom_offset[b + 1]);
    d.cell_begin = static_cast<int32_t>(cells);
    d.blk_begin = static_cast<int32_t>(blocks);
    const int64_t ncol = static_cast<int64_t>(d.dims[0]) * d.dims[1];
    d.col_begin = static_cast<int32_t>(columns);
    d.clu_begin = static_cast<int32_t>(clusters);
    clusters += (nb + p.cluster_size - 1) / p.cluster_size + ncol;  // every column may end in a partial one
    d.clu_end = static_cast<int32_t>(clusters);
    columns += ncol;
    cells += ncell;
    blocks += (nb + kBlock - 1) / kBlock;
    if (cells > INT32_MAX / 2 || clusters > INT32_MAX / 2)
      return fail(NB_ERR_CAPACITY, "too many cells for 32-bit indexing");
  }
  p.n_cells = cells;
  p.n_blocks = blocks;
  p.n_clusters_max = clusters;
  // Default: one work item per cluster.  Two items per cluster hand the hardware pieces
  // half as large, but each adds its own setup, row reductions and partial sums for
  // k_finish to add: on the 23.6k-atom box (3,120 8-atom clusters, 3 waves per SIMD of
  // the MI355X) one item per cluster gives the faster step on both paths (mixed
  // 0.098 against 0.100 ms, FP64 0.161 against 0.163 ms).
  if (p.split == 0) p.split = 1;
  p.n_columns = columns;

  Layout &l = p.lay;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  const size_t T2 = static_cast<size_t>(p.T) * p.T;
  l.status = take(256);
  l.desc = take(sizeof(SysDesc) * B);
  l.tab64 = take(sizeof(TypePair64) * T2);
  l.tab32 = take(sizeof(TypePair32) * T2);
  l.cell_count = take(4 * static_cast<size_t>(cells));
  l.cell_start = take(4 * static_cast<size_t>(cells + 1));
  l.scan_tiles = take(4 * static_cast<size_t>(cells / kScanTileCells + 1));
  l.atom_cell = take(4 * static_cast<size_t>(N));
  l.atom_slot = take(4 * static_cast<size_t>(N));
  l.atom_fix = take(16 * static_cast<size_t>(N));
  l.tmp = take(4 * static_cast<size_t>(N));
  l.s_range = cells + 1 <= kFuseCells ? take(8 * static_cast<size_t>(N)) : 0;
  l.s_fix = take(16 * static_cast<size_t>(N));
  l.s_pos64 = take(32 * static_cast<size_t>(N));
  l.s_q32 = take(4 * static_cast<size_t>(N));
  l.s_type = take(4 * static_cast<size_t>(N));
  l.excl_mask = take(16 * static_cast<size_t>(N));
  l.excl_far = take(4 * static_cast<size_t>(N));
  const int64_t cluster_waves = (clusters * p.split + 7) / 8 * 8;
  const size_t nparts = static_cast<size_t>(std::max<int64_t>(std::max<int64_t>(blocks, cluster_waves), 1));
  l.partials = take(8 * kPart * nparts);
  l.adj_partials = take(8 * 2 * static_cast<size_t>(p.T) * nparts);
  l.col_clu_start = take(4 * static_cast<size_t>(columns + 1));
  l.part = take(32 * static_cast<size_t>(N) * static_cast<size_t>(p.split));
  l.queue = take(4 * static_cast<size_t>(kXcds * kQueueStride));
  // half-shell accumulators: 4 components of one 64-bit limb (mixed) or two (FP64)
  l.jacc = p.kernel == NB_KERNEL_CLUSTER_HALF ? take((p.precision == NB_FP64 ? 64 : 32) * static_cast<size_t>(N)) : 0;
  l.p14_mask = p.has14 ? take(16 * static_cast<size_t>(N)) : 0;
  l.rtab = p.table ? take(16 * static_cast<size_t>(p.table_n + 1) * static_cast<size_t>(p.table)) : 0;
  l.vsort = take(32 * static_cast<size_t>(N));
  // one record per launch slot of the cluster kernels' static grid (at least one round of 8)
  p.n_item_slots = std::max<int64_t>(cluster_waves, kXcds);
  l.items = take(sizeof(ItemRec) * static_cast<size_t>(p.n_item_slots));
  l.col_info = take(16 * static_cast<size_t>(columns));
  l.atom_col = take(4 * static_cast<size_t>(N));
  l.total = o;
  *plan = std::move(p);
  return NB_OK;
}

Dev dev_view(const Plan &p, void *ws) {
  char *base = static_cast<char *>(ws);
  const Layout &l = p.lay;
  Dev d;
  d.status = reinterpret_cast<uint32_t *>(base + l.status);
  d.desc = reinterpret_cast<SysDesc *>(base + l.desc);
  d.B = p.B;
  d.tab64 = reinterpret_cast<TypePair64 *>(base + l.tab64);
  d.tab32 = reinterpret_cast<TypePair32 *>(base + l.tab32);
  d.T = p.T;
  d.cell_count = reinterpret_cast<int32_t *>(base + l.cell_count);
  d.cell_start = reinterpret_cast<int32_t *>(base + l.cell_start);
  d.scan_tiles = reinterpret_cast<int32_t *>(base + l.scan_tiles);
  d.n_cells = p.n_cells;
  d.atom_cell = reinterpret_cast<int32_t *>(base + l.atom_cell);
  d.atom_slot = reinterpret_cast<int32_t *>(base + l.atom_slot);
  d.tmp = reinterpret_cast<int32_t *>(base + l.tmp);
  d.s_range = p.n_cells + 1 <= kFuseCells ? reinterpret_cast<int2 *>(base + l.s_range) : nullptr;
  d.atom_fix = reinterpret_cast<uint4 *>(base + l.atom_fix);
  d.s_fix = reinterpret_cast<uint4 *>(base + l.s_fix);
  d.s_pos64 = reinterpret_cast<double4 *>(base + l.s_pos64);
  d.s_q32 = reinterpret_cast<float *>(base + l.s_q32);
  d.s_type = reinterpret_cast<int32_t *>(base + l.s_type);
  d.excl_mask = reinterpret_cast<uint4 *>(base + l.excl_mask);
  d.excl_far = reinterpret_cast<uint32_t *>(base + l.excl_far);
  d.partials = reinterpret_cast<double *>(base + l.partials);
  d.adj_partials = reinterpret_cast<double *>(base + l.adj_partials);
  d.n_slots = std::max<int64_t>(std::max<int64_t>(p.n_blocks, (p.n_clusters_max * p.split + 7) / 8 * 8), 1);
  d.N = p.N;
  d.n_blocks = p.n_blocks;
  d.col_clu_start = reinterpret_cast<int32_t *>(base + l.col_clu_start);
  d.part = reinterpret_cast<double4 *>(base + l.part);
  d.n_columns = p.n_columns;
  d.n_clusters_max = p.n_clusters_max;
  d.queue = reinterpret_cast<uint32_t *>(base + l.queue);
  d.p14_mask = p.has14 ? reinterpret_cast<uint4 *>(base + l.p14_mask) : nullptr;
  d.rtab = p.table ? reinterpret_cast<float4 *>(base + l.rtab) : nullptr;
  d.vsort = reinterpret_cast<double4 *>(base + l.vsort);
  d.items = reinterpret_cast<ItemRec *>(base + l.items);
  d.n_item_slots = p.n_item_slots;
  d.col_info = reinterpret_cast<int4 *>(base + l.col_info);
  d.atom_col = reinterpret_cast<int32_t *>(base + l.atom_col);
  const bool half = p.kernel == NB_KERNEL_CLUSTER_HALF;
  d.jacc_fix = half ? reinterpret_cast<long long *>(base + l.jacc) : nullptr;
  d.jacc_lo = half && p.precision == NB_FP64 ? d.jacc_fix + 4 * p.N : nullptr;
  return d;
}

}  // namespace nb

using nb::fail;

namespace {

nb_status check_ws(const nb::Plan &p, const void *ws, size_t bytes) {
  if (!ws) return fail(NB_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(NB_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < p.lay.total)
    return fail(NB_ERR_WORKSPACE, "workspace too small: " + std::to_string(bytes) + " < " + std::to_string(p.lay.total));
  return NB_OK;
}

nb_status hip_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return NB_OK;
  return fail(NB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Records a message without letting a second exception escape (the message itself may
// fail to allocate, which leaves the previous one).
nb_status fail_nothrow(nb_status code, const char *what, const char *why) noexcept {
  try {
    nb::set_error(std::string(what) + ": " + why);
  } catch (...) {
  }
  return code;
}

// Runs the body of an entry point; no C++ exception crosses the C ABI.
template <typename F>
nb_status guarded(const char *what, F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail_nothrow(NB_ERR_HOST, what, "out of host memory");
  } catch (const std::exception &e) {
    return fail_nothrow(NB_ERR_HOST, what, e.what());
  } catch (...) {
    return fail_nothrow(NB_ERR_HOST, what, "unexpected exception");
  }
}

}  // namespace

extern "C" {

nb_status nb_workspace_bytes(const nb_system *sys, const nb_params *params, size_t *bytes) {
  return guarded("nb_workspace_bytes", [&]() -> nb_status {
    if (!bytes) return fail(NB_ERR_ARG, "bytes is NULL");
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    *bytes = p.lay.total;
    return NB_OK;
  });
}

nb_status nb_workspace_layout(const nb_system *sys, const nb_params *params, nb_layout *layout) {
  return guarded("nb_workspace_layout", [&]() -> nb_status {
    if (!layout) return fail(NB_ERR_ARG, "layout is NULL");
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    layout->n_atoms = p.N;
    layout->n_cells = p.n_cells;
    for (int a = 0; a < 3; ++a) layout->dims[a] = p.desc[0].dims[a];
    layout->off_cell_start = static_cast<int64_t>(p.lay.cell_start);
    layout->off_sorted_fixed = static_cast<int64_t>(p.lay.s_fix);
    layout->off_sorted_pos64 = static_cast<int64_t>(p.lay.s_pos64);
    layout->off_excl_mask = static_cast<int64_t>(p.lay.excl_mask);
    layout->off_status = static_cast<int64_t>(p.lay.status);
    layout->n_columns = p.n_columns;
    layout->n_clusters_max = p.n_clusters_max;
    layout->off_col_clu_start = static_cast<int64_t>(p.lay.col_clu_start);
    return NB_OK;
  });
}

nb_status nb_build_cells(const nb_system *sys, const nb_params *params, void *workspace,
                         size_t workspace_bytes, hipStream_t stream) {
  return guarded("nb_build_cells", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if ((st = check_ws(p, workspace, workspace_bytes)) != NB_OK) return st;
    return hip_status(nb::launch_build(p, nb::dev_view(p, workspace), sys, stream), "nb_build_cells");
  });
}

nb_status nb_nonbonded_forces(const nb_system *sys, const nb_params *params, void *workspace,
                              size_t workspace_bytes, double *force, double *energy, double *virial,
                              hipStream_t stream) {
  return guarded("nb_nonbonded_forces", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if ((st = check_ws(p, workspace, workspace_bytes)) != NB_OK) return st;
    if (!force && p.N > 0) return fail(NB_ERR_ARG, "force must not be NULL");
    return hip_status(nb::launch_forces(p, nb::dev_view(p, workspace), sys, force, energy, virial, stream),
                      "nb_nonbonded_forces");
  });
}

nb_status nb_nonbonded_energy(const nb_system *sys, const nb_params *params, void *workspace,
                              size_t workspace_bytes, double *energy, double *atom_energy,
                              hipStream_t stream) {
  return guarded("nb_nonbonded_energy", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if ((st = check_ws(p, workspace, workspace_bytes)) != NB_OK) return st;
    if (!energy) return fail(NB_ERR_ARG, "energy must not be NULL");
    return hip_status(nb::launch_energy(p, nb::dev_view(p, workspace), sys, energy, atom_energy, stream),
                      "nb_nonbonded_energy");
  });
}

nb_status nb_nonbonded_backward(const nb_system *sys, const nb_params *params, void *workspace,
                                size_t workspace_bytes, const double *grad_energy, double *grad_pos,
                                double *grad_charge, double *grad_sigma, double *grad_eps,
                                hipStream_t stream) {
  return guarded("nb_nonbonded_backward", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if ((st = check_ws(p, workspace, workspace_bytes)) != NB_OK) return st;
    if (!grad_energy) return fail(NB_ERR_ARG, "grad_energy must not be NULL");
    return hip_status(nb::launch_backward(p, nb::dev_view(p, workspace), sys, grad_energy, grad_pos,
                                          grad_charge, grad_sigma, grad_eps, stream),
                      "nb_nonbonded_backward");
  });
}

nb_status nb_nonbonded_force_vjp(const nb_system *sys, const nb_params *params, void *workspace,
                                 size_t workspace_bytes, const double *v, double *grad_charge,
                                 double *grad_sigma, double *grad_eps, hipStream_t stream) {
  return guarded("nb_nonbonded_force_vjp", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if ((st = check_ws(p, workspace, workspace_bytes)) != NB_OK) return st;
    if (!v && p.N > 0) return fail(NB_ERR_ARG, "v must not be NULL");
    if (!nb::uses_clusters(p.kernel)) return fail(NB_ERR_ARG, "the force VJP needs a cluster kernel");
    return hip_status(nb::launch_force_vjp(p, nb::dev_view(p, workspace), sys, v, grad_charge, grad_sigma,
                                           grad_eps, stream),
                      "nb_nonbonded_force_vjp");
  });
}

nb_status nb_ewald_corrections(const nb_system *sys, const nb_params *params, void *workspace,
                               size_t workspace_bytes, double *force, double *energy, double *virial,
                               hipStream_t stream) {
  return guarded("nb_ewald_corrections", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if ((st = check_ws(p, workspace, workspace_bytes)) != NB_OK) return st;
    if (!force && p.N > 0) return fail(NB_ERR_ARG, "force must not be NULL");
    return hip_status(nb::launch_ewald(p, nb::dev_view(p, workspace), sys, force, energy, virial, stream),
                      "nb_ewald_corrections");
  });
}

nb_status nb_pme_workspace_bytes(const nb_system *sys, const int32_t grid[3], size_t *bytes) {
  return guarded("nb_pme_workspace_bytes", [&]() -> nb_status {
    if (!sys || !bytes) return fail(NB_ERR_ARG, "null system or output pointer");
    if (sys->n_systems < 1) return fail(NB_ERR_ARG, "n_systems must be >= 1");
    nb::PmeLayout lay;
    std::string why = nb::pme_layout(sys->n_systems, grid, &lay);
    if (!why.empty()) return fail(NB_ERR_ARG, why);
    why = nb::pme_attach_plans(&lay);
    if (!why.empty()) return fail(NB_ERR_HIP, "nb_pme_workspace_bytes: " + why);
    *bytes = lay.total;
    return NB_OK;
  });
}

nb_status nb_pme_reciprocal(const nb_system *sys, const nb_params *params, const int32_t grid[3], void *workspace,
                            size_t workspace_bytes, double *force, double *energy, double *virial,
                            hipStream_t stream) {
  return guarded("nb_pme_reciprocal", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if (!(params->ewald_beta > 0.0)) return fail(NB_ERR_ARG, "the reciprocal sum needs ewald_beta > 0");
    nb::PmeLayout lay;
    std::string why = nb::pme_layout(sys->n_systems, grid, &lay);
    if (!why.empty()) return fail(NB_ERR_ARG, why);
    if (!force && p.N > 0) return fail(NB_ERR_ARG, "force must not be NULL");
    if (!workspace) return fail(NB_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(NB_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (workspace_bytes < lay.total)  // the grids alone do not fit
      return fail(NB_ERR_WORKSPACE,
                  "workspace too small: " + std::to_string(workspace_bytes) + " < " + std::to_string(lay.total));
    why = nb::pme_attach_plans(&lay);
    if (!why.empty()) return fail(NB_ERR_HIP, "nb_pme_reciprocal: " + why);
    if (workspace_bytes < lay.total)
      return fail(NB_ERR_WORKSPACE,
                  "workspace too small: " + std::to_string(workspace_bytes) + " < " + std::to_string(lay.total));
    std::string err;
    const hipError_t e = nb::launch_pme(lay, sys, params->ewald_beta, params->coulomb_k, workspace, force, energy,
                                        virial, stream, &err);
    if (!err.empty()) return fail(NB_ERR_HIP, "nb_pme_reciprocal: " + err);
    return hip_status(e, "nb_pme_reciprocal");
  });
}

nb_status nb_nonbonded_forces_noalloc(const nb_system *sys, const nb_params *params, double *force,
                                      double *energy, double *virial, hipStream_t stream) {
  return guarded("nb_nonbonded_forces_noalloc", [&]() -> nb_status {
    nb::Plan p;
    nb_status st = nb::make_plan(sys, params, &p);
    if (st != NB_OK) return st;
    if (!force && p.N > 0) return fail(NB_ERR_ARG, "force must not be NULL");
    std::string why;
    st = nb::noalloc_forces(p, sys, force, energy, virial, stream, &why);
    if (st != NB_OK) return fail(st, "nb_nonbonded_forces_noalloc: " + why);
    return NB_OK;
  });
}

nb_status nb_md_workspace_bytes(const nb_system *sys, const nb_params *params, const nb_md_params *md,
                                size_t *bytes) {
  return guarded("nb_md_workspace_bytes", [&]() -> nb_status {
    if (!bytes) return fail(NB_ERR_ARG, "bytes is NULL");
    nb::MdPlan mp;
    std::string why;
    const nb_status st = nb::md_plan(sys, params, md, &mp, &why);
    if (st != NB_OK) return why.empty() ? st : fail(st, "nb_md_workspace_bytes: " + why);
    *bytes = mp.ml.total;
    return NB_OK;
  });
}

namespace {
// Plan, workspace and topology checks shared by the two MD calls.
nb_status md_prepare(const char *what, const nb_system *sys, const nb_params *params, const nb_md_topology *topo,
                     const nb_md_params *md, void *workspace, size_t workspace_bytes, nb::MdPlan *mp) {
  std::string why;
  nb_status st = nb::md_plan(sys, params, md, mp, &why);
  if (st != NB_OK) return why.empty() ? st : fail(st, std::string(what) + ": " + why);
  if (!workspace) return fail(NB_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(NB_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (workspace_bytes < mp->ml.total)
    return fail(NB_ERR_WORKSPACE, "workspace too small: " + std::to_string(workspace_bytes) + " < " +
                                      std::to_string(mp->ml.total));
  why = nb::md_check_topology(*mp, topo);
  if (!why.empty()) return fail(NB_ERR_ARG, std::string(what) + ": " + why);
  if (mp->p.N > 0 && !sys->pos) return fail(NB_ERR_ARG, "pos is NULL");
  return NB_OK;
}
}  // namespace

nb_status nb_md_forces(const nb_system *sys, const nb_params *params, const nb_md_topology *topo,
                       const nb_md_params *md, void *workspace, size_t workspace_bytes, double *force,
                       double *energy, hipStream_t stream) {
  return guarded("nb_md_forces", [&]() -> nb_status {
    nb::MdPlan mp;
    nb_status st = md_prepare("nb_md_forces", sys, params, topo, md, workspace, workspace_bytes, &mp);
    if (st != NB_OK) return st;
    if (!force && mp.p.N > 0) return fail(NB_ERR_ARG, "force must not be NULL");
    std::string err;
    const hipError_t e = nb::md_forces(mp, sys, topo, md, workspace, force, energy, stream, &err);
    if (!err.empty()) return fail(NB_ERR_HIP, "nb_md_forces: " + err);
    return hip_status(e, "nb_md_forces");
  });
}

nb_status nb_md_run(const nb_system *sys, const nb_params *params, const nb_md_topology *topo,
                    const nb_md_params *md, void *workspace, size_t workspace_bytes, double *pos, double *vel,
                    int64_t first_step, int64_t n_steps, double *energy, hipStream_t stream) {
  return guarded("nb_md_run", [&]() -> nb_status {
    nb::MdPlan mp;
    nb_status st = md_prepare("nb_md_run", sys, params, topo, md, workspace, workspace_bytes, &mp);
    if (st != NB_OK) return st;
    if (n_steps < 0 || first_step < 0) return fail(NB_ERR_ARG, "first_step and n_steps must be >= 0");
    if (mp.p.N > 0 && (!vel || pos != sys->pos)) return fail(NB_ERR_ARG, "pos must be sys->pos and vel non-NULL");
    std::string err;
    const hipError_t e = nb::md_run(mp, sys, topo, md, workspace, vel, first_step, n_steps, energy, stream, &err);
    if (!err.empty()) return fail(NB_ERR_HIP, "nb_md_run: " + err);
    return hip_status(e, "nb_md_run");
  });
}

nb_status nb_read_status(const void *workspace, hipStream_t stream, uint32_t *flags) {
  return guarded("nb_read_status", [&]() -> nb_status {
    if (!workspace || !flags) return fail(NB_ERR_ARG, "workspace and flags are required");
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_status(e, "nb_read_status: stream synchronise");
    e = hipMemcpy(flags, workspace, sizeof(uint32_t), hipMemcpyDeviceToHost);
    return hip_status(e, "nb_read_status: copy");
  });
}

const char *nb_last_error(void) { return nb::g_last_error.c_str(); }

nb_status nb_pair_timer_start(int32_t capacity) {
  return guarded("nb_pair_timer_start", [&]() -> nb_status {
    if (capacity < 1 || capacity > 65536) return fail(NB_ERR_ARG, "timer capacity must be in [1, 65536]");
    nb::PairTimer &t = nb::g_pair_timer;
    if (t.on) return fail(NB_ERR_ARG, "pair timer already started");
    t.ev.clear();
    t.used = 0;
    for (int32_t k = 0; k < capacity; ++k) {
      hipEvent_t a = nullptr, b = nullptr;
      hipError_t e = hipEventCreate(&a);
      if (e == hipSuccess) e = hipEventCreate(&b);
      if (e != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        for (auto &pr : t.ev) {
          (void)hipEventDestroy(pr.first);
          (void)hipEventDestroy(pr.second);
        }
        t.ev.clear();
        return hip_status(e, "nb_pair_timer_start: event create");
      }
      t.ev.emplace_back(a, b);
    }
    t.on = true;
    return NB_OK;
  });
}

nb_status nb_pair_timer_stop(double *total_ms, int64_t *launches) {
  return guarded("nb_pair_timer_stop", [&]() -> nb_status {
    if (!total_ms || !launches) return fail(NB_ERR_ARG, "total_ms and launches are required");
    nb::PairTimer &t = nb::g_pair_timer;
    if (!t.on) return fail(NB_ERR_ARG, "pair timer not started");
    t.on = false;
    double sum = 0.0;
    hipError_t err = hipSuccess;
    for (size_t k = 0; k < t.used && err == hipSuccess; ++k) {
      err = hipEventSynchronize(t.ev[k].second);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, t.ev[k].first, t.ev[k].second);
      sum += ms;
    }
    for (auto &pr : t.ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    *total_ms = sum;
    *launches = static_cast<int64_t>(t.used);
    t.ev.clear();
    t.used = 0;
    return hip_status(err, "nb_pair_timer_stop");
  });
}

}  // extern "C"
