// Cell-list construction (ACEMD paper, section 3: atoms are binned by their
// coordinates, one thread per atom computing its cell, with atomic updates of
// the cell array).  Here the cell array is a CSR built by a counting sort:
//
//   k_init      clear counters, masks and status; write descriptors and the type-pair table
//   k_bin       per atom: box-fraction fixed point, cell id, atomic cell count (its slot),
//               and the atom's exclusion row folded into 128-bit index windows
//   k_scan      exclusive scan of the cell counts -> cell_start
//   k_scatter   atom -> cell_start[cell] + slot (order inside a cell still arbitrary)
//   k_finalize  rank inside the cell by original index (makes the sort stable and the
//               result deterministic) and write the sorted per-atom records
//
// Positions become 32-bit box fractions u = floor(x/L * 2^32) mod 2^32, which wraps
// every coordinate into the box; the 32-bit difference of two such values is the
// minimum-image displacement in units of L/2^32.
//
// The phases normally run as one cooperative launch (k_build_fused) with grid-wide
// synchronisation between them, since on a 23k-atom box each phase is a few
// microseconds of work and separate launches would cost more than the work; the
// per-phase kernels remain for grids too large to be co-resident.
#include <hip/hip_cooperative_groups.h>

#include <cstdlib>
#include <cstring>

#include "nb_internal.h"

namespace nb {

namespace {

constexpr double kTwo32 = 4294967296.0;

struct DescChunk {
  SysDesc d[kDescChunk];
  int first, count;
};

__device__ inline int find_system(const SysDesc *desc, int B, int atom) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].atom_begin <= atom) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_put_desc(Dev d, DescChunk c) {
  const int k = threadIdx.x;
  if (k < c.count) d.desc[c.first + k] = c.d[k];
}

__device__ inline void init_body(const Dev &d, const DescChunk &c, const double *__restrict__ sigma,
                                 const double *__restrict__ eps, int kernel, int64_t tid, int64_t stride) {
  if (tid < c.count) d.desc[c.first + tid] = c.d[tid];
  if (tid == 0) {
    d.status[0] = 0u;
    d.status[1] = kBuiltMagic;
    d.status[2] = static_cast<uint32_t>(d.N);
    d.status[3] = uses_clusters(kernel) ? 1u : 0u;
  }
  for (int64_t k = tid; k < d.n_cells; k += stride) d.cell_count[k] = 0;
  for (int64_t k = tid; k < d.N; k += stride) {
    d.excl_mask[k] = make_uint4(0u, 0u, 0u, 0u);
    d.excl_far[k] = 0u;
  }
  // Type-pair table, Lorentz-Berthelot: sigma_ij = (s_i + s_j)/2, eps_ij = sqrt(e_i e_j).
  const int T = d.T;
  for (int64_t k = tid; k < static_cast<int64_t>(T) * T; k += stride) {
    const int ti = static_cast<int>(k / T), tj = static_cast<int>(k % T);
    const double sij = 0.5 * (sigma[ti] + sigma[tj]);
    const double eij = sqrt(fmax(eps[ti], 0.0) * fmax(eps[tj], 0.0));
    const double s2 = sij * sij, s6 = s2 * s2 * s2;
    TypePair64 p;
    p.c6 = 4.0 * eij * s6;
    p.c12 = 4.0 * eij * s6 * s6;
    p.inv_sig = sij > 0.0 ? 1.0 / sij : 0.0;
    p.pad = 0.0;
    d.tab64[k] = p;
    TypePair32 q;
    q.c6 = static_cast<float>(p.c6);
    q.c12 = static_cast<float>(p.c12);
    q.inv_sig = static_cast<float>(p.inv_sig);
    q.pad = 0.f;
    d.tab32[k] = q;
  }
}

__global__ void k_init(Dev d, DescChunk c, const double *__restrict__ sigma, const double *__restrict__ eps,
                       int kernel) {
  const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  init_body(d, c, sigma, eps, kernel, tid, static_cast<int64_t>(gridDim.x) * blockDim.x);
}

__device__ inline void set_status(const Dev &d, uint32_t bit) { atomicOr(d.status, bit); }

__device__ inline void window_set(const Dev &d, int atom, int delta) {
  // delta in [-64, -1] -> bit delta + 64; delta in [1, 64] -> bit delta + 63.
  const int bit = delta < 0 ? delta + kWindow : delta + kWindow - 1;
  unsigned int *w = reinterpret_cast<unsigned int *>(&d.excl_mask[atom]);
  atomicOr(&w[bit >> 5], 1u << (bit & 31));
}

template <typename Real>
__device__ inline void bin_body(const Dev &d, int i, const Real *__restrict__ pos, const int32_t *__restrict__ type,
                                const int32_t *__restrict__ excl_off, const int32_t *__restrict__ excl_idx) {
  const int b = find_system(d.desc, d.B, i);
  const SysDesc &sd = d.desc[b];
  uint32_t u[3];
  bool finite = true;
  for (int a = 0; a < 3; ++a) {
    const double x = static_cast<double>(pos[3 * static_cast<int64_t>(i) + a]);
    finite = finite && isfinite(x);
    // One IEEE division and an exact power-of-two scaling; floor to int64 then keep 32 bits.
    const double t = floor((x / sd.box[a]) * kTwo32);
    u[a] = (isfinite(t) && fabs(t) < 9.0e18) ? static_cast<uint32_t>(static_cast<uint64_t>(static_cast<int64_t>(t)))
                                             : 0u;
  }
  if (!finite) {
    set_status(d, NB_STATUS_NONFINITE_POS);
    u[0] = u[1] = u[2] = 0u;
  }
  int c[3];
  for (int a = 0; a < 3; ++a)
    c[a] = static_cast<int>((static_cast<uint64_t>(u[a]) * static_cast<uint64_t>(sd.dims[a])) >> 32);
  const int cell = sd.cell_begin + (c[0] * sd.dims[1] + c[1]) * sd.dims[2] + c[2];
  d.atom_cell[i] = cell;
  d.atom_slot[i] = atomicAdd(&d.cell_count[cell], 1);
  d.atom_fix[i] = make_uint4(u[0], u[1], u[2], static_cast<uint32_t>(b));
  const int t = type[i];
  if (t < 0 || t >= d.T) set_status(d, NB_STATUS_BAD_TYPE);

  // Exclusions: a pair listed in either row excludes both ways, so each listed pair
  // marks the windows of both atoms (section 3: bitmaps over |i - j| <= 64).
  const int lo = excl_off[i], hi = excl_off[i + 1];
  if (hi < lo) {
    set_status(d, NB_STATUS_BAD_EXCLUSION);
    return;
  }
  const int n_sys = sd.atom_end - sd.atom_begin;
  for (int k = lo; k < hi; ++k) {
    const int jl = excl_idx[k];
    if (jl < 0 || jl >= n_sys) {
      set_status(d, NB_STATUS_BAD_EXCLUSION);
      continue;
    }
    const int j = sd.atom_begin + jl;
    const int delta = j - i;
    if (delta == 0) continue;
    if (delta >= -kWindow && delta <= kWindow) {
      window_set(d, i, delta);
      window_set(d, j, -delta);
    } else {
      atomicOr(&d.excl_far[i], 1u);
      atomicOr(&d.excl_far[j], 1u);
      set_status(d, NB_STATUS_FAR_EXCLUSION);
    }
  }
}

template <typename Real>
__global__ void k_bin(Dev d, const Real *__restrict__ pos, const int32_t *__restrict__ type,
                      const int32_t *__restrict__ excl_off, const int32_t *__restrict__ excl_idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.N) bin_body(d, i, pos, type, excl_off, excl_idx);
}

// Exclusive scan of n counts into n + 1 offsets by one workgroup: each thread
// sums a contiguous chunk, the chunk sums are scanned in LDS, then each thread
// writes its chunk.
__global__ void __launch_bounds__(1024) k_scan(const int32_t *__restrict__ count, int32_t *__restrict__ start,
                                               int64_t n) {
  __shared__ int sums[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t lo = tid * chunk, hi = lo + chunk < n ? lo + chunk : n;
  int s = 0;
  for (int64_t k = lo; k < hi; ++k) s += count[k];
  sums[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = tid >= off ? sums[tid - off] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  int run = sums[tid] - s;  // exclusive prefix of this chunk
  for (int64_t k = lo; k < hi; ++k) {
    const int c = count[k];
    start[k] = run;
    run += c;
  }
  if (tid == 1023) start[n] = sums[1023];
}

__device__ inline void scatter_body(const Dev &d, int i) {
  d.tmp[d.cell_start[d.atom_cell[i]] + d.atom_slot[i]] = i;
}

__global__ void k_scatter(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.N) scatter_body(d, i);
}

template <typename Real>
__device__ inline void finalize_body(const Dev &d, int s, const Real *__restrict__ pos,
                                     const Real *__restrict__ charge, const int32_t *__restrict__ type,
                                     double sqrt_ke) {
  const int i = d.tmp[s];
  const int cell = d.atom_cell[i];
  const int lo = d.cell_start[cell], hi = d.cell_start[cell + 1];
  int rank = 0;
  for (int k = lo; k < hi; ++k) rank += d.tmp[k] < i;
  const int dst = lo + rank;
  const uint4 f = d.atom_fix[i];
  d.s_fix[dst] = make_uint4(f.x, f.y, f.z, static_cast<uint32_t>(i));
  const double q = static_cast<double>(charge[i]);
  d.s_pos64[dst] = make_double4(static_cast<double>(pos[3 * static_cast<int64_t>(i)]),
                                static_cast<double>(pos[3 * static_cast<int64_t>(i) + 1]),
                                static_cast<double>(pos[3 * static_cast<int64_t>(i) + 2]), q);
  d.s_q32[dst] = static_cast<float>(q * sqrt_ke);
  int t = type[i];
  d.s_type[dst] = (t < 0 || t >= d.T) ? 0 : t;
}

template <typename Real>
__global__ void k_finalize(Dev d, const Real *__restrict__ pos, const Real *__restrict__ charge,
                           const int32_t *__restrict__ type, double sqrt_ke) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < d.N) finalize_body(d, s, pos, charge, type, sqrt_ke);
}

// Clusters for the cluster pair kernel: the sorted atoms of each (x, y) column
// (z-cells are contiguous inside a column) are cut into runs of 8.
__device__ inline int column_system(const SysDesc *desc, int B, int col) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].col_begin <= col) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline int col_nclu_of(const Dev &d, int col) {
  const SysDesc &sd = d.desc[column_system(d.desc, d.B, col)];
  const int nz = sd.dims[2];
  const int c0 = sd.cell_begin + (col - sd.col_begin) * nz;
  const int n = d.cell_start[c0 + nz] - d.cell_start[c0];
  return (n + 7) >> 3;
}

__global__ void k_col_count(Dev d) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col < d.n_columns) d.col_nclu[col] = col_nclu_of(d, col);
}

// Cluster k (global index): its column by binary search of col_clu_start, then
// record and bounding box (centre and half extent, in fixed point, taken relative
// to the cluster's first atom so that the minimum image is respected).
__device__ inline void cluster_body(const Dev &d, int k) {
  int lo = 0, hi = static_cast<int>(d.n_columns) - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.col_clu_start[mid] <= k) lo = mid; else hi = mid - 1;
  }
  const int col = lo;
  const int sys = column_system(d.desc, d.B, col);
  const SysDesc &sd = d.desc[sys];
  const int nz = sd.dims[2];
  const int c0 = sd.cell_begin + (col - sd.col_begin) * nz;
  const int a1 = d.cell_start[c0 + nz];
  const int b = d.cell_start[c0] + 8 * (k - d.col_clu_start[col]);
  const int cnt = a1 - b < 8 ? a1 - b : 8;
  const uint4 u0 = d.s_fix[b];
  int lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0};
  for (int m = 1; m < cnt; ++m) {
    const uint4 u = d.s_fix[b + m];
    const int dd[3] = {static_cast<int>(u.x - u0.x), static_cast<int>(u.y - u0.y), static_cast<int>(u.z - u0.z)};
    for (int a = 0; a < 3; ++a) {
      lo3[a] = dd[a] < lo3[a] ? dd[a] : lo3[a];
      hi3[a] = dd[a] > hi3[a] ? dd[a] : hi3[a];
    }
  }
  uint32_t ctr[3], half[3];
  const uint32_t base[3] = {u0.x, u0.y, u0.z};
  for (int a = 0; a < 3; ++a) {
    const int64_t mid = (static_cast<int64_t>(lo3[a]) + hi3[a]) >> 1;  // floor
    const int64_t h = (hi3[a] - mid) > (mid - lo3[a]) ? (hi3[a] - mid) : (mid - lo3[a]);
    ctr[a] = base[a] + static_cast<uint32_t>(static_cast<int32_t>(mid));
    half[a] = static_cast<uint32_t>(h);
  }
  d.clusters[k] = make_int4(b, cnt, col, sys);
  d.clu_ctr[k] = make_uint4(ctr[0], ctr[1], ctr[2], 0u);
  d.clu_half[k] = make_uint4(half[0], half[1], half[2], 0u);
}

__global__ void k_make_clusters(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < d.col_clu_start[d.n_columns]) cluster_body(d, k);
}

// Exclusive scan helpers for a 256-thread workgroup.
constexpr int kFusedBlock = 256;

__device__ inline int block_excl_scan(int v, int *lds, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int w = 0; w < kFusedBlock / 64; ++w) {
    before += w < wave ? lds[w] : 0;
    all += lds[w];
  }
  __syncthreads();
  *total = all;
  return x - v + before;
}

// Exclusive scan of count[0, n) into start[0, n] by this one workgroup.
__device__ inline void block_scan_array(const int32_t *count, int32_t *start, int64_t n, int *lds) {
  int run = 0;
  for (int64_t base = 0; base < n; base += kFusedBlock) {
    const int64_t k = base + threadIdx.x;
    const int v = k < n ? count[k] : 0;
    int tot;
    const int e = block_excl_scan(v, lds, &tot);
    if (k < n) start[k] = run + e;
    run += tot;
  }
  if (threadIdx.x == 0) start[n] = run;
}

// The whole cell-list build in one cooperative launch.
template <typename Real>
__global__ void __launch_bounds__(kFusedBlock) k_build_fused(Dev d, DescChunk c, const Real *__restrict__ pos,
                                                             const Real *__restrict__ charge,
                                                             const int32_t *__restrict__ type,
                                                             const int32_t *__restrict__ excl_off,
                                                             const int32_t *__restrict__ excl_idx,
                                                             const double *__restrict__ sigma,
                                                             const double *__restrict__ eps, int kernel,
                                                             double sqrt_ke) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  __shared__ int lds[kFusedBlock / 64];
  const int G = gridDim.x;
  const int64_t tid = blockIdx.x * static_cast<int64_t>(kFusedBlock) + threadIdx.x;
  const int64_t nthr = static_cast<int64_t>(G) * kFusedBlock;

  init_body(d, c, sigma, eps, kernel, tid, nthr);
  grid.sync();
  for (int64_t i = tid; i < d.N; i += nthr) bin_body(d, static_cast<int>(i), pos, type, excl_off, excl_idx);
  grid.sync();
  // Cell scan in three steps: chunk sums, scan of the chunk sums, chunk scans.
  const int64_t chunk = (d.n_cells + G - 1) / G;
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < d.n_cells ? lo + chunk : d.n_cells;
  {
    int sum = 0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += kFusedBlock) sum += d.cell_count[k];
    int tot;
    block_excl_scan(sum, lds, &tot);
    if (threadIdx.x == 0) d.scan_tmp[blockIdx.x] = tot;
  }
  grid.sync();
  if (blockIdx.x == 0) block_scan_array(d.scan_tmp, d.scan_tmp + kMaxFusedGrid, G, lds);
  grid.sync();
  {
    int run = d.scan_tmp[kMaxFusedGrid + blockIdx.x];
    for (int64_t base = lo; base < hi; base += kFusedBlock) {
      const int64_t k = base + threadIdx.x;
      const int v = k < hi ? d.cell_count[k] : 0;
      int tot;
      const int e = block_excl_scan(v, lds, &tot);
      if (k < hi) d.cell_start[k] = run + e;
      run += tot;
    }
    if (blockIdx.x == G - 1 && threadIdx.x == 0) d.cell_start[d.n_cells] = static_cast<int32_t>(d.N);
  }
  grid.sync();
  for (int64_t i = tid; i < d.N; i += nthr) scatter_body(d, static_cast<int>(i));
  const bool clusters = uses_clusters(kernel);
  if (clusters && blockIdx.x == G - 1) {
    // one workgroup: clusters per column and their scan
    for (int64_t col = threadIdx.x; col < d.n_columns; col += kFusedBlock)
      d.col_nclu[col] = col_nclu_of(d, static_cast<int>(col));
    __syncthreads();
    block_scan_array(d.col_nclu, d.col_clu_start, d.n_columns, lds);
  }
  grid.sync();
  for (int64_t s = tid; s < d.N; s += nthr) finalize_body(d, static_cast<int>(s), pos, charge, type, sqrt_ke);
  if (!clusters) return;
  grid.sync();
  const int n_clu = d.col_clu_start[d.n_columns];
  for (int64_t k = tid; k < n_clu; k += nthr) cluster_body(d, static_cast<int>(k));
}

unsigned grid_for(int64_t n, int block) {
  const int64_t g = (n + block - 1) / block;
  return static_cast<unsigned>(g > 0 ? g : 1);
}

}  // namespace

namespace {

// Co-resident workgroups of the fused build on the current device (cached per device).
int fused_grid_limit() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_build_fused<float>, kFusedBlock, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    int per_cu64 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu64, k_build_fused<double>, kFusedBlock, 0) != hipSuccess)
      per_cu64 = 0;
    const int lim = (per_cu < per_cu64 ? per_cu : per_cu64) * cus;
    cache[dev] = lim > 0 ? lim : -1;
  }
  return cache[dev] > 0 ? cache[dev] : 0;
}

template <typename Real>
hipError_t launch_fused(const Plan &plan, const Dev &d, const DescChunk &first, const nb_system *sys, unsigned g,
                        hipStream_t s) {
  Dev dd = d;
  DescChunk cc = first;
  const Real *pos = static_cast<const Real *>(sys->pos);
  const Real *charge = static_cast<const Real *>(sys->charge);
  const int32_t *type = sys->type;
  const int32_t *eo = sys->excl_offset;
  const int32_t *ei = sys->excl_index;
  const double *sig = sys->lj_sigma;
  const double *eps = sys->lj_eps;
  int kernel = plan.kernel;
  double sqrt_ke = sqrt(plan.ke);
  void *args[] = {&dd, &cc, &pos, &charge, &type, &eo, &ei, &sig, &eps, &kernel, &sqrt_ke};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_build_fused<Real>), dim3(g),
                                    dim3(kFusedBlock), args, 0, s);
}

}  // namespace

hipError_t launch_build(const Plan &plan, const Dev &d, const nb_system *sys, hipStream_t s) {
  // Descriptors travel as kernel arguments (no host-to-device copy), kDescChunk per launch.
  DescChunk first{};
  first.first = 0;
  first.count = plan.B < kDescChunk ? plan.B : kDescChunk;
  for (int k = 0; k < first.count; ++k) first.d[k] = plan.desc[k];
  for (int b0 = kDescChunk; b0 < plan.B; b0 += kDescChunk) {
    DescChunk c{};
    c.first = b0;
    c.count = plan.B - b0 < kDescChunk ? plan.B - b0 : kDescChunk;
    for (int k = 0; k < c.count; ++k) c.d[k] = plan.desc[b0 + k];
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, c);
  }

  // Single cooperative launch when the grid can be co-resident (NBHIP_BUILD=phased
  // selects one launch per phase instead).
  const char *mode = getenv("NBHIP_BUILD");
  const bool phased = mode && strcmp(mode, "phased") == 0;
  if (plan.N > 0 && !phased) {
    const int limit = fused_grid_limit();
    const int64_t work = plan.N > plan.n_cells ? plan.N : plan.n_cells;
    int64_t g = (work + kFusedBlock - 1) / kFusedBlock;
    g = g < kMaxFusedGrid ? g : kMaxFusedGrid;
    g = g < limit ? g : limit;
    if (g >= 1 && first.count > 0) {
      const hipError_t e = sys->pos_is_f64 ? launch_fused<double>(plan, d, first, sys, static_cast<unsigned>(g), s)
                                           : launch_fused<float>(plan, d, first, sys, static_cast<unsigned>(g), s);
      if (e == hipSuccess) return hipSuccess;
      (void)hipGetLastError();  // fall back to one launch per phase
    }
  }

  const int64_t init_work = plan.N > plan.n_cells ? plan.N : plan.n_cells;
  unsigned g_init = grid_for(init_work, kBlock);
  if (g_init > 4096) g_init = 4096;
  hipLaunchKernelGGL(k_init, dim3(g_init), dim3(kBlock), 0, s, d, first, sys->lj_sigma, sys->lj_eps, plan.kernel);
  if (plan.N == 0) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, d.cell_count, d.cell_start, d.n_cells);
    if (uses_clusters(plan.kernel)) {
      hipLaunchKernelGGL(k_col_count, dim3(grid_for(plan.n_columns, kBlock)), dim3(kBlock), 0, s, d);
      hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, d.col_nclu, d.col_clu_start, d.n_columns);
    }
    return hipGetLastError();
  }
  const unsigned g = grid_for(plan.N, kBlock);
  if (sys->pos_is_f64)
    hipLaunchKernelGGL(k_bin<double>, dim3(g), dim3(kBlock), 0, s, d, static_cast<const double *>(sys->pos),
                       sys->type, sys->excl_offset, sys->excl_index);
  else
    hipLaunchKernelGGL(k_bin<float>, dim3(g), dim3(kBlock), 0, s, d, static_cast<const float *>(sys->pos),
                       sys->type, sys->excl_offset, sys->excl_index);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, d.cell_count, d.cell_start, d.n_cells);
  hipLaunchKernelGGL(k_scatter, dim3(g), dim3(kBlock), 0, s, d);
  const double sqrt_ke = sqrt(plan.ke);
  if (sys->pos_is_f64)
    hipLaunchKernelGGL(k_finalize<double>, dim3(g), dim3(kBlock), 0, s, d, static_cast<const double *>(sys->pos),
                       static_cast<const double *>(sys->charge), sys->type, sqrt_ke);
  else
    hipLaunchKernelGGL(k_finalize<float>, dim3(g), dim3(kBlock), 0, s, d, static_cast<const float *>(sys->pos),
                       static_cast<const float *>(sys->charge), sys->type, sqrt_ke);
  if (uses_clusters(plan.kernel)) {
    hipLaunchKernelGGL(k_col_count, dim3(grid_for(plan.n_columns, kBlock)), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, d.col_nclu, d.col_clu_start, d.n_columns);
    hipLaunchKernelGGL(k_make_clusters, dim3(grid_for(plan.n_clusters_max, kBlock)), dim3(kBlock), 0, s, d);
  }
  return hipGetLastError();
}

}  // namespace nb
