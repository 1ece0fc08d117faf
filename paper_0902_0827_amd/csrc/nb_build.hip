// Cell-list construction (ACEMD paper, section 3: atoms are binned by their
// coordinates, one thread per atom computing its cell, with atomic updates of
// the cell array).  Here the cell array is a CSR built by a counting sort:
//
//   k_init      clear counters, masks and status; write descriptors and the type-pair table
//   k_bin       per atom: box-fraction fixed point, cell id, atomic cell count (its slot),
//               and the atom's exclusion row folded into 128-bit index windows
//   scan        exclusive scan of the cell counts -> cell_start; for the cluster kernels
//               also the clusters per (x, y) column and their scan -> col_clu_start
//   k_scatter   atom -> cell_start[cell] + slot (order inside a cell still arbitrary)
//   k_finalize  rank inside the cell by original index (makes the sort stable and the
//               result deterministic) and write the sorted per-atom records (the raw
//               double-precision positions only when the FP64 path will read them); for
//               the cluster kernels also the work item of every launch slot (ItemRec),
//               from the atoms that begin and end each cluster
//
// When the cell counts fit in LDS the scan and the scatter are one launch
// (k_scan_scatter), each workgroup scanning the counts itself, and one more workgroup
// (the last, without atoms) the columns.  Larger grids scan in two launches (k_scan_tiles, k_scan_apply); their
// column counts are written by k_scatter and scanned by the first workgroup of
// k_finalize, and the work items by k_item_records after it.  Empty batches take k_scan
// (one workgroup).
//
// Positions become 32-bit box fractions u = floor(x/L * 2^32) mod 2^32, which wraps
// every coordinate into the box; the 32-bit difference of two such values is the
// minimum-image displacement in units of L/2^32.
//
// Each phase depends on the whole previous one, so each is its own launch: a
// single cooperative launch with grid-wide synchronisation between the phases was
// measured slower on MI355X (a device-wide barrier across the 8 XCDs costs more
// than a kernel boundary).
#include "nb_internal.h"
#include "nb_pair_math.h"

namespace nb {

namespace {

constexpr double kTwo32 = 4294967296.0;
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 16;  // rows of kScanBlock counts per pass of block_scan
static_assert(kScanBlock * kScanPer == kScanTileCells, "one pass of block_scan covers one scan tile");

// A system descriptor as it travels in kernel arguments: the fields that cannot be
// derived on the device (80 bytes instead of 176, so that 40 fit in one launch).
struct alignas(8) PackedDesc {
  int32_t atom_begin, atom_end, cell_begin, blk_begin;
  int32_t dims[3], reach[3];
  int32_t clu_begin, clu_end, col_begin, pad;
  double box[3];
};
static_assert(sizeof(PackedDesc) == 80, "packed descriptor layout");

struct DescChunk {
  PackedDesc d[kDescChunk];
  int first, count;
};

PackedDesc pack_desc(const SysDesc &s) {
  PackedDesc p{};
  p.atom_begin = s.atom_begin;
  p.atom_end = s.atom_end;
  p.cell_begin = s.cell_begin;
  p.blk_begin = s.blk_begin;
  for (int a = 0; a < 3; ++a) {
    p.dims[a] = s.dims[a];
    p.reach[a] = s.reach[a];
    p.box[a] = s.box[a];
  }
  p.clu_begin = s.clu_begin;
  p.clu_end = s.clu_end;
  p.col_begin = s.col_begin;
  return p;
}

// The full descriptor, with the derived fields computed by the same IEEE operations as
// on the host (a correctly rounded division, an exact power-of-two scaling).
__device__ SysDesc unpack_desc(const PackedDesc &p) {
  SysDesc s;
  s.atom_begin = p.atom_begin;
  s.atom_end = p.atom_end;
  s.cell_begin = p.cell_begin;
  s.blk_begin = p.blk_begin;
  for (int a = 0; a < 3; ++a) {
    const double L = p.box[a];
    s.dims[a] = p.dims[a];
    s.reach[a] = p.reach[a];
    s.box[a] = L;
    s.inv_box[a] = 1.0 / L;
    s.scale[a] = L / 4294967296.0;
    s.scale2f[a] = static_cast<float>(s.scale[a] * s.scale[a]);
  }
  s.dims[3] = 0;
  s.reach[3] = 0;
  s.box[3] = s.inv_box[3] = s.scale[3] = 0.0;
  s.scale2f[3] = 0.f;
  s.clu_begin = p.clu_begin;
  s.clu_end = p.clu_end;
  s.col_begin = p.col_begin;
  s.pad0 = 0;
  return s;
}

__device__ inline int find_system(const SysDesc *desc, int B, int atom) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].atom_begin <= atom) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline int column_system(const SysDesc *desc, int B, int col) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].col_begin <= col) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_put_desc(Dev d, DescChunk c) {
  const int k = threadIdx.x;
  if (k < c.count) d.desc[c.first + k] = unpack_desc(c.d[k]);
}

// Radial tables of the tabulated variant (kind 1 linear, 2 cubic Hermite), n intervals of
// width h over [0, R]: node k holds, at r = k h (node 0 repeats node 1), r^-12, r^-6,
// EC = erfc(beta r)/r and FC = [erfc(beta r)/r + (2 beta/sqrt(pi)) exp(-beta^2 r^2)]/r^2,
// computed in FP64 and rounded to float; cubic tables add h times the r-derivatives:
//   -12 r^-13, -6 r^-7, -r FC, and -3 g/r^3 - 2 beta^2 (2 beta/sqrt(pi)) exp(-beta^2 r^2)/r
// with g = r^2 FC.
struct TableArgs {
  int kind, n, short_erfc;
  double h, beta, two_beta_sqrtpi;
};

__device__ inline void table_node(const Dev &d, const TableArgs &ta, int k) {
  const double r = (k == 0 ? 1 : k) * ta.h;
  const double r2 = r * r, rinv = 1.0 / r, rinv2 = rinv * rinv;
  const double r6 = rinv2 * rinv2 * rinv2;
  const double e = exp_neg_f64(ta.beta * ta.beta * r2);
  const double ec = erfcx_f64(ta.beta * r, ta.short_erfc != 0) * e * rinv;
  const double g = ec + ta.two_beta_sqrtpi * e;
  const double fc = g * rinv2;
  const float4 v = make_float4(static_cast<float>(r6 * r6), static_cast<float>(r6), static_cast<float>(ec),
                               static_cast<float>(fc));
  if (ta.kind == 1) {
    d.rtab[k] = v;
  } else {
    const double dfc = -3.0 * g * rinv2 * rinv - 2.0 * ta.beta * ta.beta * ta.two_beta_sqrtpi * e * rinv;
    d.rtab[2 * k] = v;
    d.rtab[2 * k + 1] = make_float4(static_cast<float>(-12.0 * r6 * r6 * rinv * ta.h),
                                    static_cast<float>(-6.0 * r6 * rinv * ta.h), static_cast<float>(-r * fc * ta.h),
                                    static_cast<float>(dfc * ta.h));
  }
}

__global__ void k_init(Dev d, DescChunk c, const double *__restrict__ sigma, const double *__restrict__ eps,
                       int kernel, int f64, TableArgs ta, uint32_t cluster_key) {
  const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  if (tid < c.count) d.desc[c.first + tid] = unpack_desc(c.d[tid]);
  if (tid == 0) {
    d.status[0] = 0u;
    d.status[1] = kBuiltMagic;
    d.status[2] = static_cast<uint32_t>(d.N);
    d.status[3] = (uses_clusters(kernel) ? kBuiltClusters : 0u) | (f64 ? kBuiltF64 : 0u) | (d.jacc_fix ? kBuiltJacc : 0u);
    d.status[4] = cluster_key;
  }
  // work-item slots start empty; the build fills those that have an item
  if (cluster_key)
    for (int64_t k = tid; k < d.n_item_slots; k += stride) d.items[k].count = 0;
  if (tid < kXcds) d.queue[tid * kQueueStride] = 0u;
  for (int64_t k = tid; k < d.n_cells; k += stride) d.cell_count[k] = 0;
  for (int64_t k = tid; k < d.N; k += stride) {
    d.excl_mask[k] = make_uint4(0u, 0u, 0u, 0u);
    if (d.p14_mask) d.p14_mask[k] = make_uint4(0u, 0u, 0u, 0u);
    d.excl_far[k] = 0u;
    for (int c = 0; c < 4; ++c) {
      if (d.jacc_fix) d.jacc_fix[c * d.N + k] = 0;
      if (d.jacc_lo) d.jacc_lo[c * d.N + k] = 0;
    }
  }
  if (ta.kind != 0)
    for (int64_t k = tid; k <= ta.n; k += stride) table_node(d, ta, static_cast<int>(k));
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

__device__ inline void set_status(const Dev &d, uint32_t bit) { atomicOr(d.status, bit); }

__device__ inline void window_set(uint4 *masks, int atom, int delta) {
  // delta in [-64, -1] -> bit delta + 64; delta in [1, 64] -> bit delta + 63.
  const int bit = delta < 0 ? delta + kWindow : delta + kWindow - 1;
  unsigned int *w = reinterpret_cast<unsigned int *>(&masks[atom]);
  atomicOr(&w[bit >> 5], 1u << (bit & 31));
}

// Folds atom i's row of a pair list (exclusions or scaled 1-4 pairs) into the 128-bit index
// windows `masks` (section 3: bitmaps over |i - j| <= 64).  A pair listed in either row
// counts both ways: the bits of this atom's own row are gathered in registers and added
// with one atomicOr per window word that has any; the partner's bit for this atom is set
// here only when the partner's row does not list this atom (else the partner sets it from
// its own row).  Lists usually name each pair from both sides, so this replaces four
// device-scope atomics per listed pair by about one per atom.  Pairs farther apart than the
// window call far(j); a bad row or index sets NB_STATUS_BAD_EXCLUSION.
template <typename Far>
__device__ inline void fold_row(const Dev &d, uint4 *masks, const int32_t *__restrict__ off,
                                const int32_t *__restrict__ idx, int i, const SysDesc &sd, Far far) {
  const int lo = off[i], hi = off[i + 1];
  if (hi < lo) {
    set_status(d, NB_STATUS_BAD_EXCLUSION);
    return;
  }
  const int n_sys = sd.atom_end - sd.atom_begin;
  const int il = i - sd.atom_begin;
  uint32_t own0 = 0u, own1 = 0u, own2 = 0u, own3 = 0u;
  // Entries in batches of kFoldBatch, each stage's loads independent of one another (the
  // row's partners, then their row bounds, then the first kFoldScan entries of their rows),
  // so that a row costs a few dependent load latencies instead of one per load.
  constexpr int kFoldBatch = 4, kFoldScan = 4;
  for (int k0 = lo; k0 < hi; k0 += kFoldBatch) {
    int j[kFoldBatch], jlo[kFoldBatch], jhi[kFoldBatch];
    bool win[kFoldBatch], listed[kFoldBatch];
#pragma unroll
    for (int u = 0; u < kFoldBatch; ++u) j[u] = k0 + u < hi ? idx[k0 + u] : -1;
#pragma unroll
    for (int u = 0; u < kFoldBatch; ++u) {
      const int jl = j[u];
      const bool real = k0 + u < hi;
      const bool ok = jl >= 0 && jl < n_sys;
      if (real && !ok) set_status(d, NB_STATUS_BAD_EXCLUSION);
      j[u] = ok ? sd.atom_begin + jl : i;  // a bad or missing entry acts as j = i (skipped)
      const int delta = j[u] - i;
      win[u] = delta != 0 && delta >= -kWindow && delta <= kWindow;
      if (ok && delta != 0 && !win[u]) far(j[u]);
      jlo[u] = win[u] ? off[j[u]] : 0;
      jhi[u] = win[u] ? off[j[u] + 1] : 0;
      listed[u] = false;
    }
#pragma unroll
    for (int q = 0; q < kFoldScan; ++q)
#pragma unroll
      for (int u = 0; u < kFoldBatch; ++u)
        if (jlo[u] + q < jhi[u]) listed[u] = listed[u] || idx[jlo[u] + q] == il;
#pragma unroll
    for (int u = 0; u < kFoldBatch; ++u) {
      if (!win[u]) continue;
      for (int q = jlo[u] + kFoldScan; q < jhi[u] && !listed[u]; ++q) listed[u] = idx[q] == il;  // long rows
      const int delta = j[u] - i;
      const int bit = delta < 0 ? delta + kWindow : delta + kWindow - 1;
      const uint32_t m = 1u << (bit & 31);
      const int ws = bit >> 5;
      own0 |= ws == 0 ? m : 0u;
      own1 |= ws == 1 ? m : 0u;
      own2 |= ws == 2 ? m : 0u;
      own3 |= ws == 3 ? m : 0u;
      if (!listed[u]) window_set(masks, j[u], -delta);
    }
  }
  unsigned int *w = reinterpret_cast<unsigned int *>(&masks[i]);
  if (own0) atomicOr(&w[0], own0);
  if (own1) atomicOr(&w[1], own1);
  if (own2) atomicOr(&w[2], own2);
  if (own3) atomicOr(&w[3], own3);
}

template <typename Real>
__global__ void k_bin(Dev d, const Real *__restrict__ pos, const int32_t *__restrict__ type,
                      const int32_t *__restrict__ excl_off, const int32_t *__restrict__ excl_idx,
                      const int32_t *__restrict__ p14_off, const int32_t *__restrict__ p14_idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.N) return;
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
  // the arrival slot is stored last, so that the exclusion rows' loads below are issued
  // while the atomic is in flight instead of after it has returned
  const int slot = atomicAdd(&d.cell_count[cell], 1);
  d.atom_cell[i] = cell;
  d.atom_col[i] = sd.col_begin + c[0] * sd.dims[1] + c[1];
  d.atom_fix[i] = make_uint4(u[0], u[1], u[2], static_cast<uint32_t>(b));
  const int t = type[i];
  if (t < 0 || t >= d.T) set_status(d, NB_STATUS_BAD_TYPE);

  // Exclusions: a pair listed in either row excludes both ways; beyond the window the
  // atoms carry the far flag and the pair kernels search their rows.
  fold_row(d, d.excl_mask, excl_off, excl_idx, i, sd, [&](int j) {
    atomicOr(&d.excl_far[i], 1u);
    atomicOr(&d.excl_far[j], 1u);
    set_status(d, NB_STATUS_FAR_EXCLUSION);
  });
  // Scaled 1-4 pairs: the paper's bitmaps hold them within the window only; a farther one
  // is reported and left unscaled.
  if (d.p14_mask) fold_row(d, d.p14_mask, p14_off, p14_idx, i, sd, [&](int) { set_status(d, NB_STATUS_FAR_PAIR14); });
  d.atom_slot[i] = slot;
}

// Exclusive scan of count(0 .. n-1) into store(k, prefix) for k < n and store(n, total),
// by one workgroup of kScanBlock threads.  A pass covers Rows rows of kScanBlock
// consecutive entries; thread t takes entry t of every row, so that the loads and the
// stores are coalesced.  Each row is scanned by wave shuffles (rows past n are
// skipped); the (row, wave) totals are then scanned once to give every wave of every
// row its offset.  lds holds block_scan_lds<Rows>() ints.
template <int Rows, int Block = kScanBlock>
constexpr int block_scan_lds() {
  return Rows * (Block / 64) + (Rows * (Block / 64) + 63) / 64;
}

// One pass of block_scan: v[m] is entry base + m kScanBlock + threadIdx.x (zero past n).
// Stores run + the exclusive prefix of each of the pass's entries below n and returns
// the pass total.
template <int Rows, int Block, typename Store>
__device__ inline int scan_pass(const int (&v)[Rows], int64_t base, int64_t n, int run, Store store, int *lds) {
  constexpr int kW = Block / 64;       // waves
  constexpr int kT = Rows * kW;        // (row, wave) totals per pass
  constexpr int kTW = (kT + 63) / 64;  // waves that scan them
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  {
    int ex[Rows];
#pragma unroll
    for (int m = 0; m < Rows; ++m) {
      int incl = v[m];
      if (base + static_cast<int64_t>(m) * Block < n) {  // wave-uniform
        for (int off = 1; off < 64; off <<= 1) {
          const int y = __shfl_up(incl, off, 64);
          if (lane >= off) incl += y;
        }
      }
      ex[m] = incl - v[m];
      if (lane == 63) lds[m * kW + wave] = incl;
    }
    __syncthreads();
    int tot_all = 0;
    {
      int x = threadIdx.x < kT ? lds[threadIdx.x] : 0;
      int incl = x;
      if (wave < kTW) {
        for (int off = 1; off < 64; off <<= 1) {
          const int y = __shfl_up(incl, off, 64);
          if (lane >= off) incl += y;
        }
      }
      __syncthreads();
      if (threadIdx.x < kT) lds[threadIdx.x] = incl - x;
      if (wave < kTW && lane == 63) lds[kT + wave] = incl;
      __syncthreads();
      int before = 0;
      for (int w = 0; w < kTW; ++w) {
        const int t = lds[kT + w];
        before += w < wave ? t : 0;
        tot_all += t;
      }
      __syncthreads();
      if (threadIdx.x < kT) lds[threadIdx.x] += before;
      __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < Rows; ++m) {
      const int64_t k = base + static_cast<int64_t>(m) * Block + threadIdx.x;
      if (k < n) store(k, run + lds[m * kW + wave] + ex[m]);
    }
    __syncthreads();  // lds is reused by the next pass
    return tot_all;
  }
}

template <int Rows, int Block = kScanBlock, typename Count, typename Store>
__device__ inline void block_scan(Count count, Store store, int64_t n, int *lds) {
  int run = 0;
  for (int64_t base = 0; base < n; base += static_cast<int64_t>(Block) * Rows) {
    int v[Rows];
#pragma unroll
    for (int m = 0; m < Rows; ++m) {
      const int64_t k = base + static_cast<int64_t>(m) * Block + threadIdx.x;
      const int x = count(k < n ? k : n - 1);  // unconditional load, zeroed below
      v[m] = k < n ? x : 0;
    }
    run += scan_pass<Rows, Block>(v, base, n, run, store, lds);
  }
  if (threadIdx.x == 0) store(n, run);
}

// The record of column col for the work-item records: its first cell, its sorted atoms
// [first, end) and cx | cy << 16.
__device__ inline int4 column_info(int c0, int s0, int s1, int col_local, int ny) {
  const int cx = col_local / ny;
  return make_int4(c0, s0, s1, cx | ((col_local - cx * ny) << 16));
}

// Clusters of K atoms in column `col` (ceil of its atom count over K), from cell starts
// held in `cs` (any address space); also stores the column's col_info record.  A single
// system's descriptor is read once.
struct ColumnClusters {
  const SysDesc *desc;
  int4 *info;
  int B, K;
  int cell_begin0, col_begin0, ny0, nz0;
  __device__ ColumnClusters(const Dev &d, int k) : desc(d.desc), info(d.col_info), B(d.B), K(k) {
    cell_begin0 = d.desc[0].cell_begin;
    col_begin0 = d.desc[0].col_begin;
    ny0 = d.desc[0].dims[1];
    nz0 = d.desc[0].dims[2];
  }
  template <typename Starts>
  __device__ int operator()(const Starts &cs, int col) const {
    int cb = cell_begin0, cbeg = col_begin0, ny = ny0, nz = nz0;
    if (B > 1) {
      const SysDesc &sd = desc[column_system(desc, B, col)];
      cb = sd.cell_begin;
      cbeg = sd.col_begin;
      ny = sd.dims[1];
      nz = sd.dims[2];
    }
    const int c0 = cb + (col - cbeg) * nz;
    const int s0 = cs[c0], s1 = cs[c0 + nz];
    info[col] = column_info(c0, s0, s1, col - cbeg, ny);
    return (s1 - s0 + K - 1) / K;
  }
};

// One workgroup: cell_start from the cell counts, then (cluster kernel) the number
// of K-atom clusters of every (x, y) column and their scan.
__global__ void __launch_bounds__(kScanBlock) k_scan(Dev d, int clusters, int K) {
  __shared__ int lds[block_scan_lds<kScanPer>()];
  const int32_t *cnt = d.cell_count;
  int32_t *cstart = d.cell_start;
  block_scan<kScanPer>([cnt](int64_t k) { return static_cast<int>(cnt[k]); },
                       [cstart](int64_t k, int v) { cstart[k] = v; }, d.n_cells, lds);
  if (!clusters) return;
  __syncthreads();  // cell_start is visible to the whole workgroup
  const ColumnClusters cc(d, K);
  const int32_t *cs = d.cell_start;
  int32_t *ccs = d.col_clu_start;
  block_scan<1>([cc, cs](int64_t col) { return cc(cs, static_cast<int>(col)); },
                [ccs](int64_t k, int v) { ccs[k] = v; }, d.n_columns, lds);
}

// Sum of v over the workgroup (kScanBlock threads), returned to every thread.
__device__ inline int block_sum_int(int v, int *lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
  for (int w = 0; w < kScanBlock / 64; ++w) t += lds[w];
  __syncthreads();  // lds may be reused
  return t;
}

// Cell scan of large grids, in two launches without inter-workgroup waiting: each
// workgroup first sums its tile of kScanTileCells counts, then (next launch) adds up
// the totals of the tiles before its own and scans its tile from there.
__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(Dev d) {
  __shared__ int lds[kScanBlock / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTileCells;
  int acc = 0;
#pragma unroll
  for (int m = 0; m < kScanPer; ++m) {
    const int64_t k = base + static_cast<int64_t>(m) * kScanBlock + threadIdx.x;
    acc += k < d.n_cells ? d.cell_count[k] : 0;
  }
  acc = block_sum_int(acc, lds);
  if (threadIdx.x == 0) d.scan_tiles[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(Dev d) {
  __shared__ int lds[block_scan_lds<kScanPer>()];
  int pre = 0;
  for (int t = threadIdx.x; t < static_cast<int>(blockIdx.x); t += kScanBlock) pre += d.scan_tiles[t];
  pre = block_sum_int(pre, lds);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTileCells;
  const int64_t rest = d.n_cells - base;
  const int64_t n = rest < kScanTileCells ? rest : kScanTileCells;
  const bool last = blockIdx.x == gridDim.x - 1;  // writes cell_start[n_cells], the total
  const int32_t *cnt = d.cell_count + base;
  int32_t *cstart = d.cell_start + base;
  block_scan<kScanPer>([cnt](int64_t k) { return static_cast<int>(cnt[k]); },
                       [cstart, pre, n, last](int64_t k, int v) {
                         if (k < n || last) cstart[k] = pre + v;
                       },
                       n, lds);
}

constexpr int kColSysLds = 2048;  // systems whose column ranges the column scan keeps in LDS


// Scatter by arrival slot (large grids).  With the cluster kernel the first
// ceil(n_columns / kBlock) workgroups also write each column's cluster count into
// col_clu_start (k_finalize scans it in place): a column's system is found by a binary
// search over the systems' first columns, held in LDS for up to kColSysLds systems.
__global__ void __launch_bounds__(kBlock) k_scatter(Dev d, int clusters, int K) {
  __shared__ int sys_col[kColSysLds], sys_cell[kColSysLds], sys_ny[kColSysLds], sys_nz[kColSysLds];
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (clusters && static_cast<int64_t>(blockIdx.x) * kBlock < d.n_columns) {  // workgroup-uniform
    const int B = d.B;
    const int col = static_cast<int>(t);
    const bool in = t < d.n_columns;
    int cb, cbeg, ny, nz;
    if (B <= kColSysLds) {
      for (int b = threadIdx.x; b < B; b += kBlock) {
        sys_col[b] = d.desc[b].col_begin;
        sys_cell[b] = d.desc[b].cell_begin;
        sys_ny[b] = d.desc[b].dims[1];
        sys_nz[b] = d.desc[b].dims[2];
      }
      __syncthreads();
      int lo = 0, hi = B - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys_col[mid] <= col) lo = mid; else hi = mid - 1;
      }
      cb = sys_cell[lo];
      cbeg = sys_col[lo];
      ny = sys_ny[lo];
      nz = sys_nz[lo];
    } else {
      const SysDesc &sd = d.desc[in ? column_system(d.desc, B, col) : 0];
      cb = sd.cell_begin;
      cbeg = sd.col_begin;
      ny = sd.dims[1];
      nz = sd.dims[2];
    }
    if (in) {
      const int c0 = cb + (col - cbeg) * nz;
      const int s0 = d.cell_start[c0], s1 = d.cell_start[c0 + nz];
      d.col_clu_start[col] = (s1 - s0 + K - 1) / K;
      d.col_info[col] = column_info(c0, s0, s1, col - cbeg, ny);
    }
  }
  if (t >= d.N) return;
  d.tmp[d.cell_start[d.atom_cell[t]] + d.atom_slot[t]] = static_cast<int32_t>(t);
}

// Work-item records of the clusters that begin or end at sorted atom p (in cell `cell`
// of global column col, system b), once col_info and col_clu_start are complete (M: the
// work-item count): a cluster's first atom writes the record of each of its Q items but
// the last atom's z-cell, which its last atom writes.  The column's and the system's
// loads are issued together.
__device__ inline void item_records(const Dev &d, int p, int cell, int col, int b, int K, int Q, int64_t M) {
  const int4 ci = d.col_info[col];
  const int clu0 = d.col_clu_start[col];
  const SysDesc &sd = d.desc[b];
  const int4 dims = make_int4(sd.dims[0], sd.dims[1], sd.dims[2], sd.reach[0]);
  const int ky = sd.reach[1], kz = sd.reach[2], cell_begin = sd.cell_begin;
  // (the system's values are used below only by a cluster's first atom: this keeps their
  // loads beside the column's instead of after the test)
  asm volatile("" ::"v"(dims.x), "v"(dims.y), "v"(dims.z), "v"(dims.w), "v"(ky), "v"(kz), "v"(cell_begin), "v"(clu0));
  const int j = p - ci.y;
  const bool head = j % K == 0, tail = j % K == K - 1 || p == ci.z - 1;
  if (!head && !tail) return;
  const int I = clu0 + j / K;
  const int z = cell - ci.x;
  for (int q = 0; q < Q; ++q) {
    const int m = I * Q + q;
    ItemRec &r = d.items[item_slot(m, M)];
    if (head) {
      int4 *w = reinterpret_cast<int4 *>(&r);
      w[0] = make_int4(p, ci.z - p < K ? ci.z - p : K, m, b);
      w[1] = make_int4(ci.w & 0xFFFF, ci.w >> 16, z, cell_begin);
      w[2] = dims;
      r.ky = ky;
      r.kz = kz;
    }
    if (tail) r.cz1 = z;
  }
}

// Large grids, cluster kernels: the work-item records, one thread per sorted atom, after
// k_finalize has scanned the column cluster counts.
__global__ void __launch_bounds__(kBlock) k_item_records(Dev d, int K, int Q) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= d.N) return;
  const int64_t M = static_cast<int64_t>(d.col_clu_start[d.n_columns]) * Q;
  const int i = static_cast<int>(d.s_fix[p].w);
  item_records(d, p, d.atom_cell[i], d.atom_col[i], static_cast<int>(d.atom_fix[i].w), K, Q, M);
}

// With col_scan (large grids, cluster kernel) the first workgroup turns the column
// cluster counts written by k_scatter into their exclusive scan, in place, while the
// others place the atoms.  With K > 0 (cluster kernel, column starts complete) every
// atom that begins or ends a cluster also writes the records of its work items.
template <typename Real>
__global__ void __launch_bounds__(kBlock) k_finalize(Dev d, const Real *__restrict__ pos,
                                                    const Real *__restrict__ charge,
                                                    const int32_t *__restrict__ type, double sqrt_ke, int f64,
                                                    int have_range, int col_scan, int K, int Q) {
  if (col_scan && blockIdx.x == 0) {
    __shared__ int lds[block_scan_lds<kScanPer, kBlock>()];
    int32_t *ccs = d.col_clu_start;
    block_scan<kScanPer, kBlock>([ccs](int64_t k) { return static_cast<int>(ccs[k]); },
                                 [ccs](int64_t k, int v) { ccs[k] = v; }, d.n_columns, lds);
    return;
  }
  const int s = (blockIdx.x - col_scan) * kBlock + threadIdx.x;
  if (s >= d.N) return;
  const int i = d.tmp[s];
  const int64_t M = K > 0 ? static_cast<int64_t>(d.col_clu_start[d.n_columns]) * Q : 0;
  // The cell's positions: stored per position by the fused scatter (one load away), or
  // looked up through the atom's cell.  (For large batches the extra scattered store
  // costs more than the two dependent loads it saves.)
  int lo, hi;
  const int cell = (K > 0 || !have_range) ? d.atom_cell[i] : 0;
  const int col = K > 0 ? d.atom_col[i] : 0;
  if (have_range) {
    const int2 cr = d.s_range[s];
    lo = cr.x;
    hi = cr.y;
  } else {
    lo = d.cell_start[cell];
    hi = d.cell_start[cell + 1];
  }
  int rank = 0;
  for (int k = lo; k < hi; ++k) rank += d.tmp[k] < i;
  const int dst = lo + rank;
  const uint4 f = d.atom_fix[i];
  d.s_fix[dst] = make_uint4(f.x, f.y, f.z, static_cast<uint32_t>(i));
  const double q = static_cast<double>(charge[i]);
  if (f64)  // the raw positions are read by the double-precision kernels only
    d.s_pos64[dst] = make_double4(static_cast<double>(pos[3 * static_cast<int64_t>(i)]),
                                  static_cast<double>(pos[3 * static_cast<int64_t>(i) + 1]),
                                  static_cast<double>(pos[3 * static_cast<int64_t>(i) + 2]), q);
  d.s_q32[dst] = static_cast<float>(q * sqrt_ke);
  int t = type[i];
  d.s_type[dst] = (t < 0 || t >= d.T) ? 0 : t;
  if (K > 0) item_records(d, dst, cell, col, static_cast<int>(f.w), K, Q, M);
}

// Scan and scatter in one launch, for grids whose cell counts fit in LDS: every
// workgroup scans all the counts itself (cheaper than a launch of its own at these
// sizes) and places its atoms; workgroup 0 also stores cell_start and the column
// cluster starts.
__global__ void __launch_bounds__(kScanBlock) k_scan_scatter(Dev d, int clusters, int K) {
  extern __shared__ int cs[];  // [n_cells + 1]
  __shared__ int lds[block_scan_lds<kScanPer>()];
  // this workgroup's atoms (one per thread), loaded while the counts are scanned
  const int64_t i = blockIdx.x * static_cast<int64_t>(kScanBlock) + threadIdx.x;
  const bool have = i < d.N;
  const int cell = have ? d.atom_cell[i] : 0;
  const int slot = have ? d.atom_slot[i] : 0;
  const ColumnClusters cc(d, K);
  const int32_t *cnt = d.cell_count;
  int *csl = cs;
  block_scan<kScanPer>([cnt](int64_t k) { return static_cast<int>(cnt[k]); },
                       [csl](int64_t k, int v) { csl[k] = v; }, d.n_cells, lds);
  __syncthreads();
  if (have) {
    d.tmp[cs[cell] + slot] = static_cast<int32_t>(i);
    d.s_range[cs[cell] + slot] = make_int2(cs[cell], cs[cell + 1]);  // for k_finalize, one load away
  }
  // cell_start: each workgroup stores a slice
  const int64_t per = (d.n_cells + 1 + gridDim.x - 1) / gridDim.x;
  const int64_t k0 = per * blockIdx.x, k1 = k0 + per < d.n_cells + 1 ? k0 + per : d.n_cells + 1;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kScanBlock) d.cell_start[k] = cs[k];
  if (clusters && blockIdx.x == gridDim.x - 1) {
    int32_t *ccs = d.col_clu_start;
    block_scan<1>([cc, csl](int64_t col) { return cc(csl, static_cast<int>(col)); },
                  [ccs](int64_t k, int v) { ccs[k] = v; }, d.n_columns, lds);
  }
}

unsigned grid_for(int64_t n, int block) {
  const int64_t g = (n + block - 1) / block;
  return static_cast<unsigned>(g > 0 ? g : 1);
}

}  // namespace

hipError_t launch_build(const Plan &plan, const Dev &d, const nb_system *sys, hipStream_t s) {
  // Descriptors travel as kernel arguments (no host-to-device copy), kDescChunk per launch.
  DescChunk first{};
  first.first = 0;
  first.count = plan.B < kDescChunk ? plan.B : kDescChunk;
  for (int k = 0; k < first.count; ++k) first.d[k] = pack_desc(plan.desc[k]);
  const int64_t init_work = plan.N > plan.n_cells ? plan.N : plan.n_cells;
  unsigned g_init = grid_for(init_work, kBlock);
  if (g_init > 4096) g_init = 4096;
  const int f64 = plan.precision == NB_FP64 ? 1 : 0;
  TableArgs ta{};
  ta.kind = plan.table;
  ta.n = plan.table_n;
  if (plan.table) {
    ta.h = plan.cutoff / plan.table_n;
    ta.beta = plan.beta;
    ta.two_beta_sqrtpi = 2.0 * plan.beta / 1.7724538509055160273;
    ta.short_erfc = plan.beta * plan.cutoff <= kErfcxShortMax ? 1 : 0;
  }
  const int clusters = uses_clusters(plan.kernel) ? 1 : 0;
  const uint32_t cluster_key =
      clusters ? static_cast<uint32_t>(plan.cluster_size) | (static_cast<uint32_t>(plan.split) << 8) : 0u;
  hipLaunchKernelGGL(k_init, dim3(g_init), dim3(kBlock), 0, s, d, first, sys->lj_sigma, sys->lj_eps, plan.kernel, f64,
                     ta, cluster_key);
  for (int b0 = kDescChunk; b0 < plan.B; b0 += kDescChunk) {
    DescChunk c{};
    c.first = b0;
    c.count = plan.B - b0 < kDescChunk ? plan.B - b0 : kDescChunk;
    for (int k = 0; k < c.count; ++k) c.d[k] = pack_desc(plan.desc[b0 + k]);
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, c);
  }
  if (plan.N == 0) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanBlock), 0, s, d, clusters, plan.cluster_size);
    return hipGetLastError();
  }
  const unsigned g = grid_for(plan.N, kBlock);
  if (sys->pos_is_f64)
    hipLaunchKernelGGL(k_bin<double>, dim3(g), dim3(kBlock), 0, s, d, static_cast<const double *>(sys->pos),
                       sys->type, sys->excl_offset, sys->excl_index, sys->pair14_offset, sys->pair14_index);
  else
    hipLaunchKernelGGL(k_bin<float>, dim3(g), dim3(kBlock), 0, s, d, static_cast<const float *>(sys->pos),
                       sys->type, sys->excl_offset, sys->excl_index, sys->pair14_offset, sys->pair14_index);
  if (plan.n_cells + 1 <= kFuseCells) {
    // one workgroup per kScanBlock atoms, and for the cluster kernels one more that scans
    // the column cluster counts (beside the scatter, not after one workgroup's share of it)
    const unsigned gs = grid_for(plan.N, kScanBlock) + (clusters ? 1u : 0u);
    hipLaunchKernelGGL(k_scan_scatter, dim3(gs), dim3(kScanBlock), 4 * static_cast<size_t>(plan.n_cells + 1), s, d,
                       clusters, plan.cluster_size);
  } else {
    const unsigned tiles = static_cast<unsigned>((plan.n_cells + kScanTileCells - 1) / kScanTileCells);
    const unsigned gc = clusters ? grid_for(plan.n_columns, kBlock) : 0;  // column count workgroups
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanBlock), 0, s, d);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(kScanBlock), 0, s, d);
    hipLaunchKernelGGL(k_scatter, dim3(g > gc ? g : gc), dim3(kBlock), 0, s, d, clusters, plan.cluster_size);
  }
  const double sqrt_ke = sqrt(plan.ke);
  const int have_range = plan.n_cells + 1 <= kFuseCells ? 1 : 0;  // written by k_scan_scatter
  const int col_scan = (!have_range && clusters) ? 1 : 0;           // column counts written by k_scatter
  const unsigned gf = g + static_cast<unsigned>(col_scan);
  // work items written by k_finalize when the column starts are complete before it
  const int rec_k = clusters && !col_scan ? plan.cluster_size : 0;
  if (sys->pos_is_f64)
    hipLaunchKernelGGL(k_finalize<double>, dim3(gf), dim3(kBlock), 0, s, d, static_cast<const double *>(sys->pos),
                       static_cast<const double *>(sys->charge), sys->type, sqrt_ke, f64, have_range, col_scan, rec_k,
                       plan.split);
  else
    hipLaunchKernelGGL(k_finalize<float>, dim3(gf), dim3(kBlock), 0, s, d, static_cast<const float *>(sys->pos),
                       static_cast<const float *>(sys->charge), sys->type, sqrt_ke, f64, have_range, col_scan, rec_k,
                       plan.split);
  if (clusters && col_scan)
    hipLaunchKernelGGL(k_item_records, dim3(g), dim3(kBlock), 0, s, d, plan.cluster_size, plan.split);
  return hipGetLastError();
}

}  // namespace nb
