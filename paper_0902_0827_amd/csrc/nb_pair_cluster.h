// Cluster pair kernel: waves own i-clusters of up to K consecutive sorted atoms of
// one (x, y) column (K = 4 or 8); lane = (ii, jj) = (lane / J, lane % J), J = 64 / K.
//
// The paper's kernel (section 3) processes one cell per thread block and stages
// every cell within R into shared memory, one thread per i atom.  Here, for a
// 64-wide wavefront and ~10 atoms per cell, a wave instead owns K i atoms and
// streams the j atoms of the neighbouring columns:
//
//   1. stage: the atoms of each neighbouring column's z-window are read 64 at a
//      time (coalesced; the next chunk's loads are issued before the current one
//      is used), each tested against the i-cluster's bounding box; the survivors
//      (those within R of the box) are compacted, ballot + mbcnt, into a ring
//      buffer in LDS;
//   2. pairs: whenever the ring holds J atoms, each lane evaluates the pair
//      (i atom ii, j atom jj), so all 64 lanes work on candidates that passed the
//      box test (on the 23.6k-atom box about 60% of them are inside R for K = 4,
//      48% for K = 8, against ~25% for a plain cell stencil); a lane without a pair
//      adds zeros, so a group has no branch;
//   3. each row of J lanes accumulates its i atom's sums in registers; rows are
//      reduced with cross-lane shuffles at the end.
//
// Full shell (every pair evaluated from both sides, as in the paper): by default each
// cluster is one work item, and its wave writes the per-atom results in the caller's
// atom order itself.  A cluster's candidates may instead be split over Q work items
// (Q = 2..8): each writes its part of every atom's sums to its own slot, and k_finish
// adds the Q parts in a fixed order and converts them to the caller's atom order.
// k_finish also reduces energies, virials and per-type sums.  Nothing is accumulated
// with atomics: results are deterministic.  The half-shell form (each pair once; the
// mixed path's default for forces and energies) is described with the kernel: its
// candidates' shares go to per-atom accumulators by atomics, in 64-bit fixed point on
// the mixed path so that the sums stay deterministic.
#pragma once

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <utility>

#include "nb_pair_common.h"
#include "nb_pair_math.h"

namespace nb {

namespace {

constexpr int kRing = 128;           // ring buffer of staged j atoms (power of two)
constexpr int kTabLds = 16;          // type tables up to 16 x 16 are copied to LDS
constexpr int kMaxRuns = 2 * 9 * 9;  // up to 9 x 9 neighbour columns, <= 2 z-runs each
constexpr int kRunPad = 4;           // sentinel entries after the last run
// FP64 pair kernels: registers are allocated for 4 resident waves per SIMD (at most
// 128 VGPRs; a few values outside the loops go to scratch); left alone the compiler
// takes 134 and 3 waves fit.
constexpr int kF64WavesPerEu = 4;
// The FP64 half shell with 8-atom clusters has about three items per SIMD on the 23.6k-atom
// box: held to 168 registers (3 waves per SIMD) it does not spill (88.1 against 88.9 us).
constexpr int kF64HalfWavesPerEu = 3;
constexpr int kFinishBlock = 256;
constexpr int kPairs2WavesPerCu = 16;  // 4 SIMDs x 4 resident waves of the two-group kernel
// Exclusion window of one i atom in LDS, one byte per index difference: byte d is 1 when
// j - i = d - 64 is excluded (d = 0..128; d = 64, the atom itself, is 1), and bytes
// 129-131 are 0, so a difference outside the window reads byte 129.
constexpr int kExBytes = 132;
constexpr uint32_t kExClear = 2u * kWindow + 1u;

__device__ __forceinline__ uint32_t uabs_diff(uint32_t a, uint32_t b) {
  const int32_t d = static_cast<int32_t>(a - b);
  return d < 0 ? static_cast<uint32_t>(-static_cast<int64_t>(d)) : static_cast<uint32_t>(d);
}

// Squared distance (A^2, single precision) from a fixed-point point to a box given
// by centre and half extents, with minimum image per dimension.
__device__ __forceinline__ float box_dist2(const uint4 &p, const uint4 &ctr, const uint4 &half, float s2x, float s2y,
                                           float s2z) {
  const uint32_t ax = uabs_diff(p.x, ctr.x), ay = uabs_diff(p.y, ctr.y), az = uabs_diff(p.z, ctr.z);
  // max(a - h, 0): one saturating subtraction each
  const float ex = static_cast<float>(__builtin_elementwise_sub_sat(ax, half.x));
  const float ey = static_cast<float>(__builtin_elementwise_sub_sat(ay, half.y));
  const float ez = static_cast<float>(__builtin_elementwise_sub_sat(az, half.z));
  return fmaf(s2z * ez, ez, fmaf(s2y * ey, ey, s2x * ex * ex));
}

// Wave-uniform copies (scalar registers) of values read from memory.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(b)));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32)));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15) (gfx9 encoding): every vector-memory load
// issued so far has returned.
__device__ __forceinline__ void wait_vm_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Min / max over the rows (lanes J apart) and sum over a row's J lanes.
template <int J>
__device__ __forceinline__ int shfl_rows_min(int v) {
  for (int off = J; off < 64; off <<= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

template <int J>
__device__ __forceinline__ int shfl_rows_max(int v) {
  for (int off = J; off < 64; off <<= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// Cross-lane moves within DPP rows (no LDS): lane l reads lane l ^ 1, l ^ 2, or 7 - (l % 8)
// of its 8-lane half row.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

// Min / max over the K = 4 or 8 lanes of one aligned group of consecutive lanes (the
// rows of the half-shell kernel's lane layout), by DPP moves: after the two quad
// exchanges each lane holds its quad's extreme, and the half-row mirror pairs the two
// quads of an 8-lane group.
template <int K>
__device__ __forceinline__ int shfl_group_min(int v) {
  static_assert(K == 4 || K == 8, "groups of 4 or 8 lanes");
  v = min(v, dpp_i32<kDppXor1>(v));
  v = min(v, dpp_i32<kDppXor2>(v));
  if constexpr (K == 8) v = min(v, dpp_i32<kDppHalfMirror>(v));
  return v;
}

template <int K>
__device__ __forceinline__ int shfl_group_max(int v) {
  static_assert(K == 4 || K == 8, "groups of 4 or 8 lanes");
  v = max(v, dpp_i32<kDppXor1>(v));
  v = max(v, dpp_i32<kDppXor2>(v));
  if constexpr (K == 8) v = max(v, dpp_i32<kDppHalfMirror>(v));
  return v;
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  // every lane of a row reads a lane of its row (full masks), so "old" and bound_ctrl never
  // take effect: with old = 0 and bound_ctrl set the move folds into the addition
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                                     static_cast<unsigned>(lo)));
}
// Sum over each aligned group of K = 4 or 8 consecutive lanes, in every lane of the group,
// by DPP moves (the additions in a fixed order: deterministic).
template <int K, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(K == 4 || K == 8, "groups of 4 or 8 lanes");
  if constexpr (std::is_same_v<T, float>) {
    v += dpp_f32<kDppXor1>(v);
    v += dpp_f32<kDppXor2>(v);
    if constexpr (K == 8) v += dpp_f32<kDppHalfMirror>(v);
  } else {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    if constexpr (K == 8) v += dpp_f64<kDppHalfMirror>(v);
  }
  return v;
}

// 64-bit fixed point of the mixed-path half-shell accumulators: v * 2^32 rounded to the
// nearest integer (|v| < 2^31: forces in kJ/mol/A, energies in kJ/mol).  Integer
// addition is associative, so the accumulated sums do not depend on the order of the
// atomic additions.
constexpr double kFixScale = 4294967296.0;
__device__ __forceinline__ long long to_fixed(double v) {
  const double s = rint(v * kFixScale);
  const double hi = floor(s * (1.0 / kFixScale));
  const double lo = s - hi * kFixScale;  // exact, in [0, 2^32)
  return static_cast<long long>((static_cast<unsigned long long>(static_cast<long long>(static_cast<int>(hi))) << 32) +
                                static_cast<unsigned long long>(static_cast<unsigned>(lo)));
}
__device__ __forceinline__ double from_fixed(long long a) {
  const int hi = static_cast<int>(a >> 32);
  const unsigned lo = static_cast<unsigned>(a);
  return (static_cast<double>(hi) * kFixScale + static_cast<double>(lo)) * (1.0 / kFixScale);
}

// Two limbs for the FP64 path's half-shell accumulators: hi = floor(v 2^32) and lo =
// round((v 2^32 - hi) 2^32) in [0, 2^32], each summed by integer additions, so that
// sum(hi) 2^-32 + sum(lo) 2^-64 is the sum of the v to within 2^-64 per term (far below
// FP64 rounding of forces of order 1) whatever the order of the additions.
__device__ __forceinline__ void to_fixed2(double v, long long &hi, long long &lo) {
  const double t = v * kFixScale;  // exact
  const double th = floor(t);
  lo = static_cast<long long>(rint((t - th) * kFixScale));
  const double h = floor(th * (1.0 / kFixScale));
  const double l = th - h * kFixScale;  // exact, in [0, 2^32)
  hi = static_cast<long long>((static_cast<unsigned long long>(static_cast<long long>(static_cast<int>(h))) << 32) +
                              static_cast<unsigned long long>(static_cast<unsigned>(l)));
}
__device__ __forceinline__ double from_fixed2(long long hi, long long lo) {
  return from_fixed(hi) + static_cast<double>(lo) * (1.0 / (kFixScale * kFixScale));
}

// One step of reduce_scatter below at lane offset OFF, N values still carried.
template <int OFF, int N, int NV>
__device__ __forceinline__ double reduce_scatter_step(double (&v)[NV], int lane) {
  if constexpr (N > 1) {
    constexpr int h = N / 2;
    const bool up = (lane & OFF) != 0;
#pragma unroll
    for (int k = 0; k < h; ++k) {
      const double keep = up ? v[h + k] : v[k];
      const double give = up ? v[k] : v[h + k];
      v[k] = keep + __shfl_xor(give, OFF, 64);
    }
    return reduce_scatter_step<OFF / 2, h, NV>(v, lane);
  } else if constexpr (OFF > 0) {
    v[0] += __shfl_xor(v[0], OFF, 64);
    return reduce_scatter_step<OFF / 2, 1, NV>(v, lane);
  } else {
    return v[0];
  }
}

// Sums of NV values over each aligned group of G lanes (NV and G powers of two, NV <= G),
// each sum ending in its own lanes: lane l returns the group's sum of value
// (l % G) / (G / NV).  The first log2(NV) butterfly steps halve the values a lane
// carries (it keeps the half its lane bit selects and hands the other half to its
// partner), the rest are plain butterfly steps: NV - 1 + log2(G / NV) shuffles instead
// of NV log2(G).  The order of the additions is fixed, so the sums are deterministic.
template <int G, int NV>
__device__ __forceinline__ double reduce_scatter(const double (&in)[NV], int lane_in) {
  static_assert((NV & (NV - 1)) == 0 && (G & (G - 1)) == 0 && NV <= G, "powers of two");
  // The lane index is taken anew here, so that the compiler does not hoist the lane
  // masks out of the enclosing loops and keep them in registers all along.
  int lane = lane_in;
  asm volatile("" : "+v"(lane));
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = in[k];
  return reduce_scatter_step<G / 2, NV, NV>(v, lane);
}

// Index of the last column whose first cluster is <= k: a 64-way search, each lane
// probing one position per round (two or three rounds for any practical grid).
__device__ __forceinline__ int cluster_column(const int32_t *__restrict__ col_clu_start, int n_columns, int k) {
  int lo = 0, hi = n_columns - 1;  // answer in [lo, hi]
  const int lane = threadIdx.x & 63;
  while (hi > lo) {
    const int span = hi - lo + 1;
    const int step = (span + 63) >> 6;
    const int probe = lo + lane * step;
    const bool le = probe <= hi && col_clu_start[probe] <= k;
    const uint64_t m = __ballot(le);
    const int last = 63 - __clzll(static_cast<long long>(m));  // lane 0 always passes
    lo = lo + last * step;
    const int nhi = lo + step - 1;
    hi = nhi < hi ? nhi : hi;
  }
  return lo;
}

template <bool F64, bool FF>
struct WaveLds;

// One staged j atom of the mixed-precision kernel (one 32-byte slot, so that a group
// reads it at one address plus offsets).
struct alignas(16) RingF32 {
  uint4 fix;   // fixed-point x, y, z, original index
  float2 qt;   // q * sqrt(k_e), type (as int bits)
  int2 sidx;   // sorted index (half-shell kernel), unused
};

// Row windows of the i atoms: byte d of row ii describes j - i = d - 64: bit 0 excluded,
// bit 1 a scaled 1-4 pair (FF variants).
template <bool FF>
struct WaveLds<false, FF> {
  RingF32 ring[kRing];
  int2 runs[kMaxRuns + kRunPad];  // non-empty candidate runs: (first sorted atom, first candidate position)
  uint32_t exw[8 * kExBytes / 4];  // exclusion window of each row's i atom, bytes
};

template <>
struct WaveLds<true, false> {
  double4 pos[kRing];  // x, y, z, q
  int4 meta[kRing];    // original index, type, sorted index (half-shell kernel), unused
  int2 runs[kMaxRuns + kRunPad];  // non-empty candidate runs: (first sorted atom, first candidate position)
};

template <>
struct WaveLds<true, true> {  // the FP64 FF variants read their windows from LDS as well
  double4 pos[kRing];
  int4 meta[kRing];
  int2 runs[kMaxRuns + kRunPad];
  uint32_t exw[8 * kExBytes / 4];
};

// Type-pair table entry of each precision; the table is copied into dynamic LDS sized
// for the system's own type count (T x T entries).
template <bool F64>
using TypePairT = std::conditional_t<F64, TypePair64, TypePair32>;

// The entry as held in LDS: the FP64 path needs only c6 and c12 (and 1/sigma in the
// adjoint), 16 or 24 bytes instead of 32, which lets one more wave per CU be resident
// (the LDS, not the registers, limits that kernel).
struct TypePairF64Adj { double c6, c12, inv_sig; };
template <bool F64, int MODE>
using TypePairLds = std::conditional_t<!F64, TypePairT<F64>,
                                       std::conditional_t<MODE == kAdjoint || MODE == kVJP, TypePairF64Adj, double2>>;

template <bool F64, int MODE>
constexpr size_t tab_lds_bytes(int T) {
  return static_cast<size_t>(T) * static_cast<size_t>(T) * sizeof(TypePairLds<F64, MODE>);
}

// Half-shell kernel: the candidates' shares of one item wait in LDS (after the type
// table) and go to the accumulators by atomics when the stage is full and at the end
// of the item.  (A global write in flight makes every later wait for the prefetched
// candidates a wait for all outstanding memory operations, so none is issued inside
// the candidate loop.)  Sizes keep 20 one-wave workgroups (mixed) or 16 (FP64) per CU
// within the 160 KB of LDS.
struct alignas(16) StageF32 { float x, y, z; int s; };
struct alignas(16) StageF64 { double x, y, z; int s, pad; };
template <bool F64>
using StageT = std::conditional_t<F64, StageF64, StageF32>;
template <bool F64>
constexpr int kStage = F64 ? 64 : 144;  // entries, multiples of 16

template <bool F64, int MODE, bool TABLDS, bool HALF>
constexpr size_t dyn_lds_bytes(int T) {
  return (TABLDS ? tab_lds_bytes<F64, MODE>(T) : 0) + (HALF ? kStage<F64> * sizeof(StageT<F64>) : 0);
}

// Orders this wave's LDS accesses (one wave's LDS operations execute in issue order;
// this only stops the compiler from moving them across the point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Accelerator complex die (XCD) of the executing wave, from the XCC_ID hardware
// register; only used to pick a work queue, so any value is correct.
__device__ __forceinline__ int xcd_id() {
  return static_cast<int>(__builtin_amdgcn_s_getreg((20) | (0 << 6) | (15 << 11))) & (kXcds - 1);
}

// A work item's record, read through the constant address space: the kernel never writes
// the records, and wave-uniform loads from it are scalar loads into scalar registers.
__device__ __forceinline__ ItemRec load_item(const ItemRec *items, int slot) {
  using ConstInt = const __attribute__((address_space(4))) int32_t;
  ConstInt *q = (ConstInt *)(items + slot);
  ItemRec r;
  r.first = q[0], r.count = q[1], r.item = q[2], r.sys = q[3];
  r.cx = q[4], r.cy = q[5], r.cz0 = q[6], r.cell_begin = q[7];
  r.nx = q[8], r.ny = q[9], r.nz = q[10], r.kx = q[11];
  r.ky = q[12], r.kz = q[13], r.cz1 = q[14], r.pad = 0;
  return r;
}

// Work item m = (cluster m / Q, part m % Q): part q evaluates the cluster's i atoms
// against the q-th of Q equal shares of its candidate j atoms (the atoms of the
// neighbouring columns' z-windows, in run order).  Items of one cluster are
// consecutive, and the clusters of one (x, y) column are consecutive, so that a range
// of items is a compact region of space.
//
// The items are cut into 8 contiguous ranges, one per XCD (workgroups are dealt to
// the XCDs round robin, and each XCD has its own L2).  Every wave (one per workgroup)
// first takes one item of its XCD's range by its workgroup index: the build has written
// each launch slot's item record (first atom, atom count, column, z-cells, the system's
// grid), so that a wave starts with one scalar load instead of searching the columns
// and the cell starts for its cluster.  With the static schedule the grid covers every
// item and that is all.  With the dynamic schedule the
// grid is what fits on the GPU at once and each range continues through an atomic
// counter: a wave that finishes takes the next item of its own XCD's range, requested
// while the previous item is evaluated, and once that range is exhausted the next
// item of another XCD's range, so that the load evens out however the item costs
// vary.  Each item writes its own output slots: the result does not depend on which
// wave took which item.
//
// HALF (forces and energy only): each pair is evaluated once.  A cluster takes the
// columns of half of its stencil (positive offsets; see the run list below) and, in
// its own column, the atoms from its own first atom on, counting a pair of its own
// atoms only with j after i in sorted order.  A candidate's K rows sit in K consecutive
// lanes: every group sums the forces on its J candidates over the rows by DPP moves,
// row 0 stages the sums in LDS, and full stages go to the candidates' accumulators by
// atomic additions, consecutive sorted atoms in consecutive lanes (so that they
// coalesce); the rows' own sums go there too at the end of the item, and the finishing
// pass copies the accumulators out.  The pair work halves.  The accumulators are 64-bit
// fixed point (two limbs on the FP64 path), so the result is bitwise reproducible
// whatever the order of the additions.
//
// PAIRS2 (mixed path): the group loop takes two groups per pass, which needs more
// registers (held to 128, 4 resident waves per SIMD instead of 5); the launcher uses it
// when every item fits on the GPU at once at that occupancy.
// Variants of the pair evaluation (template parameter VAR).
constexpr int kVarPlain = 0;  // direct evaluation
constexpr int kVarFF = 1;     // direct, with the LJ switch and scaled 1-4 pairs
constexpr int kVarLin = 2;    // radial terms linearly interpolated from tables (mixed forces / energy)
constexpr int kVarCub = 3;    // radial terms from cubic Hermite tables (mixed forces / energy)

template <bool F64, int MODE, bool TABLDS, int K, bool HALF, bool PAIRS2, int VAR>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((F64 && HALF && K == 8) ? kF64HalfWavesPerEu : (F64 || PAIRS2) ? kF64WavesPerEu : 1, 8)))
k_pair_cluster(Dev d, Consts c, Out o, int Q, int dynamic) {
  // Products are fused into additions only within one expression (the explicit FMAs
  // aside), so that the copies of the group loop, and the instantiations with one or two
  // groups per pass, round every sum alike: the schedules give bitwise equal results.
#pragma clang fp contract(on)
  constexpr int J = 64 / K;  // j atoms per group (lanes per row)
  extern __shared__ uint4 tab_lds[];  // [T * T] type pairs when TABLDS, then the stage when HALF
  constexpr bool FF = VAR == kVarFF;
  constexpr int TAB = VAR == kVarLin ? 1 : VAR == kVarCub ? 2 : 0;
  // the adjoint and the force VJP share the per-atom dE/dq-like row sum and the per-type sums
  constexpr bool ADJ = MODE == kAdjoint || MODE == kVJP;
  static_assert(!(HALF && ADJ), "the adjoint and the force VJP are full-shell");
  // force VJP: each staged candidate's v_j (sorted copy), beside the ring
  __shared__ std::conditional_t<MODE == kVJP, std::conditional_t<F64, double4, float4>, int> VJ[MODE == kVJP ? kRing : 1];
  static_assert(TAB == 0 || (!F64 && MODE != kAdjoint), "tables: mixed forces and energies only");
  __shared__ WaveLds<F64, FF> L;
  TypePairLds<F64, MODE> *const TL = reinterpret_cast<TypePairLds<F64, MODE> *>(tab_lds);
  const int lane = static_cast<int>(threadIdx.x);
  // Every wave first takes the item of its own launch slot (the build wrote each slot's
  // record).  The record is loaded together with the build check's status words: the
  // launch never has more workgroups than the workspace has slots, so the load stays
  // inside the workspace whatever it holds, and a failed check discards it.
  int islot = static_cast<int>(blockIdx.x);
  ItemRec rec = load_item(d.items, islot);
  const bool built = built_for(d.status, d.N, true, F64, HALF, static_cast<uint32_t>(K) | (static_cast<uint32_t>(Q) << 8));
  // (held before the branch: otherwise the record's loads are sunk below it and wait for the check)
  asm volatile("" ::"s"(rec.first), "s"(rec.count), "s"(rec.item), "s"(rec.sys), "s"(rec.cx), "s"(rec.cy),
               "s"(rec.cz0), "s"(rec.cell_begin), "s"(rec.nx), "s"(rec.ny), "s"(rec.nz), "s"(rec.kx), "s"(rec.ky),
               "s"(rec.kz), "s"(rec.cz1));
  if (!built) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(d.status, NB_STATUS_NOT_BUILT);
    return;
  }
  // Lane = (i row ii, candidate jj).  Full shell: rows of J consecutive lanes, so that an
  // atom's sums stay in its row.  Half shell: the K rows of one candidate in K consecutive
  // lanes, so that the candidate's shares are summed by DPP moves within a DPP row.
  const int ii = HALF ? lane % K : lane / J, jj = HALF ? lane / K : lane % J;
  const int T = d.T;
  StageT<F64> *const ST = reinterpret_cast<StageT<F64> *>(reinterpret_cast<char *>(tab_lds) +
                                                          (TABLDS ? tab_lds_bytes<F64, MODE>(T) : 0));
  // Ring slots are read by every lane of a group, also those past the candidates it holds
  // (their results are discarded): zeroed once, every slot holds a valid type index.
  for (int k = lane; k < kRing; k += 64) {
    if constexpr (F64) {
      L.pos[k] = make_double4(0, 0, 0, 0);
      L.meta[k] = make_int4(0, 0, 0, 0);
    } else {
      L.ring[k].fix = make_uint4(0u, 0u, 0u, 0u);
      L.ring[k].qt = make_float2(0.f, 0.f);
      L.ring[k].sidx = make_int2(0, 0);
    }
  }
  if constexpr (TABLDS) {
    for (int k = lane; k < T * T; k += 64) {
      if constexpr (F64 && !ADJ) TL[k] = make_double2(d.tab64[k].c6, d.tab64[k].c12);
      else if constexpr (F64) TL[k] = TypePairF64Adj{d.tab64[k].c6, d.tab64[k].c12, d.tab64[k].inv_sig};
      else TL[k] = d.tab32[k];
    }
    wave_lds_sync();
  }
  // The dynamic schedule continues through the counters, and only it needs the item count M.
  const int64_t M = dynamic ? static_cast<int64_t>(uni(d.col_clu_start[d.n_columns])) * Q : 0;
  auto range_lo = [M](int x) { return xcd_range_lo(M, x); };
  const int per = static_cast<int>(gridDim.x) / kXcds;  // static items per range (grid: multiple of 8)

  // Dynamic items: queue x hands out item range_lo(x) + per + counter_x, slot 8 (per + counter_x) + x.
  const int home = dynamic ? xcd_id() : 0;
  uint32_t closed = 0xFFu;  // queues known to be exhausted (wave-uniform bit mask)
  if (dynamic) {
    closed = 0u;
    for (int x = 0; x < kXcds; ++x)  // ranges the static round covers entirely have no dynamic items
      if (range_lo(x) + per >= range_lo(x + 1)) closed |= 1u << x;
  }
  auto request = [&](int x) -> uint32_t {
    uint32_t got = 0;
    if (lane == 0) got = atomicAdd(&d.queue[x * kQueueStride], 1u);
    return got;
  };
  auto slot_of = [&](int x, uint32_t got) -> int {
    const int g = uni(static_cast<int>(got));
    const int k = per + g;
    return (g >= 0 && range_lo(x) + k < range_lo(x + 1)) ? kXcds * k + x : -1;
  };
  // Next item once the speculative request on the home queue has failed: probe every
  // counter (one load per lane), mark the exhausted ones, request from the nearest open
  // queue.  Each round returns an item or closes at least one queue: at most 8 rounds.
  auto steal = [&]() -> int {
    while (closed != 0xFFu) {
      uint32_t v = 0;
      if (lane < kXcds) v = __hip_atomic_load(&d.queue[lane * kQueueStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool open = lane < kXcds && range_lo(lane) + per + static_cast<int>(v) < range_lo(lane + 1);
      closed |= static_cast<uint32_t>(~__ballot(open)) & 0xFFu;
      if (closed == 0xFFu) break;
      int x = home;
      while (closed & (1u << x)) x = (x + 1) & (kXcds - 1);
      const int it = slot_of(x, request(x));
      if (it >= 0) return it;
      closed |= 1u << x;
    }
    return -1;
  };
  uint32_t pending = 0;
  bool have_pending = false;

  for (;;) {
    // The item: its cluster is K consecutive sorted atoms of one column from `first` on
    // (count of them), its share part of Q of their candidates.
    int count = uni(rec.count), m = uni(rec.item), sys = uni(rec.sys), first = uni(rec.first);
    if (count == 0) break;  // a slot without an item (the last ones of a range)
    // (Q is uniform; with one item per cluster the division below is skipped)
    const int part = Q == 1 ? 0 : m - (m / Q) * Q;
    // Per-system constants by scalar loads (the descriptors do not change during the
    // launch): nothing in the pair loop below then waits on a vector-memory load (so the
    // next chunk's loads stay in flight), and the set-up's vector loads are not held up
    // by them.
    using ConstDesc = const __attribute__((address_space(4))) SysDesc;
    ConstDesc *sd = (ConstDesc *)(d.desc + sys);
    const float s2x = sd->scale2f[0], s2y = sd->scale2f[1], s2z = sd->scale2f[2];
    const double bxx = sd->box[0], bxy = sd->box[1], bxz = sd->box[2];
    const double ibx = sd->inv_box[0], iby = sd->inv_box[1], ibz = sd->inv_box[2];
    const int atom_begin = sd->atom_begin;
    const int nx = uni(rec.nx), ny = uni(rec.ny), nz = uni(rec.nz);
    const int cell_begin = uni(rec.cell_begin);
    const int i = first + ii;
    const bool ivalid = ii < count;
    const int ia = ivalid ? i : first;
    const uint4 fi = d.s_fix[ia];
    const int ti = d.s_type[ia];
    double4 pi64 = make_double4(0, 0, 0, 0);
    float qi32 = 0.f;
    if constexpr (F64) pi64 = d.s_pos64[ia];
    else qi32 = d.s_q32[ia];
    const double qi64 = F64 ? pi64.w * c.ke : 0.0;
    // force VJP: the row atom's v (sorted copy; mixed path in fixed-point units)
    double4 vi64 = make_double4(0, 0, 0, 0);
    float4 vi32 = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (MODE == kVJP) {
      vi64 = d.vsort[ia];
      vi32 = make_float4(static_cast<float>(vi64.x), static_cast<float>(vi64.y), static_cast<float>(vi64.z), 0.f);
    }

    // the column, and the z-cells of the cluster's first and last atom
    const int kx = uni(rec.kx), ky = uni(rec.ky), kz = uni(rec.kz);
    const int cx = uni(rec.cx), cy = uni(rec.cy), cz0 = uni(rec.cz0), cz1 = uni(rec.cz1);
    const bool allx = 2 * kx + 1 >= nx, ally = 2 * ky + 1 >= ny;
    const bool allz = (cz1 - cz0) + 2 * kz + 1 >= nz;
    const int xn = allx ? nx : 2 * kx + 1, yn = ally ? ny : 2 * ky + 1;

    // Neighbour-column windows as runs [a0, a1) of sorted atoms (a z-window that wraps
    // around the box is two runs), listed without the empty ones as (a0, position of
    // a0 among all candidates) in LDS.  Candidate p then lies in the run r with
    // runs[r].y <= p < runs[r + 1].y, at sorted index runs[r].x + p - runs[r].y.
    const int ncol = xn * yn;
    int nrun = 0, total = 0;  // wave-uniform
    wave_lds_sync();  // the previous item's reads of the runs and windows are complete
    for (int k0 = 0; k0 < ncol; k0 += 64) {
      const int k = k0 + lane;
      int2 r0 = make_int2(0, 0), r1 = make_int2(0, 0);
      if (k < ncol) {
        const int ox = k / yn, oy = k - (k / yn) * yn;
        int x = allx ? ox : cx - kx + ox;
        x += x < 0 ? nx : (x >= nx ? -nx : 0);
        int y = ally ? oy : cy - ky + oy;
        y += y < 0 ? ny : (y >= ny ? -ny : 0);
        const int cb = cell_begin + (x * ny + y) * nz;
        // The window's cell starts, [a0, a1) and, where it wraps, [b0, b1): the indices are
        // chosen first and the four loads issued together, in one round with the row atoms'
        // loads (b0 = b1 = cb when there is one run).
        int a0 = cb, a1 = cb + nz, b0 = cb, b1 = cb;
        bool two = false;
        if (!allz) {
          const int z0 = cz0 - kz, z1 = cz1 + kz + 1;  // [z0, z1)
          if (z0 < 0) {
            a0 = cb + z0 + nz, b1 = cb + z1, two = true;
          } else if (z1 > nz) {
            a0 = cb + z0, b1 = cb + z1 - nz, two = true;
          } else {
            a0 = cb + z0, a1 = cb + z1;
          }
        }
        r0 = make_int2(d.cell_start[a0], d.cell_start[a1]);
        const int2 rb = make_int2(d.cell_start[b0], d.cell_start[b1]);
        if (two) r1 = rb;
      }
      if constexpr (HALF) {
        // Half stencil: a neighbour column is taken when its offset is positive in x,
        // or zero in x and positive in y (the opposite column takes the pair the other
        // way round, so every pair of columns is visited once and every cluster gets a
        // like share).  Where the stencil spans the whole box in a dimension offsets are
        // ambiguous and the column order decides instead; the own column is taken from
        // the cluster's first atom on.
        if (k < ncol) {
          const int ox = k / yn, oy = k - (k / yn) * yn;
          const int rx = allx ? (ox > cx) - (ox < cx) : (ox > kx) - (ox < kx);
          const int ry = ally ? (oy > cy) - (oy < cy) : (oy > ky) - (oy < ky);
          if (rx < 0 || (rx == 0 && ry < 0)) {
            r0 = r1 = make_int2(0, 0);
          } else if (rx == 0 && ry == 0) {
            r0.x = r0.x > first ? r0.x : first;
            r1.x = r1.x > first ? r1.x : first;
            if (r0.y < r0.x) r0.y = r0.x;
            if (r1.y < r1.x) r1.y = r1.x;
          }
        }
      }
      const int n0 = r0.y - r0.x, n1 = r1.y - r1.x;
      int cnt_tot, len_tot;
      const int slot = nrun + wave_excl_scan_int((n0 > 0) + (n1 > 0), &cnt_tot);
      const int pos = total + wave_excl_scan_int(n0 + n1, &len_tot);
      if (n0 > 0) L.runs[slot] = make_int2(r0.x, pos);
      if (n1 > 0) L.runs[slot + (n0 > 0)] = make_int2(r1.x, pos + n0);
      nrun += cnt_tot;
      total += len_tot;
    }
    if (lane < kRunPad) L.runs[nrun + lane] = make_int2(0, total);  // sentinels
    // This item's share of the candidates, [lo_c, hi_c).
    const int lo_c = Q == 1 ? 0 : static_cast<int>((static_cast<int64_t>(total) * part) / Q);
    const int hi_c = Q == 1 ? total : static_cast<int>((static_cast<int64_t>(total) * (part + 1)) / Q);
    wave_lds_sync();  // the runs are visible to every lane

    // The row atom's exclusion windows, by its original index, are loaded once the runs are
    // built (with the first candidates below, in one round of loads).
    const int oi = static_cast<int>(fi.w);
    // Mixed path: the window byte of candidate oj is oj - oi_lo (unsigned, clamped) in row
    // ii's window in LDS.  FP64 path: the mask stays in registers (LDS there is what limits
    // the resident waves).
    const uint32_t oi_lo = static_cast<uint32_t>(oi) - static_cast<uint32_t>(kWindow);
    const uint8_t *ex_row = nullptr;
    if constexpr (!F64 || FF) ex_row = reinterpret_cast<const uint8_t *>(L.exw) + ii * kExBytes;
    const uint4 mask_i = d.excl_mask[oi];
    uint4 mask14_i = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (FF) {
      if (d.p14_mask) mask14_i = d.p14_mask[oi];
    }
    const uint64_t mask_lo = (static_cast<uint64_t>(mask_i.y) << 32) | mask_i.x;
    const uint64_t mask_hi = (static_cast<uint64_t>(mask_i.w) << 32) | mask_i.z;
    const bool far_i = d.excl_far[oi] != 0u;
    bool any_far = false;  // (set below, once the first candidates' loads are issued)

    uint4 ctr, half;  // the cluster's bounding box (below)

    // Per-lane sums for row ii's atom: force, energy (or dE/dq) and the per-type adjoint
    // sums in double for both paths (the mixed path adds each pair's single-precision
    // terms to them).  The virial: double on the FP64 path; on the mixed path single
    // precision over this item (one lane sees every J-th candidate of the item: a few
    // dozen pairs in practice), converted to double for the wave and system reductions.
    double fx = 0, fy = 0, fz = 0, en = 0, wxx = 0, wxy = 0, wxz = 0, wyy = 0, wyz = 0, wzz = 0;
    double phi = 0, asig = 0, beps = 0;
    float swxx = 0, swxy = 0, swxz = 0, swyy = 0, swyz = 0, swzz = 0;
    // a virial accumulator as double: the FP64 path's own, or the mixed path's single-precision one
    auto D = [&](double dv, float fv) -> double {
      if constexpr (F64) return dv;
      else return static_cast<double>(fv);
    };

    uint32_t head = 0, tail = 0;  // wave-uniform ring positions

    // Mixed path: fixed-point units -> Angstrom, and phi carries one sqrt(k_e) from q'_j.
    const double scx = F64 ? 1.0 : sd->scale[0], scy = F64 ? 1.0 : sd->scale[1], scz = F64 ? 1.0 : sd->scale[2];

    // Half-shell stage: entries [0, nst) hold candidates' shares not yet added.
    int nst = 0;  // wave-uniform
    // Adds v to component c (0-2 force, 3 energy share) of sorted atom a's half-shell
    // accumulator: 64-bit fixed point, in two limbs on the FP64 path.
    auto acc_add = [&](int c, int a, double v) {
      if constexpr (F64) {
        long long hi, lo;
        to_fixed2(v, hi, lo);
        const int64_t at = static_cast<int64_t>(c) * d.N + a;
        __hip_atomic_fetch_add(&d.jacc_fix[at], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&d.jacc_lo[at], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_fetch_add(&d.jacc_fix[static_cast<int64_t>(c) * d.N + a], to_fixed(v), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    };
    auto flush = [&]() {
      wave_lds_sync();
      for (int e = lane; e < nst; e += 64) {
        const StageT<F64> st = ST[e];
        if constexpr (MODE == kForces) {
          if (st.x != 0 || st.y != 0 || st.z != 0) {  // a candidate without a pair in range adds nothing
            acc_add(0, st.s, static_cast<double>(st.x) * -scx);  // staged: the rows' sums (plus sign)
            acc_add(1, st.s, static_cast<double>(st.y) * -scy);
            acc_add(2, st.s, static_cast<double>(st.z) * -scz);
          }
        } else if (st.x != 0) {
          acc_add(3, st.s, static_cast<double>(st.x));
        }
      }
      wave_lds_sync();
      nst = 0;
    };

    // Evaluate pair (row ii's atom, ring entry head + jj) for navail <= J entries.
    // FAR and VIR: the cluster may have far exclusions, the virial may be wanted (both
    // then tested at run time).  The two-group loop has a copy for each combination, so
    // that a pair of groups of the common case is one basic block.
    // CHECK: test the half-shell stage's room for this group (false: the caller made room
    // for it beforehand, so that two groups in a row form one basic block).
    auto process_group = [&](int navail, auto far_c, auto vir_c, auto check_c) {
      constexpr bool FAR = decltype(far_c)::value;
      constexpr bool VIR = decltype(vir_c)::value;
      // head is a multiple of J (only an item's last group is partial) and J divides
      // kRing, so the group's J slots are consecutive: a scalar base plus jj.
      const int slot = static_cast<int>(head & (kRing - 1)) + jj;
      const bool jv = jj < navail;
      int oj, tj, sj = 0;
      if constexpr (F64) {
        const int4 mt = L.meta[slot];
        oj = mt.x;
        tj = mt.y;
        if constexpr (HALF) sj = mt.z;
      } else {
        oj = static_cast<int>(L.ring[slot].fix.w);
        tj = __float_as_int(L.ring[slot].qt.y);
        if constexpr (HALF) sj = L.ring[slot].sidx.x;
      }
      // Exclusions (and j = i): bit (oj - oi) + 64 of row ii's window (bits 0-63 of the
      // mask are oj - oi = -64..-1, bits 64-127 are 1..64); a difference outside the window
      // is not excluded here.  Mixed path: one byte of the window in LDS, read ahead of the
      // distance.  FP64 path: selected from the mask in registers.
      uint32_t exb;
      bool outside;
      if constexpr (F64 && !FF) {
        const int delta = oj - oi;
        outside = static_cast<uint32_t>(delta + kWindow) > 2u * kWindow;
        const uint64_t wbits = delta < 0 ? mask_lo : mask_hi;
        const int wb = delta < 0 ? delta + kWindow : delta - 1;
        exb = (static_cast<uint32_t>(wbits >> (wb & 63)) & (outside ? 0u : 1u)) | (delta == 0 ? 1u : 0u);
      } else {
        const uint32_t dw = min(static_cast<uint32_t>(oj) - oi_lo, kExClear);
        outside = dw == kExClear;
        exb = ex_row[dw];
      }
      // type pair of (ti, tj), read with the window for every lane
      TypePairT<F64> tp;
      if constexpr (TABLDS && F64 && !ADJ) {
        const double2 e = TL[ti * T + tj];
        tp.c6 = e.x;
        tp.c12 = e.y;
      } else if constexpr (TABLDS && F64) {
        const TypePairF64Adj e = TL[ti * T + tj];
        tp.c6 = e.c6;
        tp.c12 = e.c12;
        tp.inv_sig = e.inv_sig;
      } else if constexpr (TABLDS) tp = TL[ti * T + tj];
      else if constexpr (F64) tp = d.tab64[ti * T + tj];
      else tp = d.tab32[ti * T + tj];
      // Once (half shell): candidates before the cluster in sorted order come from other
      // columns and always count; from the cluster on (its own column) only those after i.
      // Both ways, j = i is the window's self bit.
      const bool other = HALF ? (sj < first || sj > i) : true;
      bool hit;
      float r2f = 0.f, dxf = 0.f, dyf = 0.f, dzf = 0.f;
      double r2d = 0.0, dxd = 0.0, dyd = 0.0, dzd = 0.0;
      double4 pj64;
      float qj = 0.f;
      if constexpr (F64) {
        pj64 = L.pos[slot];
        dxd = pi64.x - pj64.x;
        dyd = pi64.y - pj64.y;
        dzd = pi64.z - pj64.z;
        dxd -= bxx * rint(dxd * ibx);
        dyd -= bxy * rint(dyd * iby);
        dzd -= bxz * rint(dzd * ibz);
        r2d = dxd * dxd + dyd * dyd + dzd * dzd;
        hit = ivalid & jv & (r2d < c.rc2) & other;
      } else {
        const uint4 fj = L.ring[slot].fix;
        qj = L.ring[slot].qt.x;
        dxf = static_cast<float>(static_cast<int>(fi.x - fj.x));
        dyf = static_cast<float>(static_cast<int>(fi.y - fj.y));
        dzf = static_cast<float>(static_cast<int>(fi.z - fj.z));
        r2f = fmaf(s2z * dzf, dzf, fmaf(s2y * dyf, dyf, s2x * dxf * dxf));
        hit = ivalid & jv & (r2f < c.rc2f) & other;
      }
      // FF variants: bit 0 of the window byte excludes, bit 1 marks a scaled 1-4 pair
      float wljf = 1.f, wcf = 1.f;
      double wljd = 1.0, wcd = 1.0;
      if constexpr (FF) {
        hit = hit & ((exb & 1u) == 0u);
        const bool scaled = (exb & 2u) != 0u;
        if constexpr (F64) {
          wljd = scaled ? c.s14_lj : 1.0;
          wcd = scaled ? c.s14_c : 1.0;
        } else {
          wljf = scaled ? c.s14_ljf : 1.f;
          wcf = scaled ? c.s14_cf : 1.f;
        }
      } else {
        hit = hit & (exb == 0u);
      }
      // Pairs farther apart than the window only for atoms that carry the far flag.
      if (FAR && any_far) {  // wave-uniform: some atom of this cluster has an exclusion beyond the window
        const bool far_check = hit && outside && far_i;
        if (far_check && far_excluded(oi, oj, atom_begin, d.excl_far, o.excl_off, o.excl_idx)) hit = false;
      }
      // the pair's force on i (f d_ij) and energy, for the half-shell j-side sums
      std::conditional_t<F64, double, float> hgx = 0, hgy = 0, hgz = 0, hu = 0;
      // Every lane evaluates its pair and a lane without one adds zeros (its terms, possibly
      // not finite, are selected away), so the group runs without a branch.
      if constexpr (MODE == kVJP) {
        // force VJP: (v_i - v_j) . d_ij times the parameter derivatives of the force factor
        if constexpr (F64) {
          const double4 vjv = VJ[slot];
          const double wv = (vi64.x - vjv.x) * dxd + (vi64.y - vjv.y) * dyd + (vi64.z - vjv.z) * dzd;
          const PairVjpF64 p = pair_vjp_f64(r2d, tp.c6, tp.c12, wljd, wcd, c.beta, c.two_beta_sqrtpi,
                                            c.erfc_short != 0, c.sw_on2, c.sw_inv);
          const double tq = pj64.w * p.gc * wv, ts = p.dflj * tp.inv_sig * wv, te = p.flj * wv;
          phi += hit ? tq : 0.0;
          asig += hit ? ts : 0.0;
          beps += hit ? te : 0.0;
        } else {
          const float4 vjv = VJ[slot];
          const float wv = fmaf(vi32.z - vjv.z, dzf, fmaf(vi32.y - vjv.y, dyf, (vi32.x - vjv.x) * dxf));
          const PairVjpF32 p = pair_vjp_f32(r2f, tp.c6, tp.c12, wljf, wcf, c.betaf, c.two_beta_sqrtpif, c.mb2l2e,
                                            c.sw_on2f, c.sw_invf);
          const float tq = qj * p.gc * wv, ts = p.dflj * tp.inv_sig * wv, te = p.flj * wv;
          phi += static_cast<double>(hit ? tq : 0.f);
          asig += static_cast<double>(hit ? ts : 0.f);
          beps += static_cast<double>(hit ? te : 0.f);
        }
      } else {
        if constexpr (F64) {
          PairF64 p = FF ? pair_f64_ff(r2d, tp.c6, tp.c12, qi64 * pj64.w * wcd, wljd, c.beta, c.two_beta_sqrtpi,
                                       c.erfc_short != 0, c.sw_on2, c.sw_inv)
                         : pair_f64(r2d, tp.c6, tp.c12, qi64 * pj64.w, c.beta, c.two_beta_sqrtpi, c.erfc_short != 0);
          p.f = hit ? p.f : 0.0;
          p.u_lj = hit ? p.u_lj : 0.0;
          p.u_c = hit ? p.u_c : 0.0;
          if constexpr (MODE == kAdjoint) {
            p.erfc_over_r = hit ? p.erfc_over_r : 0.0;
            p.dudsig_lj = hit ? p.dudsig_lj : 0.0;
          }
          en += p.u_lj + p.u_c;
          if constexpr (HALF) {
            hgx = p.f * dxd;
            hgy = p.f * dyd;
            hgz = p.f * dzd;
            hu = p.u_lj + p.u_c;
          }
          if constexpr (MODE != kEnergy) {  // explicit FMAs: the same rounding in every copy of the loop
            fx = fma(p.f, dxd, fx);
            fy = fma(p.f, dyd, fy);
            fz = fma(p.f, dzd, fz);
          }
          if constexpr (MODE == kForces) {
            if (VIR && o.want_virial) {
              wxx += p.f * dxd * dxd; wxy += p.f * dxd * dyd; wxz += p.f * dxd * dzd;
              wyy += p.f * dyd * dyd; wyz += p.f * dyd * dzd; wzz += p.f * dzd * dzd;
            }
          }
          if constexpr (MODE == kAdjoint) {
            phi += (FF ? pj64.w * wcd : pj64.w) * p.erfc_over_r;
            asig += p.dudsig_lj * tp.inv_sig;
            beps += p.u_lj;
          }
        } else {
          PairF32 p;
          if constexpr (TAB != 0)
            p = pair_f32_tab<TAB>(r2f, tp.c6, tp.c12, qi32 * qj, d.rtab, c.tab_inv_h, c.tab_last);
          else if constexpr (FF)
            p = pair_f32_ff(r2f, tp.c6, tp.c12, qi32 * qj * wcf, wljf, c.betaf, c.two_beta_sqrtpif, c.mb2l2e,
                            c.sw_on2f, c.sw_invf);
          else
            p = pair_f32(r2f, tp.c6, tp.c12, qi32 * qj, c.betaf, c.two_beta_sqrtpif, c.mb2l2e);
          p.f = hit ? p.f : 0.f;
          if constexpr (MODE == kAdjoint) {
            p.u_lj = hit ? p.u_lj : 0.f;
            p.erfc_over_r = hit ? p.erfc_over_r : 0.f;
            p.dudsig_lj = hit ? p.dudsig_lj : 0.f;
          }
          float pu = hit ? p.u_lj + p.u_c : 0.f;  // the pair's energy, one select
          // (kept in single precision here: converted after the select, not selected in
          // double after the conversion, which takes two selects)
          asm volatile("" : "+v"(pu));
          // Per-atom sums (force, energy, dE/dq) take every pair's single-precision term
          // into a double accumulator; the virial is summed per lane in single precision
          // and reduced in double.
          en += static_cast<double>(pu);
          if constexpr (HALF) hu = pu;
          if constexpr (MODE != kEnergy) {
            const float gx = p.f * dxf, gy = p.f * dyf, gz = p.f * dzf;
            if constexpr (HALF) {
              hgx = gx;
              hgy = gy;
              hgz = gz;
            }
            fx += static_cast<double>(gx);
            fy += static_cast<double>(gy);
            fz += static_cast<double>(gz);
            if constexpr (MODE == kForces) {
              if (VIR && o.want_virial) {
                swxx = fmaf(gx, dxf, swxx); swxy = fmaf(gx, dyf, swxy); swxz = fmaf(gx, dzf, swxz);
                swyy = fmaf(gy, dyf, swyy); swyz = fmaf(gy, dzf, swyz); swzz = fmaf(gz, dzf, swzz);
              }
            }
          }
          if constexpr (MODE == kAdjoint) {
            phi += static_cast<double>((FF ? qj * wcf : qj) * p.erfc_over_r);
            asig += static_cast<double>(p.dudsig_lj * tp.inv_sig);
            beps += static_cast<double>(p.u_lj);
          }
        }
      }
      if constexpr (HALF) {
        // The J candidates' shares: sums over the K rows (K consecutive lanes), staged by row 0.
        if constexpr (MODE == kForces) {
          // the candidates' shares are minus these sums: the sign is applied at the flush
          const auto cx = group_sum<K>(hgx), cy = group_sum<K>(hgy), cz = group_sum<K>(hgz);
          // (summed in every lane, before the row-0 test: the last DPP move then folds into its
          // addition instead of being a move of its own beside an addition under the test)
          if constexpr (!F64) asm volatile("" ::"v"(cx), "v"(cy), "v"(cz));
          if constexpr (decltype(check_c)::value) {
            if (nst + J > kStage<F64>) flush();
          }
          if (ii == 0 && jv) {
            StageT<F64> &st = ST[nst + jj];
            st.x = cx;
            st.y = cy;
            st.z = cz;
            st.s = sj;
          }
          nst += navail;
        } else if constexpr (MODE == kEnergy) {
          if (o.atom_energy) {  // per-atom energies: half of each pair's energy to j
            const auto cu = group_sum<K>(hu);
            if constexpr (decltype(check_c)::value) {
              if (nst + J > kStage<F64>) flush();
            }
            if (ii == 0 && jv) {
              StageT<F64> &st = ST[nst + jj];
              st.x = static_cast<decltype(st.x)>(0.5) * cu;
              st.s = sj;
            }
            nst += navail;
          }
        }
      }
      head += static_cast<uint32_t>(navail);
    };

    // Every complete group in the ring; with PAIRS2 two at a time while there are two:
    // the two copies form one basic block, so that their loads and latencies overlap.
    // (The FP64 group would spill at twice its registers.)
    auto drain_with = [&](auto far_c, auto vir_c) {
      if constexpr (!F64 && PAIRS2) {
        while (tail - head >= 2u * static_cast<uint32_t>(J)) {
          if constexpr (HALF) {
            if (nst + 2 * J > kStage<F64>) flush();  // room for both groups' shares
          }
          process_group(J, far_c, vir_c, std::false_type{});
          process_group(J, far_c, vir_c, std::false_type{});
        }
      }
      while (tail - head >= static_cast<uint32_t>(J)) process_group(J, far_c, vir_c, std::true_type{});
    };
    auto drain = [&]() {
      if constexpr (F64 || (!PAIRS2 && !HALF)) {
        drain_with(std::true_type{}, std::true_type{});
      } else if constexpr (MODE == kForces) {
        if (any_far) {
          if (o.want_virial) drain_with(std::true_type{}, std::true_type{});
          else drain_with(std::true_type{}, std::false_type{});
        } else {
          if (o.want_virial) drain_with(std::false_type{}, std::true_type{});
          else drain_with(std::false_type{}, std::false_type{});
        }
      } else {
        if (any_far) drain_with(std::true_type{}, std::false_type{});
        else drain_with(std::false_type{}, std::false_type{});
      }
    };

    // Walk this item's candidates 64 at a time; the next chunk's loads are issued
    // before the current chunk is filtered and evaluated, to hide their latency.
    int run0 = 0;  // wave-uniform: the run holding the next chunk's first candidate
    // A chunk of 64 candidates rarely spans more than three runs: the run entries
    // run0 .. run0 + 3 are read at once (wave-uniform addresses) and each lane picks
    // its run by comparisons; the rare lane beyond them walks on.  The next chunk
    // starts in the run of this chunk's last lane or a later one.
    auto load = [&](int P, uint4 &f, int &t, float &q, double4 &p, bool &v, int &sidx, double4 &vv) {
      while (L.runs[run0 + 1].y <= P) ++run0;
      const int2 ra = L.runs[run0], rb = L.runs[run0 + 1], rc = L.runs[run0 + 2], rd = L.runs[run0 + 3];
      const int pos = P + lane;
      v = pos < hi_c;
      int r = run0;
      int2 cur = ra;
      if (pos >= rb.y) { cur = rb; r = run0 + 1; }
      if (pos >= rc.y) { cur = rc; r = run0 + 2; }
      if (pos >= rd.y) { cur = rd; r = run0 + 3; }
      if (v && r == run0 + 3) {
        while (L.runs[r + 1].y <= pos) cur = L.runs[++r];
      }
      const int aa = v ? cur.x + (pos - cur.y) : ra.x + (P - ra.y);
      run0 = __builtin_amdgcn_readlane(v ? r : run0, 63);
      sidx = aa;
      f = d.s_fix[aa];
      t = d.s_type[aa];
      if constexpr (F64) p = d.s_pos64[aa];
      else q = d.s_q32[aa];
      if constexpr (MODE == kVJP) vv = d.vsort[aa];
    };
    uint4 fj = make_uint4(0u, 0u, 0u, 0u);
    int tj = 0;
    float qj = 0.f;
    double4 pj64 = make_double4(0, 0, 0, 0);
    bool valid = false;
    int sj = 0;
    double4 vj = make_double4(0, 0, 0, 0);  // force VJP: the candidate's v (sorted copy)
    // The first chunk's loads are issued with the row atoms' windows (above), in one
    // round; the windows are spread to LDS meanwhile, and the chunk loop's first LDS
    // barrier makes them visible.
    int P = lo_c;
    if (P < hi_c) load(P, fj, tj, qj, pj64, valid, sj, vj);
    // Bounding box of the cluster, relative to its first atom (minimum image).
    {
      const uint4 u0 = make_uint4(__shfl(fi.x, 0, 64), __shfl(fi.y, 0, 64), __shfl(fi.z, 0, 64), 0u);
      const int dx = static_cast<int>(fi.x - u0.x), dy = static_cast<int>(fi.y - u0.y),
                dz = static_cast<int>(fi.z - u0.z);
      // rows without an atom repeat the first atom (ia = first), so they do not widen the box
      int lox, loy, loz, hix, hiy, hiz;
      if constexpr (HALF) {
        lox = shfl_group_min<K>(dx), loy = shfl_group_min<K>(dy), loz = shfl_group_min<K>(dz);
        hix = shfl_group_max<K>(dx), hiy = shfl_group_max<K>(dy), hiz = shfl_group_max<K>(dz);
      } else {
        lox = shfl_rows_min<J>(dx), loy = shfl_rows_min<J>(dy), loz = shfl_rows_min<J>(dz);
        hix = shfl_rows_max<J>(dx), hiy = shfl_rows_max<J>(dy), hiz = shfl_rows_max<J>(dz);
      }
      const int lo3[3] = {lox, loy, loz}, hi3[3] = {hix, hiy, hiz};
      const uint32_t base3[3] = {u0.x, u0.y, u0.z};
      uint32_t cc[3], hh[3];
      for (int a = 0; a < 3; ++a) {
        // centre floor((lo + hi) / 2) and half-width max(hi - mid, mid - lo) = ceil(extent / 2),
        // from the extent hi - lo in 32 bits (it is below 2^32)
        const uint32_t ext = static_cast<uint32_t>(hi3[a]) - static_cast<uint32_t>(lo3[a]);
        cc[a] = base3[a] + static_cast<uint32_t>(lo3[a]) + (ext >> 1);
        hh[a] = (ext >> 1) + (ext & 1u);
      }
      // wave-uniform (every row reduced to the same box): keep it in scalar registers
      ctr = make_uint4(uni(static_cast<int>(cc[0])), uni(static_cast<int>(cc[1])), uni(static_cast<int>(cc[2])), 0u);
      half = make_uint4(uni(static_cast<int>(hh[0])), uni(static_cast<int>(hh[1])), uni(static_cast<int>(hh[2])), 0u);
    }
    any_far = __ballot(ivalid && far_i) != 0;
    // Row ii's window as bytes, 4 per word: bits 0-63 of the mask are j - i = -64..-1,
    // then j = i, then mask bits 64-127 (j - i = 1..64); word m holds bits 4m..4m+3 of
    // that 132-bit string, each spread to the low bit of a byte.
    // FF variants: bit 1 of each byte from the 1-4 window, whose self position is 0.
    // Lane jj takes words jj, jj + J, ...: pass t reads 32-bit piece (jj + J t) >> 3 of the
    // string, which is t for every lane when J = 8 and 2 t or 2 t + 1 when J = 16.
    if constexpr (!F64 || FF) {
      static_assert(J == 8 || J == 16, "8 or 16 lanes per row");
      auto piece = [](const uint4 &mk, uint32_t self, int w) -> uint32_t {
        return w == 0 ? mk.x : w == 1 ? mk.y : w == 2 ? (mk.z << 1) | self : w == 3 ? (mk.w << 1) | (mk.z >> 31) : mk.w >> 31;
      };
#pragma unroll
      for (int t = 0; t < (kExBytes / 4 + J - 1) / J; ++t) {
        const int m = jj + J * t;
        const int w0 = (J / 8) * t, w1 = w0 + 1 < 4 ? w0 + 1 : 4;  // the pass's pieces
        const bool second = J == 16 && (jj & 8);
        auto spread = [&](const uint4 &mk, uint32_t self) -> uint32_t {
          const uint32_t src = second ? piece(mk, self, w1) : piece(mk, self, w0);
          const uint32_t nib = (src >> ((m & 7) * 4)) & 15u;
          return (nib * 0x00204081u) & 0x01010101u;
        };
        uint32_t word = spread(mask_i, 1u);
        if constexpr (FF) word |= spread(mask14_i, 0u) << 1;
        if (m < kExBytes / 4) L.exw[ii * (kExBytes / 4) + m] = word;
      }
    }
    wait_vm_loads();  // the cluster's own data and the first chunk have arrived
    bool requested = false;
    while (P < hi_c) {
      const int Pn = P + 64;
      uint4 fj_n = fj;
      int tj_n = tj;
      float qj_n = qj;
      double4 pj64_n = pj64;
      bool valid_n = false;
      int sj_n = sj;
      double4 vj_n = vj;
      if (Pn < hi_c) {
        load(Pn, fj_n, tj_n, qj_n, pj64_n, valid_n, sj_n, vj_n);
      } else if (dynamic && !(closed & (1u << home))) {
        // the next item, requested after this item's last loads (vector-memory waits
        // complete in issue order, so an earlier request would hold up the chunks)
        pending = request(home);
        have_pending = true;
        requested = true;
      }

      // Box filter, then compact the survivors into the ring.
      const bool keep = valid && box_dist2(fj, ctr, half, s2x, s2y, s2z) < c.rc2_box;
      const uint64_t mk = __ballot(keep);
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mk >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mk), 0u));
      const int slot = static_cast<int>((tail + below) & (kRing - 1));
      wave_lds_sync();  // earlier ring reads are complete before slots are reused
      if (keep) {
        if constexpr (F64) {
          L.pos[slot] = pj64;
          L.meta[slot] = make_int4(static_cast<int>(fj.w), tj, HALF ? sj : 0, 0);
        } else {
          L.ring[slot].fix = fj;
          L.ring[slot].qt = make_float2(qj, __int_as_float(tj));
          if constexpr (HALF) L.ring[slot].sidx = make_int2(sj, 0);
        }
        if constexpr (MODE == kVJP) {
          if constexpr (F64) VJ[slot] = vj;
          else VJ[slot] = make_float4(static_cast<float>(vj.x), static_cast<float>(vj.y), static_cast<float>(vj.z), 0.f);
        }
      }
      wave_lds_sync();
      tail += static_cast<uint32_t>(__popcll(mk));
      drain();

      P = Pn;
      fj = fj_n;
      tj = tj_n;
      qj = qj_n;
      pj64 = pj64_n;
      valid = valid_n;
      sj = sj_n;
      vj = vj_n;
    }
    if (tail != head) {
      if (any_far) process_group(static_cast<int>(tail - head), std::true_type{}, std::true_type{}, std::true_type{});
      else process_group(static_cast<int>(tail - head), std::false_type{}, std::true_type{}, std::true_type{});
    }
    if (dynamic && !requested && !(closed & (1u << home))) {  // an item without candidates
      pending = request(home);
      have_pending = true;
    }

    // The single-precision sums become double only where they are reduced, so that
    // few of them are live in double at a time.
    const double phi_scale = F64 ? c.ke : c.sqrt_ke;

    if constexpr (ADJ) {
      // Per-type sums of the sigma / eps partials over this item's rows (scaled by the
      // system's grad_energy in k_finish for the adjoint).
      const double a_l = 0.5 * asig, b_l = 0.5 * beps;
      const int my_t = ivalid ? ti : -1;
      double keep_a = 0.0, keep_b = 0.0;
      uint64_t left_t = __ballot(my_t >= 0);
      while (left_t) {
        const int lead = __ffsll(static_cast<unsigned long long>(left_t)) - 1;
        const int tt = __shfl(my_t, lead, 64);
        const bool mine = my_t == tt;
        const double sa = wave_sum(mine ? a_l : 0.0);
        const double sb = wave_sum(mine ? b_l : 0.0);
        if (lane == tt) {
          keep_a = sa;
          keep_b = sb;
        }
        left_t &= ~__ballot(mine);
      }
      if (lane < T) {
        d.adj_partials[static_cast<int64_t>(lane) * d.n_slots + m] = keep_a;
        d.adj_partials[static_cast<int64_t>(T + lane) * d.n_slots + m] = keep_b;
      }
    }

    // Per-atom sums of this item: the row's four sums (force x, y, z, then energy or
    // phi) reduced over its J lanes, sum e ending in lanes jj = e J/4 .. (e + 1) J/4 - 1,
    // whose first lane writes it.  With one item per cluster they are final and go
    // straight to the caller's arrays (original atom order); otherwise to this item's
    // part, added up by k_finish.
    if constexpr (HALF) {
      // Half shell: a row is the J lanes ii, ii + K, ...; butterfly sums over them (once per
      // item), then lane jj = 0 of each row adds its atom's sums to the accumulators.
      if (nst > 0) flush();
      double r4[4] = {fx, fy, fz, en};
#pragma unroll
      for (int off = K; off < 64; off <<= 1)
#pragma unroll
        for (int e = 0; e < 4; ++e) r4[e] += __shfl_xor(r4[e], off, 64);
      if (ivalid && jj == 0) {
        if constexpr (MODE == kForces) {
          acc_add(0, i, r4[0] * scx);
          acc_add(1, i, r4[1] * scy);
          acc_add(2, i, r4[2] * scz);
        } else if constexpr (MODE == kEnergy) {
          if (o.atom_energy) acc_add(3, i, 0.5 * r4[3]);
        }
      }
    } else {
      const double rowv[4] = {fx, fy, fz, ADJ ? phi : en};
      const int ent = jj / (J / 4);
      const double sce = ent == 0 ? scx : ent == 1 ? scy : ent == 2 ? scz : (ADJ ? phi_scale : 1.0);
      const double rv = reduce_scatter<J, 4>(rowv, lane) * sce;
      const bool writer = ivalid && jj % (J / 4) == 0;
      if (writer) {
        if (Q == 1) {
          if constexpr (MODE == kForces) {
            if (ent < 3) o.force[3 * static_cast<int64_t>(oi) + ent] = rv;
          } else if constexpr (MODE == kEnergy) {
            if (ent == 3 && o.atom_energy) o.atom_energy[oi] = 0.5 * rv;
          } else if constexpr (MODE == kVJP) {
            if (ent == 3 && o.grad_charge) o.grad_charge[oi] = rv;
          } else {
            const double g = o.grad_energy[sys];
            if (ent < 3 && o.grad_pos) o.grad_pos[3 * static_cast<int64_t>(oi) + ent] = -g * rv;
            if (ent == 3 && o.grad_charge) o.grad_charge[oi] = g * rv;
          }
        } else {
          (&d.part[static_cast<int64_t>(part) * d.N + i].x)[ent] = rv;
        }
      }
    }

    // Energy / virial sums of this item (a plain wave sum, before the row reduction),
    // one entry at a time; lane k keeps entry k.
    if constexpr (MODE == kForces || MODE == kEnergy) {
      if (o.want_part) {
        double mine = 0.0;
        if (MODE == kForces && o.want_virial) {
          // the seven distinct entries (and a zero) reduced together over the wave, sum
          // k ending in lanes 8k .. 8k + 7; each pair counted twice by the full-shell
          // form, once by the half-shell one
          constexpr double hs = HALF ? 1.0 : 0.5;
          const double v[8] = {hs * en, hs * scx * scx * D(wxx, swxx), hs * scx * scy * D(wxy, swxy),
                               hs * scx * scz * D(wxz, swxz), hs * scy * scy * D(wyy, swyy),
                               hs * scy * scz * D(wyz, swyz), hs * scz * scz * D(wzz, swzz), 0.0};
          const double r = reduce_scatter<64, 8>(v, lane);
          // entry order: energy, xx, xy, xz, yx, yy, yz, zx, zy, zz
          const int src = lane == 0 ? 0 : lane == 1 ? 1 : (lane == 2 || lane == 4) ? 2
                        : (lane == 3 || lane == 7) ? 3 : lane == 5 ? 4 : (lane == 6 || lane == 8) ? 5 : 6;
          mine = __shfl(r, 8 * src, 64);
          if (lane < kPart) d.partials[static_cast<int64_t>(lane) * d.n_slots + m] = mine;
        } else {
          mine = wave_sum((HALF ? 1.0 : 0.5) * en);
          if (lane < kPart) d.partials[static_cast<int64_t>(lane) * d.n_slots + m] = lane == 0 ? mine : 0.0;
        }
      }
    }
    // The next item (dynamic schedule): the loop leaves before its end when there is none,
    // so that no record stays live from one item to the next.
    if (!dynamic) break;
    islot = -1;
    if (have_pending) {
      islot = slot_of(home, pending);
      have_pending = false;
      if (islot < 0) closed |= 1u << home;
    }
    if (islot < 0) islot = steal();
    if (islot < 0) break;
    rec = load_item(d.items, uni(islot));
  }
}

// Sum of one partial component (energy or a virial entry of a system) over the wave
// slots [lo, hi), in a fixed order.
// Loads are unconditional (indices clamped) so that a thread's loads are all in flight.
__device__ inline double sum_component(const double *__restrict__ vals, int64_t lo, int64_t hi,
                                       double (*lds)[kPart]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int kUnroll = 8;
  double acc = 0.0;
  for (int64_t q0 = lo + threadIdx.x; q0 < hi; q0 += kUnroll * kFinishBlock) {
    double v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t q = q0 + u * kFinishBlock;
      v[u] = vals[q < hi ? q : lo];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += q0 + u * kFinishBlock < hi ? v[u] : 0.0;
  }
  const double s = wave_sum(acc);
  if (lane == 0) lds[wave][0] = s;
  __syncthreads();
  double t = 0.0;
  for (int wv = 0; wv < kFinishBlock / 64; ++wv) t += lds[wv][0];
  return t;
}

// Per-atom outputs (sum of the S parts, in order), per-system energy / virial and
// per-type gradients, in one launch: blocks [0, nA) take atoms, the next kPart B
// blocks take (system, energy or virial entry), the last 2T blocks (adjoint only)
// take types.
template <int MODE>
__global__ void __launch_bounds__(kFinishBlock) k_finish(Dev d, Out o, int S, int nA, double *energy, double *virial,
                                                        int nv, const double *__restrict__ eps, double *grad_sigma,
                                                        double *grad_eps, int half, uint32_t cluster_key) {
  __shared__ double lds[kFinishBlock / 64][kPart];
  // The pair kernel is complete: its work counters start again from zero next time.
  if (blockIdx.x == 0 && threadIdx.x < kXcds) d.queue[threadIdx.x * kQueueStride] = 0u;
  // (the pair kernel's own test: a build for another cluster size or split has another
  // layout, and then nothing is written)
  if (!built_for(d.status, d.N, true, false, half != 0, cluster_key)) return;
  const int blk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (blk < nA) {
    const int i = blk * kFinishBlock + threadIdx.x;
    if (i >= d.N) return;
    if (half) {  // half-shell accumulators: copy out, and zero for the next call
      const int oi = static_cast<int>(d.s_fix[i].w);
      // component c of atom i's accumulator (64-bit fixed point, two limbs on the FP64
      // path), then zeroed
      auto take = [&](int c) -> double {
        const int64_t at = static_cast<int64_t>(c) * d.N + i;
        double v;
        if (d.jacc_lo) {
          v = from_fixed2(d.jacc_fix[at], d.jacc_lo[at]);
          d.jacc_lo[at] = 0;
        } else {
          v = from_fixed(d.jacc_fix[at]);
        }
        d.jacc_fix[at] = 0;
        return v;
      };
      if constexpr (MODE == kForces) {
        o.force[3 * oi + 0] = take(0);
        o.force[3 * oi + 1] = take(1);
        o.force[3 * oi + 2] = take(2);
      } else if constexpr (MODE == kEnergy) {
        if (o.atom_energy) o.atom_energy[oi] = take(3);
      }
      return;
    }
    double4 s = d.part[i];
    for (int p = 1; p < S; ++p) {
      const double4 q = d.part[static_cast<int64_t>(p) * d.N + i];
      s.x += q.x;
      s.y += q.y;
      s.z += q.z;
      s.w += q.w;
    }
    const int oi = static_cast<int>(d.s_fix[i].w);
    if constexpr (MODE == kForces) {
      o.force[3 * oi + 0] = s.x;
      o.force[3 * oi + 1] = s.y;
      o.force[3 * oi + 2] = s.z;
    } else if constexpr (MODE == kEnergy) {
      if (o.atom_energy) o.atom_energy[oi] = 0.5 * s.w;
    } else if constexpr (MODE == kVJP) {
      if (o.grad_charge) o.grad_charge[oi] = s.w;
    } else {
      int lo = 0, hi = d.B - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.desc[mid].atom_begin <= i) lo = mid; else hi = mid - 1;
      }
      const double g = o.grad_energy[lo];
      if (o.grad_pos) {
        o.grad_pos[3 * oi + 0] = -g * s.x;
        o.grad_pos[3 * oi + 1] = -g * s.y;
        o.grad_pos[3 * oi + 2] = -g * s.z;
      }
      if (o.grad_charge) o.grad_charge[oi] = g * s.w;
    }
    return;
  }
  if (blk < nA + kPart * d.B) {
    const int b = (blk - nA) / kPart, k = (blk - nA) % kPart;
    if (MODE == kAdjoint || MODE == kVJP || k >= nv) return;
    const SysDesc &sd = d.desc[b];
    const int64_t lo = static_cast<int64_t>(d.col_clu_start[sd.col_begin]) * S;
    const int64_t hi = static_cast<int64_t>(d.col_clu_start[sd.col_begin + sd.dims[0] * sd.dims[1]]) * S;
    const double t = sum_component(d.partials + static_cast<int64_t>(k) * d.n_slots, lo, hi, lds);
    if (threadIdx.x == 0) {
      if (k == 0) {
        if (energy) energy[b] = t;
      } else if (virial) {
        virial[9 * b + (k - 1)] = t;
      }
    }
    return;
  }
  if constexpr (MODE == kAdjoint || MODE == kVJP) {
    // One (sigma or eps, type) entry: sum over every wave slot of every system, each
    // scaled by its system's grad_energy for the adjoint (the force VJP has no such weight).
    const int T = d.T;
    const int t = blk - nA - kPart * d.B;
    if (t >= 2 * T) return;
    double acc = 0.0;
    for (int b = 0; b < d.B; ++b) {
      const SysDesc &sd = d.desc[b];
      const int64_t lo = static_cast<int64_t>(d.col_clu_start[sd.col_begin]) * S;
      const int64_t hi = static_cast<int64_t>(d.col_clu_start[sd.col_begin + sd.dims[0] * sd.dims[1]]) * S;
      double s = 0.0;
      for (int64_t q0 = lo + threadIdx.x; q0 < hi; q0 += 4 * kFinishBlock) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t q = q0 + u * kFinishBlock;
          v[u] = d.adj_partials[static_cast<int64_t>(t) * d.n_slots + (q < hi ? q : lo)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s += q0 + u * kFinishBlock < hi ? v[u] : 0.0;
      }
      acc += MODE == kVJP ? s : o.grad_energy[b] * s;
    }
    acc = wave_sum(acc);
    if (lane == 0) lds[wave][0] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int wv = 0; wv < kFinishBlock / 64; ++wv) s += lds[wv][0];
      if (t < T) {
        if (grad_sigma) grad_sigma[t] = s;
      } else if (grad_eps) {
        grad_eps[t - T] = eps[t - T] > 0.0 ? s / eps[t - T] : 0.0;
      }
    }
  }
}

// Compute units of the current device (cached per device).
int compute_units() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Workgroups of a kernel that fit on one compute unit at once (cached per kernel and device).
template <typename Query>
int resident_workgroups(const void *kern, size_t lds_bytes, Query query) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, int, size_t>, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(kern, dev, lds_bytes);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (query(&n) != hipSuccess || n < 1) n = 1;
  cache[key] = n;
  return n;
}

template <bool F64, bool TABLDS, int K>
void launch_cluster_mode(int mode, bool half, int var, int64_t wgs, int dyn, int wg_per_cu, hipStream_t s,
                         const Dev &d, const Consts &c, const Out &o, int Q) {
  const dim3 block(64);
  auto go = [&](auto kern, auto mode_tag, auto half_tag) {
    const size_t lds = dyn_lds_bytes<F64, decltype(mode_tag)::value, TABLDS, decltype(half_tag)::value>(d.T);
    int64_t g = wgs;
    if (dyn) {
      // persistent grid: what fits on the device at once (at most wg_per_cu per CU)
      const int fit = resident_workgroups(reinterpret_cast<const void *>(kern), lds, [&](int *n) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, kern, 64, lds);
      });
      g = std::min<int64_t>(g, static_cast<int64_t>(compute_units()) * std::min(fit, wg_per_cu));
    }
    g = std::max<int64_t>((g + kXcds - 1) / kXcds * kXcds, kXcds);  // a multiple of the XCD count
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(g)), block, lds, s, d, c, o, Q, dyn);
  };
  // Two groups per pass (mixed path, full shell, static schedule) when the grid fits on
  // the GPU at once at 4 waves per SIMD: then the fifth resident wave has nothing to do
  // and the instruction-level parallelism of two groups is worth more (23.6k-atom box:
  // 64.2 -> 61.0 us; 64-replica batch, 100,000 items: 1,083 against 1,117 us with it).
  const bool pairs2 = !F64 && !dyn && wgs <= static_cast<int64_t>(compute_units()) * kPairs2WavesPerCu;
  auto dispatch = [&](auto var_c) {
    constexpr int VAR = decltype(var_c)::value;
    using M0 = std::integral_constant<int, kForces>;
    using M1 = std::integral_constant<int, kEnergy>;
    using M2 = std::integral_constant<int, kAdjoint>;
    using M3 = std::integral_constant<int, kVJP>;
    if (mode == kForces) {
      // half shell: two groups per pass only for the plain evaluation (measured on the
      // 23.6k box: 54.7 -> 52.8 us; the force-field and table variants came out 1.5-2.4 us
      // slower with it)
      constexpr bool kHalfPairs2 = VAR == kVarPlain && !F64;
      if (half && pairs2 && kHalfPairs2)
        go(k_pair_cluster<F64, kForces, TABLDS, K, true, kHalfPairs2, VAR>, M0{}, std::true_type{});
      else if (half) go(k_pair_cluster<F64, kForces, TABLDS, K, true, false, VAR>, M0{}, std::true_type{});
      else if (pairs2) go(k_pair_cluster<F64, kForces, TABLDS, K, false, !F64, VAR>, M0{}, std::false_type{});
      else go(k_pair_cluster<F64, kForces, TABLDS, K, false, false, VAR>, M0{}, std::false_type{});
    } else if (mode == kEnergy) {
      if (half) go(k_pair_cluster<F64, kEnergy, TABLDS, K, true, false, VAR>, M1{}, std::true_type{});
      else if (pairs2) go(k_pair_cluster<F64, kEnergy, TABLDS, K, false, !F64, VAR>, M1{}, std::false_type{});
      else go(k_pair_cluster<F64, kEnergy, TABLDS, K, false, false, VAR>, M1{}, std::false_type{});
    } else {
      // the adjoint and the force VJP evaluate directly (never from tables), full shell
      constexpr int VA = VAR == kVarFF ? kVarFF : kVarPlain;
      if (mode == kAdjoint) {
        if (pairs2) go(k_pair_cluster<F64, kAdjoint, TABLDS, K, false, !F64, VA>, M2{}, std::false_type{});
        else go(k_pair_cluster<F64, kAdjoint, TABLDS, K, false, false, VA>, M2{}, std::false_type{});
      } else {
        if (pairs2) go(k_pair_cluster<F64, kVJP, TABLDS, K, false, !F64, VA>, M3{}, std::false_type{});
        else go(k_pair_cluster<F64, kVJP, TABLDS, K, false, false, VA>, M3{}, std::false_type{});
      }
    }
  };
  if (var == kVarFF) dispatch(std::integral_constant<int, kVarFF>{});
  else if constexpr (!F64) {
    if (var == kVarLin) dispatch(std::integral_constant<int, kVarLin>{});
    else if (var == kVarCub) dispatch(std::integral_constant<int, kVarCub>{});
    else dispatch(std::integral_constant<int, kVarPlain>{});
  } else {
    dispatch(std::integral_constant<int, kVarPlain>{});
  }
}

template <bool F64, bool TABLDS>
void launch_cluster_k(int K, int mode, bool half, int var, int64_t wgs, int dyn, int wg_per_cu, hipStream_t s,
                      const Dev &d, const Consts &c, const Out &o, int Q) {
  if (K == 8) launch_cluster_mode<F64, TABLDS, 8>(mode, half, var, wgs, dyn, wg_per_cu, s, d, c, o, Q);
  else launch_cluster_mode<F64, TABLDS, 4>(mode, half, var, wgs, dyn, wg_per_cu, s, d, c, o, Q);
}

}  // namespace

// Pair-kernel launch for one precision; instantiated in nb_pair_cluster_f32.hip and
// nb_pair_cluster_f64.hip so that the two compile in parallel.
template <bool F64>
void launch_cluster_pair_prec(const Plan &p, const Dev &d, const Consts &c, const Out &o, int mode, bool half,
                              hipStream_t s) {
  if (p.N > 0 && p.n_clusters_max > 0) {
    const int64_t items = p.n_clusters_max * p.split;  // upper bound on the work items
    const int64_t wgs = items;  // one wave per workgroup
    const int dyn = p.schedule == NB_SCHED_DYNAMIC ? 1 : 0;
    const bool tab = p.T <= kTabLds;
    const int K = p.cluster_size;
    timer_before(s);
    const int var = p.ff ? kVarFF : p.table == 1 ? kVarLin : p.table == 2 ? kVarCub : kVarPlain;
    if (tab) launch_cluster_k<F64, true>(K, mode, half, var, wgs, dyn, p.wg_per_cu, s, d, c, o, p.split);
    else launch_cluster_k<F64, false>(K, mode, half, var, wgs, dyn, p.wg_per_cu, s, d, c, o, p.split);
    timer_after(s);
  }
}

}  // namespace nb
