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
//      48% for K = 8, against ~25% for a plain cell stencil);
//   3. each row of J lanes accumulates its i atom's sums in registers; rows are
//      reduced with cross-lane shuffles at the end.
//
// A cluster's neighbour columns may be split over S waves (S = 1..4), which gives
// the GPU S times more, shorter waves to interleave; each wave writes its part of
// every atom's sums to its own slot, and k_finish adds the S parts in a fixed order,
// converts to the caller's atom order and reduces energies, virials and per-type
// sums.  Nothing is accumulated with atomics: results are deterministic.
// Full shell (every pair is evaluated from both sides), as in the paper.
#include "nb_pair_common.h"
#include "nb_pair_math.h"

namespace nb {

namespace {

constexpr int kRing = 128;           // ring buffer of staged j atoms (power of two)
constexpr int kTabLds = 16;          // type tables up to 16 x 16 are copied to LDS
constexpr int kFlush = 32;           // groups between single -> double flushes of the sums
constexpr int kXcds = 8;             // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kMaxRuns = 2 * 9 * 9;  // up to 9 x 9 neighbour columns, <= 2 z-runs each
constexpr int kFinishBlock = 256;

__device__ __forceinline__ uint32_t uabs_diff(uint32_t a, uint32_t b) {
  const int32_t d = static_cast<int32_t>(a - b);
  return d < 0 ? static_cast<uint32_t>(-static_cast<int64_t>(d)) : static_cast<uint32_t>(d);
}

// Squared distance (A^2, single precision) from a fixed-point point to a box given
// by centre and half extents, with minimum image per dimension.
__device__ __forceinline__ float box_dist2(const uint4 &p, const uint4 &ctr, const uint4 &half, float s2x, float s2y,
                                           float s2z) {
  const uint32_t ax = uabs_diff(p.x, ctr.x), ay = uabs_diff(p.y, ctr.y), az = uabs_diff(p.z, ctr.z);
  const float ex = static_cast<float>(ax > half.x ? ax - half.x : 0u);
  const float ey = static_cast<float>(ay > half.y ? ay - half.y : 0u);
  const float ez = static_cast<float>(az > half.z ? az - half.z : 0u);
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

template <int J>
__device__ __forceinline__ double row_sum(double v) {
  for (int off = 1; off < J; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
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

template <bool F64>
struct RingLds;

template <>
struct RingLds<false> {
  uint4 fix[kRing];  // fixed-point x, y, z, original index
  float2 qt[kRing];  // q * sqrt(k_e), type (as int bits)
  TypePair32 tab[kTabLds * kTabLds];
  int2 runs[kMaxRuns];
};

template <>
struct RingLds<true> {
  double4 pos[kRing];  // x, y, z, q
  int2 meta[kRing];    // original index, type
  TypePair64 tab[kTabLds * kTabLds];
  int2 runs[kMaxRuns];
};

template <bool F64, int MODE, bool TABLDS, int K>
__global__ void __launch_bounds__(64) k_pair_cluster(Dev d, Consts c, Out o, int S) {
  constexpr int J = 64 / K;  // j atoms per group (lanes per row)
  __shared__ RingLds<F64> L;
  // Workgroups are dealt to the 8 XCDs round robin; give each XCD a contiguous
  // range of waves (neighbouring clusters) so that its L2 holds their j atoms.
  const int per_xcd = static_cast<int>(gridDim.x) / kXcds;
  const int w = static_cast<int>(blockIdx.x % kXcds) * per_xcd + static_cast<int>(blockIdx.x / kXcds);
  if (!built_for(d.status, d.N, true)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(d.status, NB_STATUS_NOT_BUILT);
    return;
  }
  const int n_clu = d.col_clu_start[d.n_columns];
  const int I = w / S, part = w - (w / S) * S;
  if (I >= n_clu) return;  // the grid is sized by an upper bound on the cluster count
  const int lane = threadIdx.x, ii = lane / J, jj = lane % J;
  const int T = d.T;
  if constexpr (TABLDS) {
    for (int k = lane; k < T * T; k += 64) {
      if constexpr (F64) L.tab[k] = d.tab64[k];
      else L.tab[k] = d.tab32[k];
    }
  }

  // The cluster: its column, system, and atoms.
  const int col = cluster_column(d.col_clu_start, static_cast<int>(d.n_columns), I);
  int sys = 0;
  {
    int lo = 0, hi = d.B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (d.desc[mid].col_begin <= col) lo = mid; else hi = mid - 1;
    }
    sys = lo;
  }
  const SysDesc &sd = d.desc[sys];
  // Per-system constants as wave-uniform scalars: nothing in the pair loop below then
  // waits on a vector-memory load (so the next chunk's loads stay in flight).
  const float s2x = uni(sd.scale2f[0]), s2y = uni(sd.scale2f[1]), s2z = uni(sd.scale2f[2]);
  const double bxx = uni(sd.box[0]), bxy = uni(sd.box[1]), bxz = uni(sd.box[2]);
  const double ibx = uni(sd.inv_box[0]), iby = uni(sd.inv_box[1]), ibz = uni(sd.inv_box[2]);
  const int atom_begin = uni(sd.atom_begin);
  const int nx = uni(sd.dims[0]), ny = uni(sd.dims[1]), nz = uni(sd.dims[2]);
  const int col_local = col - uni(sd.col_begin);
  const int cell_begin = uni(sd.cell_begin);
  const int cb0 = cell_begin + col_local * nz;
  const int first = d.cell_start[cb0] + K * (I - d.col_clu_start[col]);
  const int left = d.cell_start[cb0 + nz] - first;
  const int count = left < K ? left : K;
  const int i = first + ii;
  const bool ivalid = ii < count;
  const int ia = ivalid ? i : first;
  const uint4 fi = d.s_fix[ia];
  const int oi = static_cast<int>(fi.w);
  const uint4 mask_i = d.excl_mask[oi];
  const bool far_i = d.excl_far[oi] != 0u;
  const int ti = d.s_type[ia];
  double4 pi64 = make_double4(0, 0, 0, 0);
  float qi32 = 0.f;
  if constexpr (F64) pi64 = d.s_pos64[ia];
  else qi32 = d.s_q32[ia];
  const double qi64 = F64 ? pi64.w * c.ke : 0.0;

  // Bounding box of the cluster, relative to its first atom (minimum image).
  uint4 ctr, half;
  {
    const uint4 u0 = make_uint4(__shfl(fi.x, 0, 64), __shfl(fi.y, 0, 64), __shfl(fi.z, 0, 64), 0u);
    const int dx = static_cast<int>(fi.x - u0.x), dy = static_cast<int>(fi.y - u0.y),
              dz = static_cast<int>(fi.z - u0.z);
    // rows without an atom repeat the first atom (ia = first), so they do not widen the box
    const int lox = shfl_rows_min<J>(dx), loy = shfl_rows_min<J>(dy), loz = shfl_rows_min<J>(dz);
    const int hix = shfl_rows_max<J>(dx), hiy = shfl_rows_max<J>(dy), hiz = shfl_rows_max<J>(dz);
    const int lo3[3] = {lox, loy, loz}, hi3[3] = {hix, hiy, hiz};
    const uint32_t base[3] = {u0.x, u0.y, u0.z};
    uint32_t cc[3], hh[3];
    for (int a = 0; a < 3; ++a) {
      const int64_t mid = (static_cast<int64_t>(lo3[a]) + hi3[a]) >> 1;  // floor
      const int64_t h = (hi3[a] - mid) > (mid - lo3[a]) ? (hi3[a] - mid) : (mid - lo3[a]);
      cc[a] = base[a] + static_cast<uint32_t>(static_cast<int32_t>(mid));
      hh[a] = static_cast<uint32_t>(h);
    }
    ctr = make_uint4(cc[0], cc[1], cc[2], 0u);
    half = make_uint4(hh[0], hh[1], hh[2], 0u);
  }

  const int kx = uni(sd.reach[0]), ky = uni(sd.reach[1]), kz = uni(sd.reach[2]);
  const int cx = col_local / ny, cy = col_local - (col_local / ny) * ny;
  const int cz0 = static_cast<int>((static_cast<uint64_t>(d.s_fix[first].z) * nz) >> 32);
  const int cz1 = static_cast<int>((static_cast<uint64_t>(d.s_fix[first + count - 1].z) * nz) >> 32);
  const bool allx = 2 * kx + 1 >= nx, ally = 2 * ky + 1 >= ny;
  const bool allz = (cz1 - cz0) + 2 * kz + 1 >= nz;
  const int xn = allx ? nx : 2 * kx + 1, yn = ally ? ny : 2 * ky + 1;

  // Per-lane sums for row ii's atom: single precision for a bounded number of
  // groups (mixed path), flushed into double.
  double fx = 0, fy = 0, fz = 0, en = 0, wxx = 0, wxy = 0, wxz = 0, wyy = 0, wyz = 0, wzz = 0;
  double phi = 0, asig = 0, beps = 0;
  float sfx = 0, sfy = 0, sfz = 0, sen = 0, swxx = 0, swxy = 0, swxz = 0, swyy = 0, swyz = 0, swzz = 0;
  float sphi = 0, sasig = 0, sbeps = 0;
  int groups = 0;
  auto flush = [&]() {
    if constexpr (!F64) {
      fx += sfx; fy += sfy; fz += sfz; en += sen;
      wxx += swxx; wxy += swxy; wxz += swxz; wyy += swyy; wyz += swyz; wzz += swzz;
      phi += sphi; asig += sasig; beps += sbeps;
      sfx = sfy = sfz = sen = swxx = swxy = swxz = swyy = swyz = swzz = sphi = sasig = sbeps = 0.f;
    }
    groups = 0;
  };

  uint32_t head = 0, tail = 0;  // wave-uniform ring positions

  // Evaluate pair (row ii's atom, ring entry head + jj) for navail <= J entries.
  auto process_group = [&](int navail) {
    const int slot = static_cast<int>((head + jj) & (kRing - 1));
    const bool jv = jj < navail;
    int oj, tj;
    if constexpr (F64) {
      const int2 m = L.meta[slot];
      oj = m.x;
      tj = m.y;
    } else {
      oj = static_cast<int>(L.fix[slot].w);
      tj = __float_as_int(L.qt[slot].y);
    }
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
      hit = ivalid && jv && r2d < c.rc2 && oi != oj;
    } else {
      const uint4 fj = L.fix[slot];
      qj = L.qt[slot].x;
      dxf = static_cast<float>(static_cast<int>(fi.x - fj.x));
      dyf = static_cast<float>(static_cast<int>(fi.y - fj.y));
      dzf = static_cast<float>(static_cast<int>(fi.z - fj.z));
      r2f = fmaf(s2z * dzf, dzf, fmaf(s2y * dyf, dyf, s2x * dxf * dxf));
      hit = ivalid && jv && r2f < c.rc2f && oi != oj;
    }
    const int delta = oj - oi;
    const bool check = hit && (static_cast<unsigned>(delta + kWindow) <= 2u * kWindow || far_i);
    if (__ballot(check)) {
      if (check && pair_excluded(mask_i, far_i, oi, oj, atom_begin, d.excl_far, o.excl_off, o.excl_idx))
        hit = false;
    }
    if (hit) {
      if constexpr (F64) {
        TypePair64 tp;
        if constexpr (TABLDS) tp = L.tab[ti * T + tj];
        else tp = d.tab64[ti * T + tj];
        const PairF64 p = pair_f64(r2d, tp.c6, tp.c12, qi64 * pj64.w, c.beta, c.two_beta_sqrtpi);
        en += p.u_lj + p.u_c;
        if constexpr (MODE != kEnergy) {
          fx += p.f * dxd;
          fy += p.f * dyd;
          fz += p.f * dzd;
        }
        if constexpr (MODE == kForces) {
          if (o.want_virial) {
            wxx += p.f * dxd * dxd; wxy += p.f * dxd * dyd; wxz += p.f * dxd * dzd;
            wyy += p.f * dyd * dyd; wyz += p.f * dyd * dzd; wzz += p.f * dzd * dzd;
          }
        }
        if constexpr (MODE == kAdjoint) {
          phi += pj64.w * p.erfc_over_r;
          asig += p.dudsig_lj * tp.inv_sig;
          beps += p.u_lj;
        }
      } else {
        TypePair32 tp;
        if constexpr (TABLDS) tp = L.tab[ti * T + tj];
        else tp = d.tab32[ti * T + tj];
        const PairF32 p = pair_f32(r2f, tp.c6, tp.c12, qi32 * qj, c.betaf, c.two_beta_sqrtpif, c.mb2l2e);
        sen += p.u_lj + p.u_c;
        if constexpr (MODE != kEnergy) {
          const float gx = p.f * dxf, gy = p.f * dyf, gz = p.f * dzf;
          sfx += gx;
          sfy += gy;
          sfz += gz;
          if constexpr (MODE == kForces) {
            if (o.want_virial) {
              swxx = fmaf(gx, dxf, swxx); swxy = fmaf(gx, dyf, swxy); swxz = fmaf(gx, dzf, swxz);
              swyy = fmaf(gy, dyf, swyy); swyz = fmaf(gy, dzf, swyz); swzz = fmaf(gz, dzf, swzz);
            }
          }
        }
        if constexpr (MODE == kAdjoint) {
          sphi = fmaf(qj, p.erfc_over_r, sphi);
          sasig = fmaf(p.dudsig_lj, tp.inv_sig, sasig);
          sbeps += p.u_lj;
        }
      }
    }
    head += static_cast<uint32_t>(navail);
    if (++groups >= kFlush) flush();
  };

  // Neighbour-column windows as runs [a0, a1) of sorted atoms, two slots per column
  // (a z-window that wraps around the box is two runs; an unused slot is empty).
  const int ncol = xn * yn;
  for (int k = lane; k < ncol; k += 64) {
    const int ox = k / yn, oy = k - (k / yn) * yn;
    int x = allx ? ox : cx - kx + ox;
    x += x < 0 ? nx : (x >= nx ? -nx : 0);
    int y = ally ? oy : cy - ky + oy;
    y += y < 0 ? ny : (y >= ny ? -ny : 0);
    const int cb = cell_begin + (x * ny + y) * nz;
    int2 r0, r1 = make_int2(0, 0);
    if (allz) {
      r0 = make_int2(d.cell_start[cb], d.cell_start[cb + nz]);
    } else {
      const int z0 = cz0 - kz, z1 = cz1 + kz + 1;  // [z0, z1)
      if (z0 < 0) {
        r0 = make_int2(d.cell_start[cb + z0 + nz], d.cell_start[cb + nz]);
        r1 = make_int2(d.cell_start[cb], d.cell_start[cb + z1]);
      } else if (z1 > nz) {
        r0 = make_int2(d.cell_start[cb + z0], d.cell_start[cb + nz]);
        r1 = make_int2(d.cell_start[cb], d.cell_start[cb + z1 - nz]);
      } else {
        r0 = make_int2(d.cell_start[cb + z0], d.cell_start[cb + z1]);
      }
    }
    L.runs[2 * k] = r0;
    L.runs[2 * k + 1] = r1;
  }
  __syncthreads();
  // This wave's share of the runs.
  const int r_begin = (2 * ncol * part) / S, r_end = (2 * ncol * (part + 1)) / S;

  // Walk the runs 64 atoms at a time; the next chunk's loads are issued before the
  // current chunk is filtered and evaluated, to hide their latency.
  int base = 0, end = 0;
  auto seek = [&](int rr) {  // first non-empty run at or after rr; sets base/end
    while (rr < r_end) {
      const int2 q = L.runs[rr];
      if (q.x < q.y) {
        base = q.x;
        end = q.y;
        return rr;
      }
      ++rr;
    }
    return rr;
  };
  auto load = [&](int b0, int e0, uint4 &f, int &t, float &q, double4 &p, bool &v) {
    const int a = b0 + lane;
    v = a < e0;
    const int aa = v ? a : b0;
    f = d.s_fix[aa];
    t = d.s_type[aa];
    if constexpr (F64) p = d.s_pos64[aa];
    else q = d.s_q32[aa];
  };
  uint4 fj = make_uint4(0u, 0u, 0u, 0u);
  int tj = 0;
  float qj = 0.f;
  double4 pj64 = make_double4(0, 0, 0, 0);
  bool valid = false;
  wait_vm_loads();  // the cluster's own data has arrived before the pair loop starts
  int r = seek(r_begin);
  if (r < r_end) load(base, end, fj, tj, qj, pj64, valid);
  while (r < r_end) {
    int nr = r;
    if (base + 64 < end) base += 64;
    else nr = seek(r + 1);
    uint4 fj_n = fj;
    int tj_n = tj;
    float qj_n = qj;
    double4 pj64_n = pj64;
    bool valid_n = false;
    if (nr < r_end) load(base, end, fj_n, tj_n, qj_n, pj64_n, valid_n);

    // Box filter, then compact the survivors into the ring.
    const bool keep = valid && box_dist2(fj, ctr, half, s2x, s2y, s2z) < c.rc2_box;
    const uint64_t m = __ballot(keep);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
    const int slot = static_cast<int>((tail + below) & (kRing - 1));
    __syncthreads();  // earlier ring reads are complete before slots are reused
    if (keep) {
      if constexpr (F64) {
        L.pos[slot] = pj64;
        L.meta[slot] = make_int2(static_cast<int>(fj.w), tj);
      } else {
        L.fix[slot] = fj;
        L.qt[slot] = make_float2(qj, __int_as_float(tj));
      }
    }
    __syncthreads();
    tail += static_cast<uint32_t>(__popcll(m));
    while (tail - head >= static_cast<uint32_t>(J)) process_group(J);

    r = nr;
    fj = fj_n;
    tj = tj_n;
    qj = qj_n;
    pj64 = pj64_n;
    valid = valid_n;
  }
  if (tail != head) process_group(static_cast<int>(tail - head));
  flush();

  if constexpr (!F64) {
    // fixed-point units -> Angstrom; phi carries one sqrt(k_e) from q'_j.
    fx *= sd.scale[0];
    fy *= sd.scale[1];
    fz *= sd.scale[2];
    wxx *= sd.scale[0] * sd.scale[0]; wxy *= sd.scale[0] * sd.scale[1]; wxz *= sd.scale[0] * sd.scale[2];
    wyy *= sd.scale[1] * sd.scale[1]; wyz *= sd.scale[1] * sd.scale[2]; wzz *= sd.scale[2] * sd.scale[2];
    phi *= c.sqrt_ke;
  } else {
    phi *= c.ke;
  }

  // Energy / virial sums of this wave (a plain wave sum, before the row reduction).
  if constexpr (MODE == kForces || MODE == kEnergy) {
    if (o.want_part) {
      const double v[kPart] = {0.5 * en, 0.5 * wxx, 0.5 * wxy, 0.5 * wxz, 0.5 * wxy, 0.5 * wyy,
                               0.5 * wyz, 0.5 * wxz, 0.5 * wyz, 0.5 * wzz};
      const int nv = (MODE == kForces && o.want_virial) ? kPart : 1;
      double mine = 0.0;
      for (int k = 0; k < nv; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == k) mine = s;
      }
      if (lane < kPart) d.partials[static_cast<int64_t>(lane) * d.n_slots + w] = lane < nv ? mine : 0.0;
    }
  }
  if constexpr (MODE == kAdjoint) {
    // Per-type sums of the sigma / eps partials over this wave's rows (scaled by the
    // system's grad_energy in k_finish).
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
      d.adj_partials[static_cast<int64_t>(lane) * d.n_slots + w] = keep_a;
      d.adj_partials[static_cast<int64_t>(T + lane) * d.n_slots + w] = keep_b;
    }
  }

  // Per-atom sums of this wave's share: rows reduced over their J lanes.
  fx = row_sum<J>(fx);
  fy = row_sum<J>(fy);
  fz = row_sum<J>(fz);
  const double w4 = row_sum<J>(MODE == kAdjoint ? phi : en);
  if (jj == 0 && ivalid) d.part[static_cast<int64_t>(part) * d.N + i] = make_double4(fx, fy, fz, w4);
}

// Energy (and virial) of system b: sum of the wave slots [lo, hi), in a fixed order.
// Loads are unconditional (indices clamped) so that a thread's loads are all in flight.
template <int NV>
__device__ inline void sum_slots(const Dev &d, int64_t lo, int64_t hi, double *energy, double *virial, int b,
                                 double (*lds)[kPart]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int kUnroll = 4;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int64_t q0 = lo + threadIdx.x; q0 < hi; q0 += kUnroll * kFinishBlock) {
    double v[kUnroll][NV];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t q = q0 + u * kFinishBlock;
      const int64_t qq = q < hi ? q : lo;
#pragma unroll
      for (int k = 0; k < NV; ++k) v[u][k] = d.partials[static_cast<int64_t>(k) * d.n_slots + qq];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool in = q0 + u * kFinishBlock < hi;
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] += in ? v[u][k] : 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) lds[wave][k] = s;
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < NV) {
    double s = 0.0;
    for (int wv = 0; wv < kFinishBlock / 64; ++wv) s += lds[wv][threadIdx.x];
    if (threadIdx.x == 0) {
      if (energy) energy[b] = s;
    } else if (virial) {
      virial[9 * b + (threadIdx.x - 1)] = s;
    }
  }
}

// Per-atom outputs (sum of the S parts, in order), per-system energy / virial and
// per-type gradients, in one launch: blocks [0, nA) take atoms, the next B blocks
// take systems, the last 2T blocks (adjoint only) take types.
template <int MODE>
__global__ void __launch_bounds__(kFinishBlock) k_finish(Dev d, Out o, int S, int nA, double *energy, double *virial,
                                                        int nv, const double *__restrict__ eps, double *grad_sigma,
                                                        double *grad_eps) {
  __shared__ double lds[kFinishBlock / 64][kPart];
  if (!built_for(d.status, d.N, true)) return;
  const int blk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (blk < nA) {
    const int i = blk * kFinishBlock + threadIdx.x;
    if (i >= d.N) return;
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
  if (blk < nA + d.B) {
    if (MODE == kAdjoint || nv == 0) return;
    const int b = blk - nA;
    const SysDesc &sd = d.desc[b];
    const int64_t lo = static_cast<int64_t>(d.col_clu_start[sd.col_begin]) * S;
    const int64_t hi = static_cast<int64_t>(d.col_clu_start[sd.col_begin + sd.dims[0] * sd.dims[1]]) * S;
    if (nv == kPart) sum_slots<kPart>(d, lo, hi, energy, virial, b, lds);
    else sum_slots<1>(d, lo, hi, energy, virial, b, lds);
    return;
  }
  if constexpr (MODE == kAdjoint) {
    // One (sigma or eps, type) entry: sum over every wave slot of every system,
    // each scaled by its system's grad_energy.
    const int T = d.T;
    const int t = blk - nA - d.B;
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
      acc += o.grad_energy[b] * s;
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

template <bool F64, bool TABLDS, int K>
void launch_cluster_mode(int mode, dim3 grid, hipStream_t s, const Dev &d, const Consts &c, const Out &o, int S) {
  if (mode == kForces)
    hipLaunchKernelGGL((k_pair_cluster<F64, kForces, TABLDS, K>), grid, dim3(64), 0, s, d, c, o, S);
  else if (mode == kEnergy)
    hipLaunchKernelGGL((k_pair_cluster<F64, kEnergy, TABLDS, K>), grid, dim3(64), 0, s, d, c, o, S);
  else
    hipLaunchKernelGGL((k_pair_cluster<F64, kAdjoint, TABLDS, K>), grid, dim3(64), 0, s, d, c, o, S);
}

template <bool F64, bool TABLDS>
void launch_cluster_k(int K, int mode, dim3 grid, hipStream_t s, const Dev &d, const Consts &c, const Out &o, int S) {
  if (K == 8) launch_cluster_mode<F64, TABLDS, 8>(mode, grid, s, d, c, o, S);
  else launch_cluster_mode<F64, TABLDS, 4>(mode, grid, s, d, c, o, S);
}

}  // namespace

void launch_cluster_pair(const Plan &p, const Dev &d, const Consts &c, const Out &o, int mode, hipStream_t s,
                         double *energy, double *virial, const double *eps, double *grad_sigma, double *grad_eps) {
  if (p.N > 0 && p.n_clusters_max > 0) {
    const int64_t waves = p.n_clusters_max * p.split;
    const int64_t g = (waves + kXcds - 1) / kXcds * kXcds;  // a multiple of the XCD count
    const dim3 grid(static_cast<unsigned>(g));
    const bool tab = p.T <= kTabLds;
    const int K = p.cluster_size;
    timer_before(s);
    if (p.precision == NB_FP64) {
      if (tab) launch_cluster_k<true, true>(K, mode, grid, s, d, c, o, p.split);
      else launch_cluster_k<true, false>(K, mode, grid, s, d, c, o, p.split);
    } else {
      if (tab) launch_cluster_k<false, true>(K, mode, grid, s, d, c, o, p.split);
      else launch_cluster_k<false, false>(K, mode, grid, s, d, c, o, p.split);
    }
    timer_after(s);
  }
  const int nA = static_cast<int>((p.N + kFinishBlock - 1) / kFinishBlock);
  int nv = 0;
  if (mode == kForces) nv = o.want_part ? (virial ? kPart : 1) : 0;
  if (mode == kEnergy) nv = 1;
  const int extra = mode == kAdjoint ? ((grad_sigma || grad_eps) ? 2 * p.T : 0) : 0;
  const dim3 fg(static_cast<unsigned>(nA + p.B + extra));
  if (mode == kForces)
    hipLaunchKernelGGL(k_finish<kForces>, fg, dim3(kFinishBlock), 0, s, d, o, p.split, nA, energy, virial, nv, eps,
                       grad_sigma, grad_eps);
  else if (mode == kEnergy)
    hipLaunchKernelGGL(k_finish<kEnergy>, fg, dim3(kFinishBlock), 0, s, d, o, p.split, nA, energy, virial, nv, eps,
                       grad_sigma, grad_eps);
  else
    hipLaunchKernelGGL(k_finish<kAdjoint>, fg, dim3(kFinishBlock), 0, s, d, o, p.split, nA, energy, virial, nv, eps,
                       grad_sigma, grad_eps);
}

}  // namespace nb
