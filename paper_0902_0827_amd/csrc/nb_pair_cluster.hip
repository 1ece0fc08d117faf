// Cluster pair kernel: one wave (one 64-lane workgroup) per i-cluster of up to 8
// consecutive sorted atoms of one (x, y) column; lane = (ii, jj) = (lane / 8, lane % 8).
//
// The paper's kernel (section 3) processes one cell per thread block and stages
// every cell within R into shared memory, one thread per i atom.  Here, for a
// 64-wide wavefront and ~10 atoms per cell, the wave instead owns 8 i atoms and
// streams the j atoms of the neighbouring columns:
//
//   1. stage: the atoms of each neighbouring column's z-window are read 64 at a
//      time (coalesced), each tested against the i-cluster's bounding box; the
//      survivors (those within R of the box) are compacted, ballot + mbcnt, into a
//      ring buffer in LDS;
//   2. pairs: whenever the ring holds 8 atoms, each lane evaluates the pair
//      (i atom ii, j atom jj), so all 64 lanes work on candidates that passed the
//      box test (about 40% of them are inside R, against ~25% for a plain cell
//      stencil);
//   3. each row of 8 lanes accumulates its i atom's force, energy, virial (and
//      adjoint sums) in registers; rows are reduced with cross-lane shuffles at
//      the end.  Every atom's sums live in one wave: no atomics, deterministic.
//
// Full shell (every pair is evaluated from both sides), as in the paper.
#include <type_traits>

#include "nb_pair_common.h"
#include "nb_pair_math.h"

namespace nb {

namespace {

constexpr int kRing = 128;    // ring buffer of staged j atoms (power of two)
constexpr int kTabLds = 16;   // type tables up to 16 x 16 are copied to LDS
constexpr int kFlush = 32;    // groups between single -> double flushes of the sums
constexpr int kXcds = 8;      // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kMaxRuns = 2 * 9 * 9;  // up to 9 x 9 neighbour columns, <= 2 z-runs each
constexpr int kRowQ = 32;     // per-row queue of in-cutoff pairs (row-compacted variant)

__device__ __forceinline__ uint32_t uabs_diff(uint32_t a, uint32_t b) {
  const int32_t d = static_cast<int32_t>(a - b);
  return d < 0 ? static_cast<uint32_t>(-static_cast<int64_t>(d)) : static_cast<uint32_t>(d);
}

// Squared distance (A^2, single precision) from a fixed-point point to a box given
// by centre and half extents, with minimum image per dimension.
__device__ __forceinline__ float box_dist2(const uint4 &p, const uint4 &ctr, const uint4 &half, const SysDesc &sd) {
  const uint32_t ax = uabs_diff(p.x, ctr.x), ay = uabs_diff(p.y, ctr.y), az = uabs_diff(p.z, ctr.z);
  const float ex = static_cast<float>(ax > half.x ? ax - half.x : 0u);
  const float ey = static_cast<float>(ay > half.y ? ay - half.y : 0u);
  const float ez = static_cast<float>(az > half.z ? az - half.z : 0u);
  return fmaf(sd.scale2f[2] * ez, ez, fmaf(sd.scale2f[1] * ey, ey, sd.scale2f[0] * ex * ex));
}

template <bool F64>
struct RingLds;

template <>
struct RingLds<false> {
  uint4 fix[kRing];    // fixed-point x, y, z, original index
  float2 qt[kRing];    // q * sqrt(k_e), type (as int bits)
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

// Row queues of the row-compacted variant: for each of the 8 i atoms, the pairs
// found inside the cutoff (displacement in fixed-point units, r^2, q'_j, type).
struct RowQLds {
  float4 d[8][kRowQ];
  float2 qt[8][kRowQ];
};
struct NoRowQ {};

template <bool F64, int MODE, bool TABLDS, bool ROWQ>
__global__ void __launch_bounds__(64) k_pair_cluster(Dev d, Consts c, Out o) {
  static_assert(!(F64 && ROWQ), "row compaction is built for the single-precision path");
  __shared__ RingLds<F64> L;
  __shared__ typename std::conditional<ROWQ, RowQLds, NoRowQ>::type RQ;
  // Workgroups are dealt to the 8 XCDs round robin; give each XCD a contiguous
  // range of clusters (neighbouring columns) so that its L2 holds their j atoms.
  const int per_xcd = static_cast<int>(gridDim.x) / kXcds;
  const int I = static_cast<int>(blockIdx.x % kXcds) * per_xcd + static_cast<int>(blockIdx.x / kXcds);
  if (!built_for(d.status, d.N, true)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(d.status, NB_STATUS_NOT_BUILT);
    return;
  }
  const int n_clu = d.col_clu_start[d.n_columns];
  if (I >= n_clu) return;  // the grid is sized by an upper bound on the cluster count
  const int lane = threadIdx.x, ii = lane >> 3, jj = lane & 7;
  const int T = d.T;
  if constexpr (TABLDS) {
    for (int k = lane; k < T * T; k += 64) {
      if constexpr (F64) L.tab[k] = d.tab64[k];
      else L.tab[k] = d.tab32[k];
    }
  }

  const int4 rec = d.clusters[I];  // first atom, count, global column, system
  const SysDesc &sd = d.desc[rec.w];
  const uint4 ctr = d.clu_ctr[I], half = d.clu_half[I];
  const int i = rec.x + ii;
  const bool ivalid = ii < rec.y;
  const int ia = ivalid ? i : rec.x;
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

  const int nx = sd.dims[0], ny = sd.dims[1], nz = sd.dims[2];
  const int kx = sd.reach[0], ky = sd.reach[1], kz = sd.reach[2];
  const int col_local = rec.z - sd.col_begin;
  const int cx = col_local / ny, cy = col_local - (col_local / ny) * ny;
  const int cz0 = static_cast<int>((static_cast<uint64_t>(d.s_fix[rec.x].z) * nz) >> 32);
  const int cz1 = static_cast<int>((static_cast<uint64_t>(d.s_fix[rec.x + rec.y - 1].z) * nz) >> 32);
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

  // Single-precision pair terms for row ii's atom, added to the lane's sums.  With
  // v false every contribution is exactly zero (no branch: the lanes stay converged).
  auto accum32 = [&](float r2f, float dxf, float dyf, float dzf, float qj, int tj, bool v) {
    if constexpr (!F64) {
      TypePair32 tp;
      const int tjv = v ? tj : 0;
      if constexpr (TABLDS) tp = L.tab[ti * T + tjv];
      else tp = d.tab32[ti * T + tjv];
      const float qjv = v ? qj : 0.f;
      const PairF32 p = pair_f32(v ? r2f : 1.0f, v ? tp.c6 : 0.f, v ? tp.c12 : 0.f, qi32 * qjv, c.betaf,
                                 c.two_beta_sqrtpif, c.mb2l2e);
      sen += p.u_lj + p.u_c;
      if constexpr (MODE != kEnergy) {
        const float ex = v ? dxf : 0.f, ey = v ? dyf : 0.f, ez = v ? dzf : 0.f;
        const float gx = p.f * ex, gy = p.f * ey, gz = p.f * ez;
        sfx += gx;
        sfy += gy;
        sfz += gz;
        if constexpr (MODE == kForces) {
          if (o.want_virial) {
            swxx = fmaf(gx, ex, swxx); swxy = fmaf(gx, ey, swxy); swxz = fmaf(gx, ez, swxz);
            swyy = fmaf(gy, ey, swyy); swyz = fmaf(gy, ez, swyz); swzz = fmaf(gz, ez, swzz);
          }
        }
      }
      if constexpr (MODE == kAdjoint) {
        sphi = fmaf(qjv, p.erfc_over_r, sphi);
        sasig = fmaf(p.dudsig_lj, tp.inv_sig, sasig);
        sbeps += p.u_lj;
      }
    }
  };

  // Row queues (row-compacted variant): per-lane copies of row ii's head and count.
  int rstart = 0, rcount = 0;
  auto round = [&]() {  // one pair per lane from its row's queue
    if constexpr (ROWQ) {
      const int avail = rcount < 8 ? rcount : 8;
      const bool v = jj < avail;
      const int q = (rstart + jj) & (kRowQ - 1);
      const float4 e = RQ.d[ii][q];
      const float2 qt = RQ.qt[ii][q];
      accum32(e.w, e.x, e.y, e.z, qt.x, __float_as_int(qt.y), v);
      rstart += avail;
      rcount -= avail;
      if (++groups >= kFlush) flush();
    }
  };

  // Evaluate pair (row ii's atom, ring entry head + jj) for navail <= 8 entries.
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
      dxd -= sd.box[0] * rint(dxd * sd.inv_box[0]);
      dyd -= sd.box[1] * rint(dyd * sd.inv_box[1]);
      dzd -= sd.box[2] * rint(dzd * sd.inv_box[2]);
      r2d = dxd * dxd + dyd * dyd + dzd * dzd;
      hit = ivalid && jv && r2d < c.rc2 && oi != oj;
    } else {
      const uint4 fj = L.fix[slot];
      qj = L.qt[slot].x;
      dxf = static_cast<float>(static_cast<int>(fi.x - fj.x));
      dyf = static_cast<float>(static_cast<int>(fi.y - fj.y));
      dzf = static_cast<float>(static_cast<int>(fi.z - fj.z));
      r2f = fmaf(sd.scale2f[2] * dzf, dzf, fmaf(sd.scale2f[1] * dyf, dyf, sd.scale2f[0] * dxf * dxf));
      hit = ivalid && jv && r2f < c.rc2f && oi != oj;
    }
    const int delta = oj - oi;
    const bool check = hit && (static_cast<unsigned>(delta + kWindow) <= 2u * kWindow || far_i);
    if (__ballot(check)) {
      if (check && pair_excluded(mask_i, far_i, oi, oj, sd.atom_begin, d.excl_far, o.excl_off, o.excl_idx))
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
      } else if constexpr (!ROWQ) {
        accum32(r2f, dxf, dyf, dzf, qj, tj, true);
      }
    }
    if constexpr (ROWQ) {
      // Compact this group's in-cutoff pairs into the rows' queues ...
      const uint64_t hm = __ballot(hit);
      const uint32_t rowbits = static_cast<uint32_t>(hm >> (8 * ii)) & 0xFFu;
      const int before = __popc(rowbits & ((1u << jj) - 1u));
      if (hit) {
        const int q = (rstart + rcount + before) & (kRowQ - 1);
        RQ.d[ii][q] = make_float4(dxf, dyf, dzf, r2f);
        RQ.qt[ii][q] = make_float2(qj, __int_as_float(tj));
      }
      rcount += __popc(rowbits);
      // ... and evaluate 8 per row once every row with an atom has 8, or when a
      // queue could not take another group.
      for (;;) {
        const bool overfull = __ballot(rcount > kRowQ - 8) != 0;
        const bool waiting = __ballot(ivalid && rcount < 8) != 0;
        if ((!overfull && waiting) || __ballot(rcount > 0) == 0) break;
        __syncthreads();
        round();
      }
    }
    head += static_cast<uint32_t>(navail);
    if constexpr (!ROWQ) {
      if (++groups >= kFlush) flush();
    }
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
    const int cb = sd.cell_begin + (x * ny + y) * nz;
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
  const int nruns = 2 * ncol;

  // Walk the runs 64 atoms at a time; the next chunk's loads are issued before the
  // current chunk is filtered and evaluated, to hide their latency.
  int base = 0, end = 0;
  auto seek = [&](int rr) {  // first non-empty run at or after rr; sets base/end
    while (rr < nruns) {
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
  int r = seek(0);
  if (r < nruns) load(base, end, fj, tj, qj, pj64, valid);
  while (r < nruns) {
    int nr = r;
    if (base + 64 < end) base += 64;
    else nr = seek(r + 1);
    uint4 fj_n = fj;
    int tj_n = tj;
    float qj_n = qj;
    double4 pj64_n = pj64;
    bool valid_n = false;
    if (nr < nruns) load(base, end, fj_n, tj_n, qj_n, pj64_n, valid_n);

    // Box filter, then compact the survivors into the ring.
    const bool keep = valid && box_dist2(fj, ctr, half, sd) < c.rc2_box;
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
    while (tail - head >= 8u) process_group(8);

    r = nr;
    fj = fj_n;
    tj = tj_n;
    qj = qj_n;
    pj64 = pj64_n;
    valid = valid_n;
  }
  if (tail != head) process_group(static_cast<int>(tail - head));
  if constexpr (ROWQ) {
    while (__ballot(rcount > 0)) {
      __syncthreads();
      round();
    }
  }
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

  // Partial sums of the whole cluster (before the row reduction: a plain wave sum).
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
      if (lane < kPart) d.partials[static_cast<int64_t>(lane) * d.n_slots + I] = lane < nv ? mine : 0.0;
    }
  }

  // Per-atom results: reduce each row over its 8 lanes.
  if constexpr (MODE == kForces) {
    fx = row8_sum(fx);
    fy = row8_sum(fy);
    fz = row8_sum(fz);
    if (jj == 0 && ivalid) {
      o.force[3 * oi + 0] = fx;
      o.force[3 * oi + 1] = fy;
      o.force[3 * oi + 2] = fz;
    }
  }
  if constexpr (MODE == kEnergy) {
    en = row8_sum(en);
    if (jj == 0 && ivalid && o.atom_energy) o.atom_energy[oi] = 0.5 * en;
  }
  if constexpr (MODE == kAdjoint) {
    const double g = o.grad_energy[rec.w];
    fx = row8_sum(fx);
    fy = row8_sum(fy);
    fz = row8_sum(fz);
    phi = row8_sum(phi);
    if (jj == 0 && ivalid) {
      if (o.grad_pos) {
        o.grad_pos[3 * oi + 0] = -g * fx;
        o.grad_pos[3 * oi + 1] = -g * fy;
        o.grad_pos[3 * oi + 2] = -g * fz;
      }
      if (o.grad_charge) o.grad_charge[oi] = g * phi;
    }
    // Per-type sums of the sigma / eps partials over the cluster's atoms.
    const double a_l = 0.5 * g * asig, b_l = 0.5 * g * beps;
    const int my_t = ivalid ? ti : -1;
    double keep_a = 0.0, keep_b = 0.0;
    uint64_t left = __ballot(my_t >= 0);
    while (left) {
      const int lead = __ffsll(static_cast<unsigned long long>(left)) - 1;
      const int tt = __shfl(my_t, lead, 64);
      const bool mine = my_t == tt;
      const double sa = wave_sum(mine ? a_l : 0.0);
      const double sb = wave_sum(mine ? b_l : 0.0);
      if (lane == tt) {
        keep_a = sa;
        keep_b = sb;
      }
      left &= ~__ballot(mine);
    }
    if (lane < T) {
      d.adj_partials[static_cast<int64_t>(lane) * d.n_slots + I] = keep_a;
      d.adj_partials[static_cast<int64_t>(T + lane) * d.n_slots + I] = keep_b;
    }
  }
}

}  // namespace

template <bool F64, bool TABLDS, bool ROWQ>
void launch_cluster_mode(int mode, dim3 grid, hipStream_t s, const Dev &d, const Consts &c, const Out &o) {
  if (mode == kForces)
    hipLaunchKernelGGL((k_pair_cluster<F64, kForces, TABLDS, ROWQ>), grid, dim3(64), 0, s, d, c, o);
  else if (mode == kEnergy)
    hipLaunchKernelGGL((k_pair_cluster<F64, kEnergy, TABLDS, ROWQ>), grid, dim3(64), 0, s, d, c, o);
  else
    hipLaunchKernelGGL((k_pair_cluster<F64, kAdjoint, TABLDS, ROWQ>), grid, dim3(64), 0, s, d, c, o);
}

void launch_cluster_pair(const Plan &p, const Dev &d, const Consts &c, const Out &o, int mode, hipStream_t s) {
  if (p.n_clusters_max == 0 || p.N == 0) return;
  const int64_t g = (p.n_clusters_max + kXcds - 1) / kXcds * kXcds;  // a multiple of the XCD count
  const dim3 grid(static_cast<unsigned>(g));
  const bool tab = p.T <= kTabLds;
  const bool rowq = p.kernel == NB_KERNEL_CLUSTER_RQ;
  if (p.precision == NB_FP64) {
    if (tab) launch_cluster_mode<true, true, false>(mode, grid, s, d, c, o);
    else launch_cluster_mode<true, false, false>(mode, grid, s, d, c, o);
  } else if (rowq) {
    if (tab) launch_cluster_mode<false, true, true>(mode, grid, s, d, c, o);
    else launch_cluster_mode<false, false, true>(mode, grid, s, d, c, o);
  } else {
    if (tab) launch_cluster_mode<false, true, false>(mode, grid, s, d, c, o);
    else launch_cluster_mode<false, false, false>(mode, grid, s, d, c, o);
  }
}

}  // namespace nb
