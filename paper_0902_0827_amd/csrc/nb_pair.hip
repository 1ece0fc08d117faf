// Per-atom pair kernel (ACEMD paper, section 3: every atom's force is the sum
// over the atoms of all cells within R of its own cell, the full neighbour shell,
// with the pair term F_ij not reused as F_ji).
//
// One lane per i atom in sorted (cell) order; the lane walks the stencil of
// cells around its own cell -- for each neighbouring (x, y) column one or two
// contiguous runs of z-cells, i.e. contiguous runs of sorted atoms -- and reads
// the j atoms through the cache.  Each lane owns its atom's sums, so no atomics
// are needed and the result is deterministic.  The same source serves the FP64
// path (double positions, minimum image by rint) and the mixed path (32-bit
// fixed-point positions whose wrapped difference is the minimum image, single-
// precision pair terms, double accumulation), and three outputs: forces (with
// per-block energy/virial partials), energies, and the adjoint.
#include "nb_internal.h"
#include "nb_pair_common.h"
#include "nb_pair_math.h"

namespace nb {

namespace {

template <bool F64, int MODE>
__global__ void __launch_bounds__(kBlock) k_pair_atom(Dev d, Consts c, Out o) {
  __shared__ double red[kWaves][2 * NB_MAX_TYPES > kPart ? 2 * NB_MAX_TYPES : kPart];
  const int blk = blockIdx.x;
  if (!built_for(d.status, d.N, false, F64)) {
    if (blk == 0 && threadIdx.x == 0) atomicOr(d.status, NB_STATUS_NOT_BUILT);
    return;
  }
  const int b = find_desc<&SysDesc::blk_begin>(d.desc, d.B, blk);
  const SysDesc &sd = d.desc[b];
  const int i = sd.atom_begin + (blk - sd.blk_begin) * kBlock + static_cast<int>(threadIdx.x);
  const bool active = i < sd.atom_end;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  double fx = 0, fy = 0, fz = 0, en = 0, phi = 0, asig = 0, beps = 0;
  double wxx = 0, wxy = 0, wxz = 0, wyy = 0, wyz = 0, wzz = 0;
  int oi = 0, ti = 0;
  if (active) {
    const uint4 fi = d.s_fix[i];
    oi = static_cast<int>(fi.w);
    const uint4 mask_i = d.excl_mask[oi];
    const bool far_i = d.excl_far[oi] != 0u;
    ti = d.s_type[i];
    const TypePair64 *row64 = d.tab64 + ti * d.T;
    const TypePair32 *row32 = d.tab32 + ti * d.T;
    double4 pi64 = make_double4(0, 0, 0, 0);
    float qi32 = 0.f;
    if constexpr (F64) pi64 = d.s_pos64[i];
    else qi32 = d.s_q32[i];
    const double qi64 = F64 ? pi64.w * c.ke : 0.0;
    const int nx = sd.dims[0], ny = sd.dims[1], nz = sd.dims[2];
    const int kx = sd.reach[0], ky = sd.reach[1], kz = sd.reach[2];
    const int cx = static_cast<int>((static_cast<uint64_t>(fi.x) * nx) >> 32);
    const int cy = static_cast<int>((static_cast<uint64_t>(fi.y) * ny) >> 32);
    const int cz = static_cast<int>((static_cast<uint64_t>(fi.z) * nz) >> 32);
    // Small boxes: when the stencil is at least as wide as the grid, visit every
    // cell of that dimension once (the minimum image picks the right copy).
    const bool allx = 2 * kx + 1 >= nx, ally = 2 * ky + 1 >= ny, allz = 2 * kz + 1 >= nz;
    const int xn = allx ? nx : 2 * kx + 1, yn = ally ? ny : 2 * ky + 1;

    auto visit = [&](int j) {
      const uint4 fj = d.s_fix[j];
      const int oj = static_cast<int>(fj.w);
      if constexpr (F64) {
        const double4 pj = d.s_pos64[j];
        double dx = pi64.x - pj.x, dy = pi64.y - pj.y, dz = pi64.z - pj.z;
        dx -= sd.box[0] * rint(dx * sd.inv_box[0]);
        dy -= sd.box[1] * rint(dy * sd.inv_box[1]);
        dz -= sd.box[2] * rint(dz * sd.inv_box[2]);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < c.rc2) || j == i) return;
        if (pair_excluded(mask_i, far_i, oi, oj, sd.atom_begin, d.excl_far, o.excl_off, o.excl_idx)) return;
        const TypePair64 tp = row64[d.s_type[j]];
        const PairF64 p = pair_f64(r2, tp.c6, tp.c12, qi64 * pj.w, c.beta, c.two_beta_sqrtpi, c.erfc_short != 0);
        en += p.u_lj + p.u_c;
        if constexpr (MODE != kEnergy) {
          fx += p.f * dx;
          fy += p.f * dy;
          fz += p.f * dz;
        }
        if constexpr (MODE == kForces) {
          wxx += p.f * dx * dx; wxy += p.f * dx * dy; wxz += p.f * dx * dz;
          wyy += p.f * dy * dy; wyz += p.f * dy * dz; wzz += p.f * dz * dz;
        }
        if constexpr (MODE == kAdjoint) {
          phi += pj.w * p.erfc_over_r;
          asig += p.dudsig_lj * tp.inv_sig;
          beps += p.u_lj;
        }
      } else {
        const int ix = static_cast<int>(fi.x - fj.x);
        const int iy = static_cast<int>(fi.y - fj.y);
        const int iz = static_cast<int>(fi.z - fj.z);
        const float dx = static_cast<float>(ix), dy = static_cast<float>(iy), dz = static_cast<float>(iz);
        const float r2 = fmaf(sd.scale2f[2] * dz, dz, fmaf(sd.scale2f[1] * dy, dy, sd.scale2f[0] * dx * dx));
        if (!(r2 < c.rc2f) || j == i) return;
        if (pair_excluded(mask_i, far_i, oi, oj, sd.atom_begin, d.excl_far, o.excl_off, o.excl_idx)) return;
        const TypePair32 tp = row32[d.s_type[j]];
        const float qj = d.s_q32[j];
        const PairF32 p = pair_f32(r2, tp.c6, tp.c12, qi32 * qj, c.betaf, c.two_beta_sqrtpif, c.mb2l2e);
        en += static_cast<double>(p.u_lj + p.u_c);
        const double f = static_cast<double>(p.f);
        const double ddx = ix, ddy = iy, ddz = iz;  // exact: fixed-point units
        if constexpr (MODE != kEnergy) {
          fx += f * ddx;
          fy += f * ddy;
          fz += f * ddz;
        }
        if constexpr (MODE == kForces) {
          wxx += f * ddx * ddx; wxy += f * ddx * ddy; wxz += f * ddx * ddz;
          wyy += f * ddy * ddy; wyz += f * ddy * ddz; wzz += f * ddz * ddz;
        }
        if constexpr (MODE == kAdjoint) {
          phi += static_cast<double>(qj * p.erfc_over_r);
          asig += static_cast<double>(p.dudsig_lj * tp.inv_sig);
          beps += static_cast<double>(p.u_lj);
        }
      }
    };
    auto run = [&](int c0, int c1) {  // cells [c0, c1) of this system, as global ids
      const int j1 = d.cell_start[c1];
      for (int j = d.cell_start[c0]; j < j1; ++j) visit(j);
    };

    for (int ox = 0; ox < xn; ++ox) {
      int x = allx ? ox : cx - kx + ox;
      x += x < 0 ? nx : (x >= nx ? -nx : 0);
      for (int oy = 0; oy < yn; ++oy) {
        int y = ally ? oy : cy - ky + oy;
        y += y < 0 ? ny : (y >= ny ? -ny : 0);
        const int base = sd.cell_begin + (x * ny + y) * nz;
        if (allz) {
          run(base, base + nz);
        } else {
          const int z0 = cz - kz, z1 = cz + kz + 1;  // [z0, z1)
          if (z0 < 0) {
            run(base + z0 + nz, base + nz);
            run(base, base + z1);
          } else if (z1 > nz) {
            run(base + z0, base + nz);
            run(base, base + z1 - nz);
          } else {
            run(base + z0, base + z1);
          }
        }
      }
    }
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
  }

  // Per-atom outputs in the caller's order.
  if (active) {
    if constexpr (MODE == kForces) {
      o.force[3 * oi + 0] = fx;
      o.force[3 * oi + 1] = fy;
      o.force[3 * oi + 2] = fz;
    }
    if constexpr (MODE == kEnergy) {
      if (o.atom_energy) o.atom_energy[oi] = 0.5 * en;
    }
    if constexpr (MODE == kAdjoint) {
      const double g = o.grad_energy[b];
      if (o.grad_pos) {
        o.grad_pos[3 * oi + 0] = -g * fx;
        o.grad_pos[3 * oi + 1] = -g * fy;
        o.grad_pos[3 * oi + 2] = -g * fz;
      }
      if (o.grad_charge) o.grad_charge[oi] = g * phi;
      asig *= 0.5 * g;
      beps *= 0.5 * g;
    }
  }

  // Per-block partial sums (fixed reduction order: deterministic).
  if constexpr (MODE == kForces || MODE == kEnergy) {
    if (!o.want_part) return;
    double v[kPart] = {0.5 * en, 0.5 * wxx, 0.5 * wxy, 0.5 * wxz, 0.5 * wxy, 0.5 * wyy,
                       0.5 * wyz, 0.5 * wxz, 0.5 * wyz, 0.5 * wzz};
    const int nv = MODE == kForces ? kPart : 1;
    for (int k = 0; k < nv; ++k) {
      const double s = wave_sum(v[k]);
      if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kPart) {
      double s = 0;
      if (static_cast<int>(threadIdx.x) < nv)
        for (int w = 0; w < kWaves; ++w) s += red[w][threadIdx.x];
      d.partials[static_cast<int64_t>(threadIdx.x) * d.n_slots + blk] = s;
    }
  } else {
    // Per-type sums of the sigma and eps partials: each wave reduces over the
    // distinct types it holds, then waves are combined in a fixed order.
    const int T = d.T;
    for (int k = threadIdx.x; k < kWaves * 2 * NB_MAX_TYPES; k += kBlock) (&red[0][0])[k] = 0.0;
    __syncthreads();
    const int my_t = active ? ti : -1;
    uint64_t left = __ballot(my_t >= 0);
    while (left) {
      const int lead = __ffsll(static_cast<unsigned long long>(left)) - 1;
      const int tt = __shfl(my_t, lead, 64);
      const bool mine = my_t == tt;
      const double sa = wave_sum(mine ? asig : 0.0);
      const double sb = wave_sum(mine ? beps : 0.0);
      if (lane == 0) {
        red[wave][tt] = sa;
        red[wave][NB_MAX_TYPES + tt] = sb;
      }
      left &= ~__ballot(mine);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 2 * T; t += kBlock) {
      const int col = t < T ? t : NB_MAX_TYPES + (t - T);
      double s = 0;
      for (int w = 0; w < kWaves; ++w) s += red[w][col];
      d.adj_partials[static_cast<int64_t>(t) * d.n_slots + blk] = s;
    }
  }
}

__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < kWaves; ++w) s += lds[w];
  return s;
}

// Range of partial-sum slots owned by system b: its per-atom-kernel blocks, or
// its clusters (known on the device only, from the column scan).
__device__ __forceinline__ void partial_range(const Dev &d, int cluster, const SysDesc &sd, int *lo, int *hi) {
  if (cluster) {
    *lo = d.col_clu_start[sd.col_begin];
    *hi = d.col_clu_start[sd.col_begin + sd.dims[0] * sd.dims[1]];
  } else {
    *lo = sd.blk_begin;
    *hi = sd.blk_begin + (sd.atom_end - sd.atom_begin + kBlock - 1) / kBlock;
  }
}

// Energy and virial of system b = sum of its partials, in a fixed order: each
// thread sums a strided subset of slots (all NV components, independent loads in
// flight), then waves and the block are combined in a fixed order.
constexpr int kReduceBlock = 1024;

template <int NV>
__global__ void __launch_bounds__(kReduceBlock) k_reduce_sys(Dev d, double *energy, double *virial, int cluster) {
  __shared__ double lds[kReduceBlock / 64][NV];
  if (!built_for(d.status, d.N, cluster != 0, false)) return;
  const int b = blockIdx.x;
  const SysDesc &sd = d.desc[b];
  int lo, hi;
  partial_range(d, cluster, sd, &lo, &hi);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int q = lo + threadIdx.x; q < hi; q += kReduceBlock) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += d.partials[static_cast<int64_t>(k) * d.n_slots + q];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) lds[wave][k] = s;
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < NV) {
    double s = 0.0;
    for (int w = 0; w < kReduceBlock / 64; ++w) s += lds[w][threadIdx.x];
    if (threadIdx.x == 0) {
      if (energy) energy[b] = s;
    } else if (virial) {
      virial[9 * b + (threadIdx.x - 1)] = s;
    }
  }
}

// Per-type parameter gradients: sum the (already g-scaled) partials of every slot;
// one workgroup per (sigma or eps, type) entry, fixed reduction order.
__global__ void __launch_bounds__(kBlock) k_reduce_types(Dev d, const double *__restrict__ eps,
                                                         double *grad_sigma, double *grad_eps, int cluster) {
  __shared__ double lds[kWaves];
  if (!built_for(d.status, d.N, cluster != 0, false)) return;
  const int T = d.T;
  const int t = blockIdx.x;  // 0 .. 2T-1
  const int64_t n = cluster ? d.col_clu_start[d.n_columns] : d.n_blocks;
  double s = 0;
  for (int64_t q = threadIdx.x; q < n; q += kBlock) s += d.adj_partials[static_cast<int64_t>(t) * d.n_slots + q];
  s = block_sum(s, lds);
  if (threadIdx.x != 0) return;
  if (t < T) {
    if (grad_sigma) grad_sigma[t] = s;
  } else {
    const int tt = t - T;
    if (grad_eps) grad_eps[tt] = eps[tt] > 0.0 ? s / eps[tt] : 0.0;
  }
}

Consts make_consts(const Plan &p) {
  Consts c;
  c.rc2 = p.cutoff * p.cutoff;
  c.beta = p.beta;
  c.two_beta_sqrtpi = 2.0 * p.beta / 1.7724538509055160273;  // 2 beta / sqrt(pi)
  c.ke = p.ke;
  c.sqrt_ke = sqrt(p.ke);
  c.rc2f = static_cast<float>(c.rc2);
  c.betaf = static_cast<float>(p.beta);
  c.two_beta_sqrtpif = static_cast<float>(c.two_beta_sqrtpi);
  c.mb2l2e = static_cast<float>(-p.beta * p.beta * 1.4426950408889634074);  // -beta^2 log2(e)
  c.rc2_box = static_cast<float>(c.rc2 * 1.0001);  // generous: the box filter may only keep extra atoms
  c.erfc_short = p.beta * p.cutoff <= kErfcxShortMax ? 1 : 0;
  c.s14_lj = p.s14_lj;
  c.s14_c = p.s14_c;
  if (p.switch_on > 0.0) {
    c.sw_on2 = p.switch_on * p.switch_on;
    c.sw_inv = 1.0 / (c.rc2 - c.sw_on2);
  } else {
    c.sw_on2 = c.rc2;
    c.sw_inv = 0.0;
  }
  c.s14_ljf = static_cast<float>(c.s14_lj);
  c.s14_cf = static_cast<float>(c.s14_c);
  c.sw_on2f = static_cast<float>(c.sw_on2);
  c.sw_invf = static_cast<float>(c.sw_inv);
  c.tab_inv_h = p.table ? static_cast<float>(p.table_n / p.cutoff) : 0.f;
  c.tab_last = p.table ? static_cast<float>(p.table_n - 1) : 0.f;
  return c;
}

Out base_out(const nb_system *sys) {
  Out o{};
  o.excl_off = sys->excl_offset;
  o.excl_idx = sys->excl_index;
  return o;
}

template <int MODE>
void launch_pair(const Plan &p, const Dev &d, const Out &o, hipStream_t s) {
  const Consts c = make_consts(p);
  if (p.n_blocks == 0) return;
  timer_before(s);
  if (p.precision == NB_FP64)
    hipLaunchKernelGGL((k_pair_atom<true, MODE>), dim3(static_cast<unsigned>(p.n_blocks)), dim3(kBlock), 0, s, d, c, o);
  else
    hipLaunchKernelGGL((k_pair_atom<false, MODE>), dim3(static_cast<unsigned>(p.n_blocks)), dim3(kBlock), 0, s, d, c, o);
  timer_after(s);
}

// The force VJP's vector in sorted order: vsort[s] = v[o] for the atom o at sorted
// position s; on the mixed path each component times the system's fixed-point unit L/2^32,
// so that its product with a fixed-point displacement is in Angstrom.
__global__ void __launch_bounds__(kBlock) k_vjp_prep(Dev d, const double *__restrict__ v, int f64) {
  const int64_t s = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (s >= d.N || !built_for(d.status, d.N, false, false)) return;
  const int o = static_cast<int>(d.s_fix[s].w);
  const SysDesc &sd = d.desc[d.atom_fix[o].w];
  const double sx = f64 ? 1.0 : sd.scale[0], sy = f64 ? 1.0 : sd.scale[1], sz = f64 ? 1.0 : sd.scale[2];
  d.vsort[s] = make_double4(v[3 * static_cast<int64_t>(o)] * sx, v[3 * static_cast<int64_t>(o) + 1] * sy,
                            v[3 * static_cast<int64_t>(o) + 2] * sz, 0.0);
}

}  // namespace

hipError_t launch_force_vjp(const Plan &p, const Dev &d, const nb_system *sys, const double *v,
                            double *grad_charge, double *grad_sigma, double *grad_eps, hipStream_t s) {
  Out o = base_out(sys);
  o.grad_charge = grad_charge;
  o.vjp_v = v;
  if (p.N > 0)
    hipLaunchKernelGGL(k_vjp_prep, dim3(static_cast<unsigned>((p.N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d, v,
                       p.precision == NB_FP64 ? 1 : 0);
  launch_cluster_pair(p, d, make_consts(p), o, kVJP, s, nullptr, nullptr, sys->lj_eps, grad_sigma, grad_eps);
  return hipGetLastError();
}

hipError_t launch_forces(const Plan &p, const Dev &d, const nb_system *sys, double *force, double *energy,
                         double *virial, hipStream_t s) {
  Out o = base_out(sys);
  o.force = force;
  o.want_part = (energy || virial) ? 1 : 0;
  o.want_virial = virial ? 1 : 0;
  if (uses_clusters(p.kernel)) {
    launch_cluster_pair(p, d, make_consts(p), o, kForces, s, energy, virial, nullptr, nullptr, nullptr);
    return hipGetLastError();
  }
  launch_pair<kForces>(p, d, o, s);
  if (o.want_part) {
    const int cl = uses_clusters(p.kernel) ? 1 : 0;
    if (virial) hipLaunchKernelGGL(k_reduce_sys<kPart>, dim3(p.B), dim3(kReduceBlock), 0, s, d, energy, virial, cl);
    else hipLaunchKernelGGL(k_reduce_sys<1>, dim3(p.B), dim3(kReduceBlock), 0, s, d, energy, virial, cl);
  }
  return hipGetLastError();
}

hipError_t launch_energy(const Plan &p, const Dev &d, const nb_system *sys, double *energy,
                         double *atom_energy, hipStream_t s) {
  Out o = base_out(sys);
  o.atom_energy = atom_energy;
  o.want_part = 1;
  if (uses_clusters(p.kernel)) {
    launch_cluster_pair(p, d, make_consts(p), o, kEnergy, s, energy, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError();
  }
  launch_pair<kEnergy>(p, d, o, s);
  hipLaunchKernelGGL(k_reduce_sys<1>, dim3(p.B), dim3(kReduceBlock), 0, s, d, energy, static_cast<double *>(nullptr),
                     uses_clusters(p.kernel) ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_backward(const Plan &p, const Dev &d, const nb_system *sys, const double *grad_energy,
                           double *grad_pos, double *grad_charge, double *grad_sigma, double *grad_eps,
                           hipStream_t s) {
  Out o = base_out(sys);
  o.grad_pos = grad_pos;
  o.grad_charge = grad_charge;
  o.grad_energy = grad_energy;
  if (uses_clusters(p.kernel)) {
    launch_cluster_pair(p, d, make_consts(p), o, kAdjoint, s, nullptr, nullptr, sys->lj_eps, grad_sigma, grad_eps);
    return hipGetLastError();
  }
  launch_pair<kAdjoint>(p, d, o, s);
  if (grad_sigma || grad_eps)
    hipLaunchKernelGGL(k_reduce_types, dim3(2 * p.T), dim3(kBlock), 0, s, d, sys->lj_eps, grad_sigma, grad_eps,
                       uses_clusters(p.kernel) ? 1 : 0);
  return hipGetLastError();
}

}  // namespace nb
