// Ewald corrections around the real-space pair term (ACEMD paper, section 3: the
// electrostatics are PME, and the pair kernels compute its real-space part).  The
// reciprocal part counts every pair, excluded ones included, and every charge with
// itself; these corrections take out
//
//   for every excluded pair {i, j} (the union of both atoms' exclusion rows, at any
//   distance, minimum image):   u_ij = -k_e q_i q_j erf(beta r) / r
//                               (at r = 0 its limit -k_e q_i q_j 2 beta / sqrt(pi))
//   for every atom:             -k_e beta / sqrt(pi) q_i^2
//   for every scaled 1-4 pair {i, j} that is not excluded (the union of both 1-4 rows,
//   within the 64-index window): (1 - s14_coul) u_ij, so that with the pair kernels'
//   s14_coul erfc term and the reciprocal part the whole Coulomb interaction of the pair
//   is s14_coul k_e q_i q_j / r.
//
// The force on i from pair {i, j} is g_ij d_ij with
//   g_ij = k_e q_i q_j [(2 beta / sqrt(pi)) exp(-beta^2 r^2) / r^2 - erf(beta r) / r^3].
//
// A few pairs per atom: FP64 arithmetic on the caller's own arrays for both precisions.
// One thread per atom (caller's order) gathers its force from
//   * the partners inside its 128-bit exclusion window, from the bitmaps of the cell
//     build (which hold the union of both rows), each pair seen from both sides, and
//   * the far entries of its own row (|j - i| > 64), counted in full on this side when
//     the partner's row does not list the atom, by halves otherwise;
// a second pass adds each far pair listed in one row only to the other atom's force
// (FP64 atomics: the only additions whose order can vary, and only for atoms with more
// than one such pair).  Energies and virials go to per-block partials that a third
// launch reduces per system in a fixed order.
#include "nb_internal.h"
#include "nb_pair_common.h"

namespace nb {

namespace {

constexpr int kEwaldReduceBlock = 256;
constexpr double kTwoOverSqrtPi = 1.12837916709551257390;  // 2 / sqrt(pi)

template <typename T>
__device__ inline double3 load3(const T *p, int64_t i) {
  return make_double3(static_cast<double>(p[3 * i + 0]), static_cast<double>(p[3 * i + 1]),
                      static_cast<double>(p[3 * i + 2]));
}

// Minimum-image displacement x_i - x_j of an orthorhombic box.
__device__ inline double3 min_image(double3 xi, double3 xj, const SysDesc &sd) {
  double3 dd = make_double3(xi.x - xj.x, xi.y - xj.y, xi.z - xj.z);
  dd.x -= sd.box[0] * rint(dd.x * sd.inv_box[0]);
  dd.y -= sd.box[1] * rint(dd.y * sd.inv_box[1]);
  dd.z -= sd.box[2] * rint(dd.z * sd.inv_box[2]);
  return dd;
}

// u_ij and g_ij of one excluded pair, kqq = k_e q_i q_j.
__device__ inline void excl_pair(double kqq, double r2, double beta, double *u, double *g) {
  if (r2 > 0.0) {
    const double r = sqrt(r2);
    const double inv_r = 1.0 / r;  // the one division
    const double e = erf(beta * r);
    *u = -kqq * e * inv_r;
    *g = kqq * inv_r * inv_r * (beta * kTwoOverSqrtPi * exp(-beta * beta * r2) - e * inv_r);
  } else {
    *u = -kqq * beta * kTwoOverSqrtPi;
    *g = 0.0;
  }
}

// Does the exclusion row of atom `a` (global index; entries are local to its system)
// list the local index `bl`?
__device__ inline bool row_lists(const int32_t *__restrict__ off, const int32_t *__restrict__ idx, int a, int bl) {
  for (int k = off[a]; k < off[a + 1]; ++k)
    if (idx[k] == bl) return true;
  return false;
}

// Is entry k of the row of atom `a` (global index) a repeat of an earlier entry of it?
__device__ inline bool repeated(const int32_t *__restrict__ off, const int32_t *__restrict__ idx, int a, int k) {
  for (int k2 = off[a]; k2 < k; ++k2)
    if (idx[k2] == idx[k]) return true;
  return false;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_ewald_atoms(Dev d, const T *__restrict__ pos, const T *__restrict__ charge,
                                                        const int32_t *__restrict__ excl_off,
                                                        const int32_t *__restrict__ excl_idx, double ke, double beta,
                                                        double w14, double *force) {
  __shared__ double red[kWaves][kPart];
  const int blk = blockIdx.x;
  if (!built_for(d.status, d.N, false, false)) {
    if (blk == 0 && threadIdx.x == 0) atomicOr(d.status, NB_STATUS_NOT_BUILT);
    return;
  }
  const int b = find_desc<&SysDesc::blk_begin>(d.desc, d.B, blk);
  const SysDesc &sd = d.desc[b];
  const int i = sd.atom_begin + (blk - sd.blk_begin) * kBlock + static_cast<int>(threadIdx.x);
  double v[kPart] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // energy, then the virial row-major
  if (i < sd.atom_end) {
    const double3 xi = load3(pos, i);
    const double qi = static_cast<double>(charge[i]);
    double3 f = make_double3(0, 0, 0);
    // pair {i, j} with weight wp; w = this side's share of energy and virial
    auto add = [&](int j, double w, double wp) {
      const double3 dd = min_image(xi, load3(pos, j), sd);
      const double r2 = dd.x * dd.x + dd.y * dd.y + dd.z * dd.z;
      double u, g;
      excl_pair(wp * ke * qi * static_cast<double>(charge[j]), r2, beta, &u, &g);
      f.x += g * dd.x;
      f.y += g * dd.y;
      f.z += g * dd.z;
      const double dv[3] = {dd.x, dd.y, dd.z};
      v[0] += w * u;
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) v[1 + 3 * a + c] += w * dv[a] * g * dv[c];
    };
    // window partners: bits 0-63 are j - i = -64..-1, bits 64-127 are 1..64
    const uint4 m = d.excl_mask[i];
    const uint32_t words[4] = {m.x, m.y, m.z, m.w};
    for (int wd = 0; wd < 4; ++wd) {
      uint32_t bits = words[wd];
      while (bits) {
        const int bit = 32 * wd + __ffs(static_cast<int>(bits)) - 1;
        bits &= bits - 1u;
        add(bit < kWindow ? i + bit - kWindow : i + bit - kWindow + 1, 0.5, 1.0);
      }
    }
    // scaled 1-4 partners that are not excluded, weight 1 - s14_coul
    if (d.p14_mask && w14 != 0.0) {
      const uint4 m14 = d.p14_mask[i];
      const uint32_t w14s[4] = {m14.x & ~m.x, m14.y & ~m.y, m14.z & ~m.z, m14.w & ~m.w};
      for (int wd = 0; wd < 4; ++wd) {
        uint32_t bits = w14s[wd];
        while (bits) {
          const int bit = 32 * wd + __ffs(static_cast<int>(bits)) - 1;
          bits &= bits - 1u;
          add(bit < kWindow ? i + bit - kWindow : i + bit - kWindow + 1, 0.5, w14);
        }
      }
    }
    // far entries of the atom's own row
    if (d.excl_far[i]) {
      const int il = i - sd.atom_begin, nb = sd.atom_end - sd.atom_begin;
      for (int k = excl_off[i]; k < excl_off[i + 1]; ++k) {
        const int jl = excl_idx[k];
        const int delta = jl - il;
        if (delta >= -kWindow && delta <= kWindow) continue;  // in the window (or the atom itself)
        if (jl < 0 || jl >= nb) continue;                     // not an atom of the system (the build flags it)
        if (repeated(excl_off, excl_idx, i, k)) continue;
        const int j = sd.atom_begin + jl;
        add(j, row_lists(excl_off, excl_idx, j, il) ? 0.5 : 1.0, 1.0);
      }
    }
    v[0] -= ke * beta * 0.5 * kTwoOverSqrtPi * qi * qi;  // self term
    force[3 * static_cast<int64_t>(i) + 0] = f.x;
    force[3 * static_cast<int64_t>(i) + 1] = f.y;
    force[3 * static_cast<int64_t>(i) + 2] = f.z;
  }
  // per-block partials, summed in a fixed order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPart; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kPart) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += red[w][threadIdx.x];
    d.partials[static_cast<int64_t>(threadIdx.x) * d.n_slots + blk] = s;
  }
}

// Far pairs listed in one row only: the other atom's share of the force.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ewald_far(Dev d, const T *__restrict__ pos, const T *__restrict__ charge,
                                                      const int32_t *__restrict__ excl_off,
                                                      const int32_t *__restrict__ excl_idx, double ke, double beta,
                                                      double *force) {
  const int blk = blockIdx.x;
  if (!built_for(d.status, d.N, false, false)) return;
  // The build flags every atom with an exclusion beyond the window and, with the first
  // of them, the status word: without that bit no atom has work here (one scalar load
  // per workgroup instead of a flag per atom).
  using ConstU32 = const __attribute__((address_space(4))) uint32_t;
  if ((((ConstU32 *)d.status)[0] & NB_STATUS_FAR_EXCLUSION) == 0u) return;
  const int b = find_desc<&SysDesc::blk_begin>(d.desc, d.B, blk);
  const SysDesc &sd = d.desc[b];
  const int i = sd.atom_begin + (blk - sd.blk_begin) * kBlock + static_cast<int>(threadIdx.x);
  if (i >= sd.atom_end || !d.excl_far[i]) return;
  const int il = i - sd.atom_begin, nb = sd.atom_end - sd.atom_begin;
  const double3 xi = load3(pos, i);
  const double qi = static_cast<double>(charge[i]);
  for (int k = excl_off[i]; k < excl_off[i + 1]; ++k) {
    const int jl = excl_idx[k];
    const int delta = jl - il;
    if (delta >= -kWindow && delta <= kWindow) continue;
    if (jl < 0 || jl >= nb) continue;
    if (repeated(excl_off, excl_idx, i, k)) continue;
    const int j = sd.atom_begin + jl;
    if (row_lists(excl_off, excl_idx, j, il)) continue;  // the partner's own thread has it
    const double3 dd = min_image(xi, load3(pos, j), sd);
    double u, g;
    excl_pair(ke * qi * static_cast<double>(charge[j]), dd.x * dd.x + dd.y * dd.y + dd.z * dd.z, beta, &u, &g);
    unsafeAtomicAdd(&force[3 * static_cast<int64_t>(j) + 0], -g * dd.x);
    unsafeAtomicAdd(&force[3 * static_cast<int64_t>(j) + 1], -g * dd.y);
    unsafeAtomicAdd(&force[3 * static_cast<int64_t>(j) + 2], -g * dd.z);
  }
}

// Energy and virial of system b: its blocks' partials in order.
__global__ void __launch_bounds__(kEwaldReduceBlock) k_ewald_reduce(Dev d, double *energy, double *virial) {
  __shared__ double lds[kEwaldReduceBlock / 64][kPart];
  if (!built_for(d.status, d.N, false, false)) return;
  const int b = blockIdx.x;
  const int64_t lo = d.desc[b].blk_begin;
  const int64_t hi = b + 1 < d.B ? d.desc[b + 1].blk_begin : d.n_blocks;
  double acc[kPart];
#pragma unroll
  for (int k = 0; k < kPart; ++k) acc[k] = 0.0;
  for (int64_t q = lo + threadIdx.x; q < hi; q += kEwaldReduceBlock) {
#pragma unroll
    for (int k = 0; k < kPart; ++k) acc[k] += d.partials[static_cast<int64_t>(k) * d.n_slots + q];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPart; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) lds[wave][k] = s;
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < kPart) {
    double s = 0.0;
    for (int w = 0; w < kEwaldReduceBlock / 64; ++w) s += lds[w][threadIdx.x];
    if (threadIdx.x == 0) {
      if (energy) energy[b] = s;
    } else if (virial) {
      virial[9 * b + (threadIdx.x - 1)] = s;
    }
  }
}

}  // namespace

hipError_t launch_ewald(const Plan &p, const Dev &d, const nb_system *sys, double *force, double *energy,
                        double *virial, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(p.n_blocks)), block(kBlock);
  const double ke = p.ke, beta = p.beta;
  // A batch without atoms launches no per-atom work, but its systems' energies and
  // virials are still written (zeros: a system without blocks sums to nothing).
  if (p.n_blocks == 0) {
  } else if (sys->pos_is_f64) {
    const double *pos = static_cast<const double *>(sys->pos);
    const double *q = static_cast<const double *>(sys->charge);
    hipLaunchKernelGGL(k_ewald_atoms<double>, grid, block, 0, s, d, pos, q, sys->excl_offset, sys->excl_index, ke,
                       beta, 1.0 - p.s14_c, force);
    hipLaunchKernelGGL(k_ewald_far<double>, grid, block, 0, s, d, pos, q, sys->excl_offset, sys->excl_index, ke,
                       beta, force);
  } else {
    const float *pos = static_cast<const float *>(sys->pos);
    const float *q = static_cast<const float *>(sys->charge);
    hipLaunchKernelGGL(k_ewald_atoms<float>, grid, block, 0, s, d, pos, q, sys->excl_offset, sys->excl_index, ke,
                       beta, 1.0 - p.s14_c, force);
    hipLaunchKernelGGL(k_ewald_far<float>, grid, block, 0, s, d, pos, q, sys->excl_offset, sys->excl_index, ke,
                       beta, force);
  }
  if (energy || virial)
    hipLaunchKernelGGL(k_ewald_reduce, dim3(static_cast<unsigned>(p.B)), dim3(kEwaldReduceBlock), 0, s, d, energy,
                       virial);
  return hipGetLastError();
}

}  // namespace nb
