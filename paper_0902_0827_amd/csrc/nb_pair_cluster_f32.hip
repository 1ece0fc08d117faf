// Mixed-precision (FP32 pair arithmetic) instantiations of the cluster pair kernel,
// and the finishing pass shared by both precisions.
#include "nb_pair_cluster.h"

namespace nb {

void launch_cluster_pair_f64(const Plan &p, const Dev &d, const Consts &c, const Out &o, int mode, bool half,
                             hipStream_t s);

void launch_cluster_pair(const Plan &p, const Dev &d, const Consts &c, const Out &o, int mode, hipStream_t s,
                         double *energy, double *virial, const double *eps, double *grad_sigma, double *grad_eps) {
  // the adjoint and the force VJP stay full-shell
  const bool half = p.kernel == NB_KERNEL_CLUSTER_HALF && mode != kAdjoint && mode != kVJP;
  if (p.precision == NB_FP64) launch_cluster_pair_f64(p, d, c, o, mode, half, s);
  else launch_cluster_pair_prec<false>(p, d, c, o, mode, half, s);
  // With one item per cluster the full-shell kernel has written the per-atom outputs
  // itself; the half-shell kernel's accumulators are always copied out here.
  const int blocksA = static_cast<int>((p.N + kFinishBlock - 1) / kFinishBlock);
  const int nA = half ? ((mode == kForces || o.atom_energy) ? blocksA : 0) : (p.split == 1 ? 0 : blocksA);
  int nv = 0;
  if (mode == kForces) nv = o.want_part ? (virial ? kPart : 1) : 0;
  if (mode == kEnergy) nv = 1;
  const int extra = (mode == kAdjoint || mode == kVJP) ? ((grad_sigma || grad_eps) ? 2 * p.T : 0) : 0;
  const dim3 fg(static_cast<unsigned>(nA + kPart * p.B + extra));
  const uint32_t key = static_cast<uint32_t>(p.cluster_size) | (static_cast<uint32_t>(p.split) << 8);
  if (mode == kForces)
    hipLaunchKernelGGL(k_finish<kForces>, fg, dim3(kFinishBlock), 0, s, d, o, p.split, nA, energy, virial, nv, eps,
                       grad_sigma, grad_eps, half ? 1 : 0, key);
  else if (mode == kEnergy)
    hipLaunchKernelGGL(k_finish<kEnergy>, fg, dim3(kFinishBlock), 0, s, d, o, p.split, nA, energy, virial, nv, eps,
                       grad_sigma, grad_eps, half ? 1 : 0, key);
  else if (mode == kVJP)
    hipLaunchKernelGGL(k_finish<kVJP>, fg, dim3(kFinishBlock), 0, s, d, o, p.split, nA, energy, virial, nv, eps,
                       grad_sigma, grad_eps, 0, key);
  else
    hipLaunchKernelGGL(k_finish<kAdjoint>, fg, dim3(kFinishBlock), 0, s, d, o, p.split, nA, energy, virial, nv, eps,
                       grad_sigma, grad_eps, 0, key);
}

}  // namespace nb
