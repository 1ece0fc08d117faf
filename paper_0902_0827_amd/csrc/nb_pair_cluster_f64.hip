// Double-precision instantiations of the cluster pair kernel.
#include "nb_pair_cluster.h"

namespace nb {

void launch_cluster_pair_f64(const Plan &p, const Dev &d, const Consts &c, const Out &o, int mode, bool half,
                             hipStream_t s) {
  launch_cluster_pair_prec<true>(p, d, c, o, mode, half, s);
}

}  // namespace nb
