// Molecular dynamics around the force evaluation (nb_md.hip): workspace layout and the
// host entry points behind nb_md_workspace_bytes, nb_md_forces and nb_md_run.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "nb_internal.h"
#include "nb_pme.h"

namespace nb {

// Byte offsets into the MD workspace (all 256-aligned): the nonbonded workspace at 0,
// then the reciprocal-space workspace (absent without a PME grid), four force arrays
// (short-range, Ewald corrections, reciprocal, bonded; N*3 doubles each), the energy
// accumulators (5 per system: short-range, corrections, reciprocal, bonded, kinetic),
// the per-atom role (0 free atom, 1 water O, 2 water H) and the MD status word.
struct MdLayout {
  bool pme = false;
  size_t nb = 0, pme_ws = 0, f_nb = 0, f_corr = 0, f_rec = 0, f_bond = 0, energy = 0, role = 0, status = 0;
  size_t total = 0;
};

struct MdPlan {
  Plan p;
  PmeLayout pl;
  MdLayout ml;
};

// Validates (system, params, md) and fills the plan; attaches the FFT plans when a PME
// grid is given (a current HIP device is then needed).  Returns NB_OK or an error code
// with *why set.
nb_status md_plan(const nb_system *sys, const nb_params *prm, const nb_md_params *md, MdPlan *plan, std::string *why);

// Checks the topology's host-visible fields against the plan; "" when usable.
std::string md_check_topology(const MdPlan &mp, const nb_md_topology *topo);

hipError_t md_forces(const MdPlan &mp, const nb_system *sys, const nb_md_topology *topo, const nb_md_params *md,
                     void *ws, double *force, double *energy, hipStream_t s, std::string *err);

hipError_t md_run(const MdPlan &mp, const nb_system *sys, const nb_md_topology *topo, const nb_md_params *md,
                  void *ws, double *vel, int64_t first_step, int64_t n_steps, double *energy, hipStream_t s,
                  std::string *err);

}  // namespace nb
