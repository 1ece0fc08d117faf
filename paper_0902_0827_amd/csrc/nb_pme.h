// Reciprocal part of the Ewald sum by smooth particle-mesh Ewald (nb_pme.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "nbhip.h"

namespace nb {

// Byte offsets into the reciprocal-space workspace (all 256-aligned): per system the
// real grid (K1 K2 K3 doubles: charges, then the potential), its half-spectrum
// (K1 K2 (K3/2+1) complex doubles) and the per-block energy and virial partials; then
// the work area of the FFT plans.
struct PmeLayout {
  int B = 0;
  int K[3] = {0, 0, 0};
  int64_t grid = 0, spec = 0, conv_blocks = 0;
  size_t real = 0, cplx = 0, partials = 0, work = 0, work_bytes = 0, total = 0;
};

// Fills `lay` for this batch and grid, without the FFT work area (host only, no HIP
// call); returns "" or the reason the grid is refused.
std::string pme_layout(int B, const int32_t grid[3], PmeLayout *lay);

// Makes (or finds) the FFT plans of this layout on the current device and adds their
// work area to it; returns "" or the reason the FFT library refused them.
std::string pme_attach_plans(PmeLayout *lay);

// Launches the whole reciprocal-space evaluation on `s`.  `err` receives the failing
// step's name when the FFT library refuses a plan or a transform.
hipError_t launch_pme(const PmeLayout &lay, const nb_system *sys, double beta, double ke, void *ws, double *force,
                      double *energy, double *virial, hipStream_t s, std::string *err);

}  // namespace nb
