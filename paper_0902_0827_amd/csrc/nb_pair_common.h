// Device helpers shared by the pair kernels: system lookup, wave reductions and
// the exclusion test.
#pragma once

#include "nb_internal.h"

namespace nb {

// Index of the last system whose `field` start is <= key (systems are ordered).
template <int32_t SysDesc::*Field>
__device__ __forceinline__ int find_desc(const SysDesc *desc, int B, int key) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].*Field <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Inclusive prefix sum over the wave's lanes.
__device__ __forceinline__ int wave_incl_scan_int(int v) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Exclusive prefix sum over the wave's lanes; *total receives the sum of all lanes.
__device__ __forceinline__ int wave_excl_scan_int(int v, int *total) {
  const int incl = wave_incl_scan_int(v);
  *total = __shfl(incl, 63, 64);
  return incl - v;
}

// Is the pair (oi, oj) of original indices excluded?  Window bits of oi for
// |oj - oi| <= 64 (section 3's bitmaps); beyond that the CSR rows of both atoms
// are searched when both carry the far flag.
__device__ __forceinline__ bool pair_excluded(const uint4 &mask_i, bool far_i, int oi, int oj, int atom_begin,
                                              const uint32_t *__restrict__ excl_far,
                                              const int32_t *__restrict__ excl_off,
                                              const int32_t *__restrict__ excl_idx) {
  const int delta = oj - oi;
  if (delta >= -kWindow && delta <= kWindow) {
    const int bit = delta < 0 ? delta + kWindow : delta + kWindow - 1;
    const int wsel = bit >> 5;
    const uint32_t w = wsel == 0 ? mask_i.x : wsel == 1 ? mask_i.y : wsel == 2 ? mask_i.z : mask_i.w;
    return (w >> (bit & 31)) & 1u;
  }
  if (!far_i || excl_far[oj] == 0u) return false;
  const int il = oi - atom_begin, jl = oj - atom_begin;
  for (int k = excl_off[oi]; k < excl_off[oi + 1]; ++k)
    if (excl_idx[k] == jl) return true;
  for (int k = excl_off[oj]; k < excl_off[oj + 1]; ++k)
    if (excl_idx[k] == il) return true;
  return false;
}

// Exclusion beyond the bitmap window: the CSR rows of both atoms are searched (only
// called for atoms that carry the far flag).
__device__ __forceinline__ bool far_excluded(int oi, int oj, int atom_begin, const uint32_t *__restrict__ excl_far,
                                             const int32_t *__restrict__ excl_off,
                                             const int32_t *__restrict__ excl_idx) {
  if (excl_far[oj] == 0u) return false;
  const int il = oi - atom_begin, jl = oj - atom_begin;
  for (int k = excl_off[oi]; k < excl_off[oi + 1]; ++k)
    if (excl_idx[k] == jl) return true;
  for (int k = excl_off[oj]; k < excl_off[oj + 1]; ++k)
    if (excl_idx[k] == il) return true;
  return false;
}

}  // namespace nb
