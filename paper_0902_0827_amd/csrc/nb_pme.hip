// Reciprocal part of the Ewald sum by smooth particle-mesh Ewald (ACEMD paper, section 3:
// the long-range electrostatics are PME with fourth-order interpolation; the method is
// that of Essmann et al., J. Chem. Phys. 103, 8577 (1995)).  With u_a = K_a x_a / L_a
// the scaled fractional coordinates and M_4 the cubic cardinal B-spline:
//
//   Q(k)   = sum_i q_i prod_a M_4(u_ai - k_a)           (periodic in k)
//   E      = k_e/(2 pi V) sum_{m != 0} C(m) |FFT(Q)(m)|^2,
//   C(m)   = exp(-pi^2 m^2/beta^2)/m^2 prod_a 9/(2 + cos(2 pi m_a/K_a))^2
//   phi    = dE/dQ = k_e/(pi V) IFFT(C FFT(Q))          (unnormalised inverse)
//   F_i    = -q_i sum_k phi(k) grad_i prod_a M_4(u_ai - k_a)
//   W_ab   = sum_m E_m [delta_ab - 2 (1 + pi^2 m^2/beta^2) m_a m_b / m^2].
//
// The factor 9/(2 + cos t)^2 is |b(m)|^2 for order 4: the Euler exponential spline's
// denominator 1/6 + (2/3) e^{it} + (1/6) e^{2it} has modulus (2 + cos t)/3.
//
// All arithmetic is FP64 (positions and charges of either precision are promoted).
// In order on the caller's stream, each kernel launched per system:
//   k_pme_spread_planes  one workgroup per x-plane, the plane accumulated in LDS (planes
//                  of up to 8192 points); else k_pme_zero and k_pme_spread, 16 lanes per
//                  atom with 4 FP64 atomic additions into the grid each;
//   D2Z FFT        (hipFFT, one batched call for all systems; a plan per grid shape,
//                  batch size and device, made on first use);
//   k_pme_convolve one thread per element of the half spectrum: C(m), the energy and
//                  virial terms (per-block partials) and the product C FFT(Q);
//   Z2D FFT        giving phi on the real grid (one batched call);
//   k_pme_gather   16 lanes per atom: its force from phi and the spline derivatives.
// k_pme_reduce then sums each system's partials in a fixed order.  The grid additions
// of the spread (LDS or global atomics) are the only ones whose order varies from run
// to run.
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "nb_internal.h"
#include "nb_pair_common.h"
#include "nb_pme.h"

namespace nb {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMinGrid = 4;     // the spline's four points must be distinct grid points
constexpr int kMaxGrid = 1024;

struct PmeSys {
  double L[3];
  double invL[3];
  double a;       // pi^2 / beta^2
  double escale;  // k_e / (2 pi V)
  int K[3];
  int H;  // K3/2 + 1: the half spectrum's last dimension
};

// Systems of one launch (at most kPmeChunk; a larger batch takes several launches per
// step).  Only what differs between systems travels here; the rest of PmeSys is formed on
// the device with the same IEEE operations as on the host (make_sys), so every system's
// constants are the ones a launch per system would have used.
constexpr int kPmeChunk = 32;
struct PmeBatch {
  int nsys;    // systems in this launch
  int first;   // batch index of its first system (grid and partial offsets)
  int K[3];
  double a;    // pi^2 / beta^2
  double ke;
  double L[kPmeChunk][3];
  int64_t a0[kPmeChunk];          // first atom of each system
  int32_t n[kPmeChunk];           // atoms of each system
  int32_t blk0[kPmeChunk + 1];    // first gather workgroup of each system (prefix sums)
};

__host__ __device__ inline PmeSys make_sys(const double L[3], const int K[3], double a, double ke) {
  PmeSys ps;
  for (int d = 0; d < 3; ++d) {
    ps.L[d] = L[d];
    ps.invL[d] = 1.0 / L[d];
    ps.K[d] = K[d];
  }
  ps.H = K[2] / 2 + 1;
  ps.a = a;
  ps.escale = ke / (2.0 * kPi * L[0] * L[1] * L[2]);
  return ps;
}

inline size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Grid cell of coordinate x: u = K (x/L mod 1), base = floor(u) in [0, K), t = u - base.
__device__ inline void grid_cell(double x, double invL, int K, int *base_out, double *t_out) {
  double f = x * invL;
  f -= floor(f);  // in [0, 1] for finite x
  const double u = f * K;
  int base = 0;
  double t;
  if (u >= 0.0 && u < K) {
    base = static_cast<int>(floor(u));
    t = u - base;
  } else if (u == K) {  // f rounded up to 1: the point K is the point 0
    t = 0.0;
  } else {  // non-finite coordinate: indices stay in range, the results are NaN
    t = u - u;
  }
  *base_out = base;
  *t_out = t;
}

// The four grid points k = base - j (mod K), j = 0..3, of coordinate x, with M_4(u - k)
// and dM_4/du at u - k = t + j, t = u - base in [0, 1).
__device__ inline void spline4(double x, double invL, int K, int idx[4], double w[4], double dw[4]) {
  int base;
  double t;
  grid_cell(x, invL, K, &base, &t);
  const double t2 = t * t, t3 = t2 * t, s = 1.0 - t;
  w[0] = t3 * (1.0 / 6.0);
  w[1] = (1.0 + 3.0 * t + 3.0 * t2 - 3.0 * t3) * (1.0 / 6.0);
  w[2] = (4.0 - 6.0 * t2 + 3.0 * t3) * (1.0 / 6.0);
  w[3] = s * s * s * (1.0 / 6.0);
  dw[0] = 0.5 * t2;
  dw[1] = 0.5 * (1.0 + 2.0 * t - 3.0 * t2);
  dw[2] = 0.5 * (3.0 * t2 - 4.0 * t);
  dw[3] = -0.5 * s * s;
#pragma unroll
  for (int j = 0; j < 4; ++j) idx[j] = base - j < 0 ? base - j + K : base - j;
}

__global__ void __launch_bounds__(kBlock) k_pme_zero(double *__restrict__ g, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * kBlock)
    g[e] = 0.0;
}

// 16 lanes per atom, one per (x, y) row of its 4 x 4 x 4 footprint: each lane adds the
// row's four z points.  Lane t of the grid takes atom t / 16 and row (t / 4 % 4, t % 4).
constexpr int kLanesPerAtom = 16;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_pme_spread(const T *__restrict__ pos, const T *__restrict__ charge, int n,
                                                       PmeSys ps, double *__restrict__ grid) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  const int i = static_cast<int>(t / kLanesPerAtom);
  if (i >= n) return;
  const int a = static_cast<int>(t >> 2) & 3, b = static_cast<int>(t) & 3;
  int ix[4], iy[4], iz[4];
  double wx[4], wy[4], wz[4], d[4];
  spline4(static_cast<double>(pos[3 * i + 0]), ps.invL[0], ps.K[0], ix, wx, d);
  spline4(static_cast<double>(pos[3 * i + 1]), ps.invL[1], ps.K[1], iy, wy, d);
  spline4(static_cast<double>(pos[3 * i + 2]), ps.invL[2], ps.K[2], iz, wz, d);
  const double qab = static_cast<double>(charge[i]) * wx[a] * wy[b];
  double *row = grid + (static_cast<int64_t>(ix[a]) * ps.K[1] + iy[b]) * ps.K[2];
#pragma unroll
  for (int c = 0; c < 4; ++c) unsafeAtomicAdd(&row[iz[c]], qab * wz[c]);
}

// One workgroup per x-plane of the grid: it reads every atom, keeps those whose
// footprint covers its plane (four planes per atom) and adds their 4 x 4 (y, z) points
// with LDS atomics into the plane held in LDS, then stores the plane.  No global
// atomics and no clearing pass.  Used when a plane fits in kPlaneMaxPoints doubles.
constexpr int kPlaneBlock = 1024;
constexpr int kPlaneMaxPoints = 8192;  // 64 KB of LDS

template <typename T>
__global__ void __launch_bounds__(kPlaneBlock) k_pme_spread_planes(const T *__restrict__ pos_all,
                                                                   const T *__restrict__ charge_all, PmeBatch pb,
                                                                   int64_t grid_points, double *__restrict__ grids) {
  extern __shared__ double plane[];
  // workgroup (system b of the launch, plane x)
  const int b = static_cast<int>(blockIdx.x) / pb.K[0];
  const int x = static_cast<int>(blockIdx.x) - b * pb.K[0];
  const PmeSys ps = make_sys(pb.L[b], pb.K, pb.a, pb.ke);
  const T *__restrict__ pos = pos_all + 3 * pb.a0[b];
  const T *__restrict__ charge = charge_all + pb.a0[b];
  const int n = pb.n[b];
  double *__restrict__ grid = grids + static_cast<int64_t>(pb.first + b) * grid_points;
  const int P = ps.K[1] * ps.K[2];
  for (int j = threadIdx.x; j < P; j += kPlaneBlock) plane[j] = 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kPlaneBlock) {
    int bx;
    double tx;
    grid_cell(static_cast<double>(pos[3 * i + 0]), ps.invL[0], ps.K[0], &bx, &tx);
    int a = bx - x;  // the atom covers plane x as its point base - a (mod K), a in [0, 4)
    if (a < 0) a += ps.K[0];
    if (a >= 4) continue;
    const double s = 1.0 - tx;
    const double wa = a == 0 ? tx * tx * tx * (1.0 / 6.0)
                    : a == 1 ? (1.0 + 3.0 * tx + 3.0 * tx * tx - 3.0 * tx * tx * tx) * (1.0 / 6.0)
                    : a == 2 ? (4.0 - 6.0 * tx * tx + 3.0 * tx * tx * tx) * (1.0 / 6.0)
                             : s * s * s * (1.0 / 6.0);
    int iy[4], iz[4];
    double wy[4], wz[4], d[4];
    spline4(static_cast<double>(pos[3 * i + 1]), ps.invL[1], ps.K[1], iy, wy, d);
    spline4(static_cast<double>(pos[3 * i + 2]), ps.invL[2], ps.K[2], iz, wz, d);
    const double qa = static_cast<double>(charge[i]) * wa;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) unsafeAtomicAdd(&plane[iy[b] * ps.K[2] + iz[c]], qa * wy[b] * wz[c]);
  }
  __syncthreads();
  double *out = grid + static_cast<int64_t>(x) * P;
  for (int j = threadIdx.x; j < P; j += kPlaneBlock) out[j] = plane[j];
}

// Signed reciprocal index of grid index i: i for i <= K/2, else i - K.
__device__ inline int signed_index(int i, int K) { return 2 * i <= K ? i : i - K; }

// (2 + cos(2 pi i / K))^2 / 9: the reciprocal of the order-4 spline factor |b(m)|^2
__device__ inline double inv_bmod2(int i, int K) {
  const double c = 2.0 + cospi(2.0 * static_cast<double>(i) / static_cast<double>(K));
  return c * c * (1.0 / 9.0);
}

__global__ void __launch_bounds__(kBlock) k_pme_convolve(double2 *__restrict__ specs, PmeBatch pb, int64_t n_spec,
                                                         double *__restrict__ partials_all, int64_t n_part_blocks) {
  __shared__ double red[kWaves][kPart];
  // workgroup (system b of the launch, block blk of its half spectrum)
  const int b = static_cast<int>(blockIdx.x / n_part_blocks);
  const int64_t blk = blockIdx.x - static_cast<int64_t>(b) * n_part_blocks;
  const PmeSys ps = make_sys(pb.L[b], pb.K, pb.a, pb.ke);
  double2 *__restrict__ spec = specs + static_cast<int64_t>(pb.first + b) * n_spec;
  double *__restrict__ partials = partials_all + static_cast<int64_t>(pb.first + b) * kPart * n_part_blocks;
  const int64_t e = blk * kBlock + threadIdx.x;
  double v[kPart] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (e < n_spec) {
    const int iz = static_cast<int>(e % ps.H);
    const int64_t r = e / ps.H;
    const int iy = static_cast<int>(r % ps.K[1]);
    const int ix = static_cast<int>(r / ps.K[1]);
    const double m[3] = {signed_index(ix, ps.K[0]) * ps.invL[0], signed_index(iy, ps.K[1]) * ps.invL[1],
                         signed_index(iz, ps.K[2]) * ps.invL[2]};
    const double m2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    double2 F = spec[e];
    if (m2 > 0.0) {
      const double inv_m2 = 1.0 / m2;
      const double C =
          exp(-ps.a * m2) * inv_m2 / (inv_bmod2(ix, ps.K[0]) * inv_bmod2(iy, ps.K[1]) * inv_bmod2(iz, ps.K[2]));
      const double em = ps.escale * C * (F.x * F.x + F.y * F.y);
      const double vf = 2.0 * (1.0 + ps.a * m2) * inv_m2;
      // The half spectrum holds each element and its conjugate partner (K - i mod K per
      // dimension) once, except in the planes iz = 0 and iz = K3/2, whose partners are
      // elements of their own.  The partner has the same |F|^2 and m^2; its signed
      // indices are -m except on a Nyquist index K/2, which stays +K/2.
      const bool pair = !(iz == 0 || 2 * iz == ps.K[2]);
      const int jx = ix == 0 ? 0 : ps.K[0] - ix, jy = iy == 0 ? 0 : ps.K[1] - iy;
      const double mp[3] = {signed_index(jx, ps.K[0]) * ps.invL[0], signed_index(jy, ps.K[1]) * ps.invL[1],
                            signed_index(ps.K[2] - iz, ps.K[2]) * ps.invL[2]};
      v[0] = pair ? 2.0 * em : em;
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double d = p == q ? 1.0 : 0.0;
          v[1 + 3 * p + q] = em * (d - vf * m[p] * m[q]) + (pair ? em * (d - vf * mp[p] * mp[q]) : 0.0);
        }
      const double sc = 2.0 * ps.escale * C;  // k_e / (pi V) C
      F.x *= sc;
      F.y *= sc;
    } else {
      F.x = 0.0;
      F.y = 0.0;
    }
    spec[e] = F;
  }
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
    partials[static_cast<int64_t>(threadIdx.x) * n_part_blocks + blk] = s;
  }
}

// 16 lanes per atom as in the spread; the row sums meet by shuffles within the 16.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pme_gather(const T *__restrict__ pos_all, const T *__restrict__ charge_all,
                                                       PmeBatch pb, int64_t grid_points,
                                                       const double *__restrict__ phis,
                                                       double *__restrict__ force_all) {
  // system of this workgroup: the last one whose first workgroup is <= blockIdx.x
  int sb = 0;
  while (sb + 1 < pb.nsys && pb.blk0[sb + 1] <= static_cast<int>(blockIdx.x)) ++sb;
  const PmeSys ps = make_sys(pb.L[sb], pb.K, pb.a, pb.ke);
  const T *__restrict__ pos = pos_all + 3 * pb.a0[sb];
  const T *__restrict__ charge = charge_all + pb.a0[sb];
  const int n = pb.n[sb];
  const double *__restrict__ phi = phis + static_cast<int64_t>(pb.first + sb) * grid_points;
  double *__restrict__ force = force_all + 3 * pb.a0[sb];
  const int64_t t = (static_cast<int64_t>(blockIdx.x) - pb.blk0[sb]) * kBlock + threadIdx.x;
  const int i_raw = static_cast<int>(t / kLanesPerAtom);
  const bool valid = i_raw < n;
  const int i = valid ? i_raw : n - 1;  // lanes past the end still join the shuffles
  const int a = static_cast<int>(t >> 2) & 3, b = static_cast<int>(t) & 3;
  int ix[4], iy[4], iz[4];
  double wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
  spline4(static_cast<double>(pos[3 * i + 0]), ps.invL[0], ps.K[0], ix, wx, dx);
  spline4(static_cast<double>(pos[3 * i + 1]), ps.invL[1], ps.K[1], iy, wy, dy);
  spline4(static_cast<double>(pos[3 * i + 2]), ps.invL[2], ps.K[2], iz, wz, dz);
  const double *row = phi + (static_cast<int64_t>(ix[a]) * ps.K[1] + iy[b]) * ps.K[2];
  double sz = 0.0, sdz = 0.0;  // sum_c phi wz[c] and sum_c phi dz[c] along the row
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double p = row[iz[c]];
    sz += p * wz[c];
    sdz += p * dz[c];
  }
  double gx = dx[a] * wy[b] * sz, gy = wx[a] * dy[b] * sz, gz = wx[a] * wy[b] * sdz;
#pragma unroll
  for (int off = kLanesPerAtom / 2; off > 0; off >>= 1) {
    gx += __shfl_xor(gx, off, kLanesPerAtom);
    gy += __shfl_xor(gy, off, kLanesPerAtom);
    gz += __shfl_xor(gz, off, kLanesPerAtom);
  }
  if (valid && (t & (kLanesPerAtom - 1)) == 0) {
    const double q = static_cast<double>(charge[i]);
    force[3 * static_cast<int64_t>(i) + 0] = -q * gx * (ps.K[0] / ps.L[0]);
    force[3 * static_cast<int64_t>(i) + 1] = -q * gy * (ps.K[1] / ps.L[1]);
    force[3 * static_cast<int64_t>(i) + 2] = -q * gz * (ps.K[2] / ps.L[2]);
  }
}

// Energy and virial of system blockIdx.x: its convolution partials in block order.
__global__ void __launch_bounds__(kBlock) k_pme_reduce(const double *__restrict__ partials, int64_t n_part_blocks,
                                                       double *energy, double *virial) {
  __shared__ double red[kWaves][kPart];
  const int b = blockIdx.x;
  const double *pb = partials + static_cast<int64_t>(b) * kPart * n_part_blocks;
  double acc[kPart];
#pragma unroll
  for (int k = 0; k < kPart; ++k) acc[k] = 0.0;
  for (int64_t q = threadIdx.x; q < n_part_blocks; q += kBlock) {
#pragma unroll
    for (int k = 0; k < kPart; ++k) acc[k] += pb[static_cast<int64_t>(k) * n_part_blocks + q];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kPart; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < kPart) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += red[w][threadIdx.x];
    if (threadIdx.x == 0) {
      if (energy) energy[b] = s;
    } else if (virial) {
      virial[9 * b + (threadIdx.x - 1)] = s;
    }
  }
}

// FFT plans, one forward (D2Z) and one inverse (Z2D) per grid shape, batch size and
// device, each transforming the B systems' grids (contiguous, one after the other) in
// one call; made on first use and kept for the life of the process (at most
// kMaxFftPlans of them).  The plans do not allocate their work buffers: every call hands
// them the work area of its own workspace, so calls on different streams with different
// workspaces share nothing but the plans' read-only tables.  The mutex covers the cache
// and, per call, setting a plan's stream and work area and enqueueing its transform.
struct FftPlans {
  hipfftHandle fwd = nullptr, inv = nullptr;
  size_t work = 0;  // bytes of work area either transform needs
};
constexpr size_t kMaxFftPlans = 32;
std::mutex g_fft_mu;
std::map<std::tuple<int, int, int, int, int>, FftPlans> g_fft;

const char *fft_error(hipfftResult r) {
  switch (r) {
    case HIPFFT_ALLOC_FAILED: return "FFT allocation failed";
    case HIPFFT_INVALID_SIZE: return "FFT size refused";
    case HIPFFT_EXEC_FAILED: return "FFT execution failed";
    default: return "FFT library error";
  }
}

// The plans for this layout on the current device, made if needed.  Returns "" or the
// reason they could not be made.  Caller holds g_fft_mu.
std::string fft_plans_locked(int B, const int K[3], int64_t grid, int64_t spec, FftPlans *out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "no current HIP device";
  const auto key = std::make_tuple(dev, K[0], K[1], K[2], B);
  auto it = g_fft.find(key);
  if (it != g_fft.end()) {
    *out = it->second;
    return "";
  }
  if (g_fft.size() >= kMaxFftPlans)
    return "more than 32 distinct (grid shape, batch size, device) FFT plans in this process";
  FftPlans p;
  int dims[3] = {K[0], K[1], K[2]};
  // contiguous grids, unit stride: K1 K2 K3 reals and K1 K2 (K3/2+1) complex values per
  // system, one system after the other
  int real_embed[3] = {K[0], K[1], K[2]};
  int spec_embed[3] = {K[0], K[1], K[2] / 2 + 1};
  const int grid_dist = static_cast<int>(grid), spec_dist = static_cast<int>(spec);
  size_t wf = 0, wi = 0;
  hipfftResult r = hipfftCreate(&p.fwd);
  if (r == HIPFFT_SUCCESS) r = hipfftSetAutoAllocation(p.fwd, 0);
  if (r == HIPFFT_SUCCESS)
    r = hipfftMakePlanMany(p.fwd, 3, dims, real_embed, 1, grid_dist, spec_embed, 1, spec_dist, HIPFFT_D2Z, B, &wf);
  if (r != HIPFFT_SUCCESS) {
    if (p.fwd) hipfftDestroy(p.fwd);
    return std::string("hipfftMakePlanMany (D2Z): ") + fft_error(r);
  }
  r = hipfftCreate(&p.inv);
  if (r == HIPFFT_SUCCESS) r = hipfftSetAutoAllocation(p.inv, 0);
  if (r == HIPFFT_SUCCESS)
    r = hipfftMakePlanMany(p.inv, 3, dims, spec_embed, 1, spec_dist, real_embed, 1, grid_dist, HIPFFT_Z2D, B, &wi);
  if (r != HIPFFT_SUCCESS) {
    hipfftDestroy(p.fwd);
    if (p.inv) hipfftDestroy(p.inv);
    return std::string("hipfftMakePlanMany (Z2D): ") + fft_error(r);
  }
  p.work = std::max(wf, wi);
  g_fft.emplace(key, p);
  *out = p;
  return "";
}

}  // namespace

std::string pme_layout(int B, const int32_t grid[3], PmeLayout *lay) {
  if (!grid) return "grid is NULL";
  for (int a = 0; a < 3; ++a)
    if (grid[a] < kMinGrid || grid[a] > kMaxGrid) return "grid sizes must be in [4, 1024]";
  PmeLayout l;
  l.B = B;
  for (int a = 0; a < 3; ++a) l.K[a] = grid[a];
  l.grid = static_cast<int64_t>(grid[0]) * grid[1] * grid[2];
  l.spec = static_cast<int64_t>(grid[0]) * grid[1] * (grid[2] / 2 + 1);
  if (l.grid > (int64_t{1} << 28)) return "grid larger than 2^28 points";
  if (static_cast<int64_t>(B) * l.grid > (int64_t{1} << 31)) return "batch grids larger than 2^31 points";
  l.conv_blocks = (l.spec + kBlock - 1) / kBlock;
  size_t off = 0;
  l.real = off;
  off = align256(off + sizeof(double) * static_cast<size_t>(B) * l.grid);
  l.cplx = off;
  off = align256(off + 2 * sizeof(double) * static_cast<size_t>(B) * l.spec);
  l.partials = off;
  off = align256(off + sizeof(double) * static_cast<size_t>(B) * kPart * l.conv_blocks);
  l.work = off;
  l.total = off;
  *lay = l;
  return "";
}

std::string pme_attach_plans(PmeLayout *lay) {
  FftPlans plans;
  {
    std::lock_guard<std::mutex> lock(g_fft_mu);
    const std::string why = fft_plans_locked(lay->B, lay->K, lay->grid, lay->spec, &plans);
    if (!why.empty()) return why;
  }
  lay->work_bytes = plans.work;
  lay->total = align256(lay->work + plans.work);
  return "";
}

hipError_t launch_pme(const PmeLayout &lay, const nb_system *sys, double beta, double ke, void *ws, double *force,
                      double *energy, double *virial, hipStream_t s, std::string *err) {
  char *base = static_cast<char *>(ws);
  double *real = reinterpret_cast<double *>(base + lay.real);
  double2 *cplx = reinterpret_cast<double2 *>(base + lay.cplx);
  double *partials = reinterpret_cast<double *>(base + lay.partials);
  void *work = lay.work_bytes ? static_cast<void *>(base + lay.work) : nullptr;
  auto stride_blocks = [](int64_t n) {
    return dim3(static_cast<unsigned>(std::min<int64_t>((n + kBlock - 1) / kBlock, 65536)));
  };
  FftPlans plans;
  {
    std::lock_guard<std::mutex> lock(g_fft_mu);
    const std::string why = fft_plans_locked(lay.B, lay.K, lay.grid, lay.spec, &plans);
    if (!why.empty()) {
      *err = why;
      return hipErrorUnknown;
    }
  }
  if (plans.work > lay.work_bytes) {  // the workspace was sized for another device's plans
    *err = "workspace sized for FFT plans of another device";
    return hipErrorUnknown;
  }
  const int64_t plane_points = static_cast<int64_t>(lay.K[1]) * lay.K[2];
  const bool planes = plane_points <= kPlaneMaxPoints;
  const bool f64 = sys->pos_is_f64 != 0;
  const double a = kPi * kPi / (beta * beta);
  // the launch descriptor of systems [first, first + nsys)
  auto chunk = [&](int first, int nsys) {
    PmeBatch pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.nsys = nsys;
    pb.first = first;
    for (int d = 0; d < 3; ++d) pb.K[d] = lay.K[d];
    pb.a = a;
    pb.ke = ke;
    int32_t blocks = 0;
    for (int k = 0; k < nsys; ++k) {
      const int b = first + k;
      for (int d = 0; d < 3; ++d) pb.L[k][d] = sys->box[3 * b + d];
      pb.a0[k] = sys->atom_offset[b];
      pb.n[k] = static_cast<int32_t>(sys->atom_offset[b + 1] - sys->atom_offset[b]);
      pb.blk0[k] = blocks;
      blocks += static_cast<int32_t>((static_cast<int64_t>(pb.n[k]) * kLanesPerAtom + kBlock - 1) / kBlock);
    }
    pb.blk0[nsys] = blocks;
    return pb;
  };
  const dim3 blk(kBlock);
  // charge grids
  if (!planes)
    hipLaunchKernelGGL(k_pme_zero, stride_blocks(lay.grid * lay.B), dim3(kBlock), 0, s, real, lay.grid * lay.B);
  for (int first = 0; first < lay.B; first += kPmeChunk) {
    const PmeBatch pb = chunk(first, std::min(kPmeChunk, lay.B - first));
    if (planes) {
      const dim3 gp(static_cast<unsigned>(lay.K[0] * pb.nsys)), bp(kPlaneBlock);
      const size_t lds = sizeof(double) * static_cast<size_t>(plane_points);
      if (f64)
        hipLaunchKernelGGL(k_pme_spread_planes<double>, gp, bp, lds, s, static_cast<const double *>(sys->pos),
                           static_cast<const double *>(sys->charge), pb, lay.grid, real);
      else
        hipLaunchKernelGGL(k_pme_spread_planes<float>, gp, bp, lds, s, static_cast<const float *>(sys->pos),
                           static_cast<const float *>(sys->charge), pb, lay.grid, real);
    } else {
      for (int k = 0; k < pb.nsys; ++k) {  // grids too large for a plane in LDS: per system
        const int64_t n = pb.n[k];
        if (n == 0) continue;
        const PmeSys ps = make_sys(pb.L[k], pb.K, a, ke);
        double *g = real + static_cast<int64_t>(first + k) * lay.grid;
        const dim3 ga(static_cast<unsigned>((n * kLanesPerAtom + kBlock - 1) / kBlock));
        if (f64)
          hipLaunchKernelGGL(k_pme_spread<double>, ga, blk, 0, s, static_cast<const double *>(sys->pos) + 3 * pb.a0[k],
                             static_cast<const double *>(sys->charge) + pb.a0[k], static_cast<int>(n), ps, g);
        else
          hipLaunchKernelGGL(k_pme_spread<float>, ga, blk, 0, s, static_cast<const float *>(sys->pos) + 3 * pb.a0[k],
                             static_cast<const float *>(sys->charge) + pb.a0[k], static_cast<int>(n), ps, g);
      }
    }
  }
  {
    std::lock_guard<std::mutex> lock(g_fft_mu);
    hipfftResult r = hipfftSetStream(plans.fwd, s);
    if (r == HIPFFT_SUCCESS) r = hipfftSetWorkArea(plans.fwd, work);
    if (r == HIPFFT_SUCCESS) r = hipfftExecD2Z(plans.fwd, real, reinterpret_cast<hipfftDoubleComplex *>(cplx));
    if (r != HIPFFT_SUCCESS) {
      *err = std::string("hipfftExecD2Z: ") + fft_error(r);
      return hipErrorUnknown;
    }
  }
  for (int first = 0; first < lay.B; first += kPmeChunk) {  // convolution, energy and virial partials
    const PmeBatch pb = chunk(first, std::min(kPmeChunk, lay.B - first));
    hipLaunchKernelGGL(k_pme_convolve, dim3(static_cast<unsigned>(lay.conv_blocks * pb.nsys)), blk, 0, s, cplx, pb,
                       lay.spec, partials, lay.conv_blocks);
  }
  {
    std::lock_guard<std::mutex> lock(g_fft_mu);
    hipfftResult r = hipfftSetStream(plans.inv, s);
    if (r == HIPFFT_SUCCESS) r = hipfftSetWorkArea(plans.inv, work);
    if (r == HIPFFT_SUCCESS) r = hipfftExecZ2D(plans.inv, reinterpret_cast<hipfftDoubleComplex *>(cplx), real);
    if (r != HIPFFT_SUCCESS) {
      *err = std::string("hipfftExecZ2D: ") + fft_error(r);
      return hipErrorUnknown;
    }
  }
  for (int first = 0; first < lay.B; first += kPmeChunk) {  // forces from the potential grids
    const PmeBatch pb = chunk(first, std::min(kPmeChunk, lay.B - first));
    if (pb.blk0[pb.nsys] == 0) continue;
    const dim3 ga(static_cast<unsigned>(pb.blk0[pb.nsys]));
    if (f64)
      hipLaunchKernelGGL(k_pme_gather<double>, ga, blk, 0, s, static_cast<const double *>(sys->pos),
                         static_cast<const double *>(sys->charge), pb, lay.grid, real, force);
    else
      hipLaunchKernelGGL(k_pme_gather<float>, ga, blk, 0, s, static_cast<const float *>(sys->pos),
                         static_cast<const float *>(sys->charge), pb, lay.grid, real, force);
  }
  if (energy || virial)
    hipLaunchKernelGGL(k_pme_reduce, dim3(static_cast<unsigned>(lay.B)), dim3(kBlock), 0, s, partials,
                       lay.conv_blocks, energy, virial);
  return hipGetLastError();
}

}  // namespace nb
