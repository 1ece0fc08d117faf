// Molecular dynamics around the force evaluation (section 3: NVT production runs
// evaluate bonded and nonbonded forces, integrate with velocity Verlet under a Langevin
// thermostat, use PME electrostatics and constrain bonds to hydrogen; Table 5 gives
// their ns/day at a 4 fs step with PME every step).
//
// One step, from positions x, velocities v and the forces F(x) (c = exp(-gamma dt/2),
// xi and xi' standard normal, s_i^2 = kT/m_i; Bussi and Parrinello's Langevin form of
// velocity Verlet):
//   v <- c v + sqrt(1 - c^2) s_i xi;  v <- v + (dt/2) F/m
//   x' <- x + dt v, constrained;  v <- (x' - x)/dt
//   F <- F(x');  v <- v + (dt/2) F/m;  v <- c v + sqrt(1 - c^2) s_i xi';  v constrained
// The second half of step s and the first half of step s + 1 use the same forces, so
// inside a run they are one launch (k_md_integrate<kEndStart>).
//
// Rigid 3-site waters are the constrained molecules.  Their positions: the constrained
// displacement of each atom is a sum of the pre-move bond vectors times multipliers,
// which the water's three lanes find by Newton's method on the three length equations
// (a 3 x 3 solve per iteration; quadratic convergence from zero takes 3-5 iterations at
// MD displacements).  Their velocities: the three multipliers that remove the relative
// velocity along each bond solve one 3 x 3 linear system.  Both are the solutions of the
// SHAKE and RATTLE equations (Ryckaert, Ciccotti and Berendsen 1977; Andersen 1983),
// computed directly instead of by their one-constraint-at-a-time iteration.
//
// The thermostat's normals come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// SC'11), counter (atom, step mod 2^32, step div 2^32, half), key (seed mod 2^32, seed
// div 2^32); words u_k -> uniforms (u_k + 1/2)/2^32 -> Box-Muller: x, y from (u_0, u_1),
// z from (u_2, u_3).
//
// Units: Angstrom, ps, g/mol, kJ/mol, K: F/m is 100 A/ps^2 per (kJ/mol/A)/(g/mol).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "nb_md.h"
#include "nb_pair_common.h"

namespace nb {

namespace {

constexpr double kAccel = 100.0;          // (kJ/mol/A)/(g/mol) in A/ps^2
constexpr double kBoltzmann = 8.314462618e-3;  // molar gas constant, kJ/mol/K
constexpr double kKineticUnit = 0.01;     // g/mol A^2/ps^2 in kJ/mol
constexpr int kNewtonMax = 12;
constexpr int kWatersPerWave = 21;  // three lanes each
constexpr int kMdBlock = 256;
constexpr uint32_t kMdStatusBad = NB_STATUS_BAD_TOPOLOGY;

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

enum MdPhase : int { kStart = 1, kEnd = 2, kEndStart = 3 };

struct MdArgs {
  double *pos, *vel, *f_bond;
  const double *f_nb, *f_corr, *f_rec;  // f_corr and f_rec null without the reciprocal part
  const double *mass;
  const uint8_t *role;
  const SysDesc *desc;
  int B;
  int64_t N;
  double dt, c, noise_var;  // noise_var = (1 - c^2) 100 k_B T: times 1/m, the variance added to v
  double r_oh2, r_hh2;
  uint32_t key0, key1;
  int64_t step_end, step_start;  // the step a kEnd half finishes, the step a kStart half begins
  int thermostat;                // 0: gamma = 0, no noise is drawn
  const int32_t *water_o;
  int64_t n_waters;
};

__device__ inline int system_of(const SysDesc *desc, int B, int64_t atom) {
  return find_desc<&SysDesc::atom_begin>(desc, B, static_cast<int>(atom));
}

__device__ inline double minimage(double d, double L, double inv_L) { return d - L * rint(d * inv_L); }

// Philox4x32-10.
__device__ inline uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ inline double3 normals(const MdArgs &k, int64_t atom, int64_t step, uint32_t half) {
  const uint4 u = philox(make_uint4(static_cast<uint32_t>(atom), static_cast<uint32_t>(step),
                                    static_cast<uint32_t>(static_cast<uint64_t>(step) >> 32), half),
                         k.key0, k.key1);
  constexpr double s = 1.0 / 4294967296.0;
  const double u0 = (u.x + 0.5) * s, u1 = (u.y + 0.5) * s, u2 = (u.z + 0.5) * s, u3 = (u.w + 0.5) * s;
  const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
  double s1, c1;
  sincospi(2.0 * u1, &s1, &c1);
  return make_double3(r01 * c1, r01 * s1, r23 * cospi(2.0 * u3));
}

__device__ inline double dot3(const double (&a)[3], const double (&b)[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Solves the 3 x 3 system A x = r by Cramer's rule.
__device__ inline void solve3(const double (&A)[3][3], const double (&r)[3], double (&x)[3]) {
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  const double inv = 1.0 / det;
  x[0] = (r[0] * c00 + A[0][1] * (A[1][2] * r[2] - r[1] * A[2][2]) + A[0][2] * (r[1] * A[2][1] - A[1][1] * r[2])) * inv;
  x[1] = (A[0][0] * (r[1] * A[2][2] - A[1][2] * r[2]) + r[0] * c01 + A[0][2] * (A[1][0] * r[2] - r[1] * A[2][0])) * inv;
  x[2] = (A[0][0] * (A[1][1] * r[2] - r[1] * A[2][1]) + A[0][1] * (r[1] * A[2][0] - A[1][0] * r[2]) + r[0] * c02) * inv;
}

// Constraint p joins atoms (P0[p], P1[p]) of the water (0 = O, 1 = H1, 2 = H2).  Moving
// atom a by w_a sum_p m_p sigma_pa s_p (sigma_pa = +1 for the first atom of p, -1 for the
// second) changes the bond vector of constraint q by sum_p m_p C[q][p] s_p with
// C[q][p] = w_i sigma_pi - w_j sigma_pj for q = (i, j).
struct WaterCoupling {
  double C[3][3];
  __device__ explicit WaterCoupling(const double (&w)[3]) {
    C[0][0] = w[0] + w[1]; C[0][1] = w[0];        C[0][2] = -w[1];
    C[1][0] = w[0];        C[1][1] = w[0] + w[2]; C[1][2] = w[2];
    C[2][0] = -w[1];       C[2][1] = w[2];        C[2][2] = w[1] + w[2];
  }
};

// The move of atom a: w_a sum_p m_p sigma_pa s_p (component c).
__device__ inline double multiplier_move(int a, double wa, const double (&m)[3], const double (&s)[3][3], int c) {
  return a == 0 ? wa * (m[0] * s[0][c] + m[1] * s[1][c])
       : a == 1 ? wa * (-m[0] * s[0][c] + m[2] * s[2][c])
                : wa * (-m[1] * s[1][c] - m[2] * s[2][c]);
}

__device__ inline void bond_vectors(const double (&y)[3][3], double (&s)[3][3]) {
  for (int c = 0; c < 3; ++c) {
    s[0][c] = y[0][c] - y[1][c];
    s[1][c] = y[0][c] - y[2][c];
    s[2][c] = y[1][c] - y[2][c];
  }
}

// v <- c v + sqrt(noise_var / m) xi for one atom.
__device__ inline void thermostat(const MdArgs &k, double (&v)[3], double w, int64_t atom, int64_t step,
                                  uint32_t half) {
  const double3 z = normals(k, atom, step, half);
  const double sd = sqrt(k.noise_var * w);
  v[0] = k.c * v[0] + sd * z.x;
  v[1] = k.c * v[1] + sd * z.y;
  v[2] = k.c * v[2] + sd * z.z;
}

// Reads atom `at`'s position, velocity, summed force and inverse mass; zeroes its bonded
// force for the next evaluation.
__device__ inline void load_atom(const MdArgs &k, int64_t at, double (&x)[3], double (&v)[3], double (&f)[3],
                                 double &w) {
  w = 1.0 / k.mass[at];
  for (int c = 0; c < 3; ++c) {
    const int64_t e = 3 * at + c;
    x[c] = k.pos[e];
    v[c] = k.vel[e];
    double fs = k.f_nb[e] + k.f_bond[e];
    if (k.f_corr) fs += k.f_corr[e] + k.f_rec[e];
    f[c] = fs;
    k.f_bond[e] = 0.0;
  }
}

// A free atom (one thread).
template <int PH>
__device__ inline void integrate_free(const MdArgs &k, int64_t i) {
  double x[3], v[3], f[3], w;
  load_atom(k, i, x, v, f, w);
  const double hdt = 0.5 * k.dt * kAccel;
  if constexpr ((PH & kEnd) != 0) {
    for (int c = 0; c < 3; ++c) v[c] += hdt * f[c] * w;
    if (k.thermostat) thermostat(k, v, w, i, k.step_end, 1u);
  }
  if constexpr ((PH & kStart) != 0) {
    if (k.thermostat) thermostat(k, v, w, i, k.step_start, 0u);
    for (int c = 0; c < 3; ++c) {
      v[c] += hdt * f[c] * w;
      x[c] += k.dt * v[c];
      k.pos[3 * i + c] = x[c];
    }
  }
  for (int c = 0; c < 3; ++c) k.vel[3 * i + c] = v[c];
}

// A rigid water: three consecutive lanes (base, base + 1, base + 2 of one wave), lane a
// holding atom O + a.  Each lane draws its own atom's noise; the molecule's multipliers
// are solved by all three lanes alike from the values shuffled between them, and each
// lane moves its own atom.  Lanes with valid = false only take part in the shuffles.
template <int PH>
__device__ inline void integrate_water(const MdArgs &k, int64_t o, int a, int base, bool valid) {
  double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, f[3] = {0, 0, 0}, w = 1.0;
  int b = 0;
  if (valid) {
    load_atom(k, o + a, x, v, f, w);
    b = system_of(k.desc, k.B, o);
  }
  const double L[3] = {k.desc[b].box[0], k.desc[b].box[1], k.desc[b].box[2]};
  const double iL[3] = {k.desc[b].inv_box[0], k.desc[b].inv_box[1], k.desc[b].inv_box[2]};
  // own position relative to the O atom (minimum image within the molecule); every shuffle
  // runs on all lanes (a lane that skips one leaves its value unreadable to the others)
  double y[3];
  for (int c = 0; c < 3; ++c) {
    const double xo = __shfl(x[c], base, 64);
    y[c] = a == 0 ? 0.0 : minimage(x[c] - xo, L[c], iL[c]);
  }
  double W[3], Y[3][3];
  for (int q = 0; q < 3; ++q) {
    W[q] = __shfl(w, base + q, 64);
    for (int c = 0; c < 3; ++c) Y[q][c] = __shfl(y[c], base + q, 64);
  }
  const WaterCoupling cp(W);
  double s[3][3];
  bond_vectors(Y, s);  // the bond vectors at the current positions
  const double hdt = 0.5 * k.dt * kAccel;

  if constexpr ((PH & kEnd) != 0) {
    for (int c = 0; c < 3; ++c) v[c] += hdt * f[c] * w;
    if (k.thermostat && valid) thermostat(k, v, w, o + a, k.step_end, 1u);
    // velocity constraints: (v_i - v_j) . s_q = 0 for the three bonds
    double V[3][3];
    for (int q = 0; q < 3; ++q)
      for (int c = 0; c < 3; ++c) V[q][c] = __shfl(v[c], base + q, 64);
    const int P0[3] = {0, 0, 1}, P1[3] = {1, 2, 2};
    double A[3][3], r[3], mu[3];
    for (int q = 0; q < 3; ++q) {
      double dv[3];
      for (int c = 0; c < 3; ++c) dv[c] = V[P0[q]][c] - V[P1[q]][c];
      r[q] = -dot3(dv, s[q]);
      for (int p = 0; p < 3; ++p) A[q][p] = cp.C[q][p] * dot3(s[p], s[q]);
    }
    solve3(A, r, mu);
    for (int c = 0; c < 3; ++c) v[c] += multiplier_move(a, w, mu, s, c);
  }

  if constexpr ((PH & kStart) != 0) {
    if (k.thermostat && valid) thermostat(k, v, w, o + a, k.step_start, 0u);
    for (int c = 0; c < 3; ++c) v[c] += hdt * f[c] * w;
    // positions: yc = y + dt v + w_a sum_p m_p sigma_pa s_p with the three lengths held
    double YU[3][3];
    for (int q = 0; q < 3; ++q)
      for (int c = 0; c < 3; ++c) YU[q][c] = __shfl(y[c] + k.dt * v[c], base + q, 64);
    const double d2[3] = {k.r_oh2, k.r_oh2, k.r_hh2};
    double m[3] = {0.0, 0.0, 0.0};
    for (int it = 0; it < kNewtonMax; ++it) {
      double yc[3][3];
      for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 3; ++c) yc[q][c] = YU[q][c] + multiplier_move(q, W[q], m, s, c);
      double u[3][3];
      bond_vectors(yc, u);
      double g[3], J[3][3], dm[3];
      double worst = 0.0;
      for (int q = 0; q < 3; ++q) {
        g[q] = -(dot3(u[q], u[q]) - d2[q]);
        worst = fmax(worst, fabs(g[q]) / d2[q]);
        for (int p = 0; p < 3; ++p) J[q][p] = 2.0 * cp.C[q][p] * dot3(u[q], s[p]);
      }
      if (!(worst >= 2e-15)) break;  // converged (or not a number: nothing more to gain)
      solve3(J, g, dm);
      m[0] += dm[0];
      m[1] += dm[1];
      m[2] += dm[2];
    }
    const double inv_dt = 1.0 / k.dt;
    for (int c = 0; c < 3; ++c) {
      const double dx = YU[a][c] + multiplier_move(a, w, m, s, c) - y[c];
      x[c] += dx;
      v[c] = dx * inv_dt;
    }
    if (valid)
      for (int c = 0; c < 3; ++c) k.pos[3 * (o + a) + c] = x[c];
  }
  if (valid)
    for (int c = 0; c < 3; ++c) k.vel[3 * (o + a) + c] = v[c];
}

// Blocks [0, water_blocks) take the waters, 21 per wave (lanes 3u, 3u + 1, 3u + 2 for
// water u; lane 63 idle); the other blocks take the free atoms, one thread per atom.
template <int PH>
__global__ void __launch_bounds__(kMdBlock) k_md_integrate(MdArgs k, unsigned water_blocks) {
  if (blockIdx.x < water_blocks) {
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kMdBlock + threadIdx.x) >> 6;
    const int grp = lane / 3, a = lane - 3 * grp;
    const int64_t w = wave * kWatersPerWave + grp;
    bool valid = grp < kWatersPerWave && w < k.n_waters;
    int64_t o = 0;
    if (valid) {
      o = k.water_o[w];
      valid = o >= 0 && o + 2 < k.N && k.role[o] == 1;  // the waters k_md_roles accepted
      if (!valid) o = 0;
    }
    integrate_water<PH>(k, o, a, 3 * grp, valid);
    return;
  }
  const int64_t i = static_cast<int64_t>(blockIdx.x - water_blocks) * kMdBlock + threadIdx.x;
  if (i >= k.N || k.role[i] != 0) return;  // water atoms are the water lanes' own
  integrate_free<PH>(k, i);
}

// Clears the roles, the bonded forces, the energy accumulators and the MD status.
__global__ void k_md_setup(uint8_t *role, double *f_bond, double *energy, int n_energy, uint32_t *md_status,
                           int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kMdBlock + threadIdx.x;
  if (i < N) {
    role[i] = 0;
    f_bond[3 * i] = 0.0;
    f_bond[3 * i + 1] = 0.0;
    f_bond[3 * i + 2] = 0.0;
  }
  if (i < n_energy) energy[i] = 0.0;
  if (i == 0) *md_status = 0u;
}

// Marks every water's atoms (after k_md_setup); a water whose atoms are not three
// consecutive atoms of one system is skipped (its atoms stay free) and reported.
__global__ void k_md_roles(uint8_t *role, const int32_t *__restrict__ water_o, int64_t n_waters, const SysDesc *desc,
                           int B, int64_t N, uint32_t *md_status) {
  const int64_t w = static_cast<int64_t>(blockIdx.x) * kMdBlock + threadIdx.x;
  if (w >= n_waters) return;
  const int64_t o = water_o[w];
  if (o < 0 || o + 2 >= N || system_of(desc, B, o) != system_of(desc, B, o + 2)) {
    atomicOr(md_status, kMdStatusBad);
    return;
  }
  role[o] = 1;
  role[o + 1] = 2;
  role[o + 2] = 2;
}

struct BondedArgs {
  const double *pos;
  double *f, *energy;  // energy [B] or null
  const int32_t *bond_atoms, *angle_atoms;
  const double *bond_k, *bond_r0, *angle_k, *angle_t0;
  int64_t n_bonds, n_angles, N;
  const SysDesc *desc;
  int B;
  uint32_t *md_status;
};

__device__ inline void add_force(double *f, int64_t a, const double (&g)[3]) {
  atomicAdd(&f[3 * a + 0], g[0]);
  atomicAdd(&f[3 * a + 1], g[1]);
  atomicAdd(&f[3 * a + 2], g[2]);
}

// Harmonic bonds E = k (r - r0)^2 and angles E = k (theta - theta0)^2 (theta at the middle
// atom), minimum image; one thread per term, the forces added by FP64 atomics.
__global__ void __launch_bounds__(kMdBlock) k_md_bonded(BondedArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kMdBlock + threadIdx.x;
  if (t >= a.n_bonds + a.n_angles) return;
  const bool is_bond = t < a.n_bonds;
  const int na = is_bond ? 2 : 3;
  int64_t at[3] = {0, 0, 0};
  for (int m = 0; m < na; ++m)
    at[m] = is_bond ? a.bond_atoms[2 * t + m] : a.angle_atoms[3 * (t - a.n_bonds) + m];
  for (int m = 0; m < na; ++m)
    if (at[m] < 0 || at[m] >= a.N) {
      atomicOr(a.md_status, kMdStatusBad);
      return;
    }
  const int b = system_of(a.desc, a.B, at[0]);
  for (int m = 1; m < na; ++m)
    if (system_of(a.desc, a.B, at[m]) != b) {
      atomicOr(a.md_status, kMdStatusBad);
      return;
    }
  const SysDesc &sd = a.desc[b];
  auto delta = [&](int64_t p, int64_t q, double (&d)[3]) {
    for (int c = 0; c < 3; ++c) d[c] = minimage(a.pos[3 * p + c] - a.pos[3 * q + c], sd.box[c], sd.inv_box[c]);
  };
  double e;
  if (is_bond) {
    double d[3];
    delta(at[0], at[1], d);
    const double r = sqrt(dot3(d, d));
    const double kb = a.bond_k[t], dr = r - a.bond_r0[t];
    e = kb * dr * dr;
    const double s = -2.0 * kb * dr / r;
    double g[3] = {s * d[0], s * d[1], s * d[2]}, h[3] = {-g[0], -g[1], -g[2]};
    add_force(a.f, at[0], g);
    add_force(a.f, at[1], h);
  } else {
    const int64_t u = t - a.n_bonds;
    double p[3], q[3];
    delta(at[0], at[1], p);
    delta(at[2], at[1], q);
    const double lp = sqrt(dot3(p, p)), lq = sqrt(dot3(q, q));
    const double cs = fmin(1.0, fmax(-1.0, dot3(p, q) / (lp * lq)));
    const double th = acos(cs);
    const double ka = a.angle_k[u], dth = th - a.angle_t0[u];
    e = ka * dth * dth;
    // F_i = (dE/dtheta)/sin(theta) * d(cos theta)/dr_i, and likewise for k; F_j balances
    const double g = 2.0 * ka * dth / sqrt(fmax(1.0 - cs * cs, 1e-300));
    double fi[3], fk[3], fj[3];
    for (int c = 0; c < 3; ++c) {
      fi[c] = g * (q[c] / (lp * lq) - cs * p[c] / (lp * lp));
      fk[c] = g * (p[c] / (lp * lq) - cs * q[c] / (lq * lq));
      fj[c] = -(fi[c] + fk[c]);
    }
    add_force(a.f, at[0], fi);
    add_force(a.f, at[2], fk);
    add_force(a.f, at[1], fj);
  }
  if (a.energy) atomicAdd(&a.energy[b], e);
}

// force = the sum of the four parts (nb_md_forces).
__global__ void k_md_sum(double *force, const double *f_nb, const double *f_corr, const double *f_rec,
                         const double *f_bond, int64_t n3) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kMdBlock + threadIdx.x;
  if (e >= n3) return;
  double s = f_nb[e] + f_bond[e];
  if (f_corr) s += f_corr[e] + f_rec[e];
  force[e] = s;
}

// Kinetic energy per system into kin[b] (zeroed before): wave sums where a wave's atoms
// are all in one system, per-atom atomics otherwise.
__global__ void __launch_bounds__(kMdBlock) k_md_kinetic(const double *vel, const double *mass, const SysDesc *desc,
                                                         int B, int64_t N, double *kin) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kMdBlock + threadIdx.x;
  const bool live = i < N;
  double e = 0.0;
  int b = 0;
  if (live) {
    const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
    e = 0.5 * kKineticUnit * mass[i] * (vx * vx + vy * vy + vz * vz);
    b = system_of(desc, B, i);
  }
  const int b0 = __shfl(b, 0, 64);
  const bool uniform = __all(!live || b == b0);
  if (uniform) {
    const double s = wave_sum(e);
    if ((threadIdx.x & 63) == 0) atomicAdd(&kin[b0], s);
  } else if (live) {
    atomicAdd(&kin[b], e);
  }
}

// energy_out[K b + k] = the k-th accumulator of system b (k < K).
__global__ void k_md_pack(double *out, const double *acc, int B, int K) {
  const int t = static_cast<int>(blockIdx.x * kMdBlock + threadIdx.x);
  if (t >= B * K) return;
  const int b = t / K, k = t % K;
  out[t] = acc[static_cast<int64_t>(k) * B + b];
}

__global__ void k_md_status(uint32_t *status, const uint32_t *md_status) {
  if (threadIdx.x == 0 && *md_status) atomicOr(status, *md_status);
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>(std::max<int64_t>(1, (n + kMdBlock - 1) / kMdBlock)); }

struct Views {
  Dev d;
  void *pme_ws;
  double *f_nb, *f_corr, *f_rec, *f_bond, *energy;
  uint8_t *role;
  uint32_t *md_status;
};

Views views(const MdPlan &mp, void *ws) {
  char *base = static_cast<char *>(ws);
  Views v;
  v.d = dev_view(mp.p, ws);
  v.pme_ws = mp.ml.pme ? base + mp.ml.pme_ws : nullptr;
  v.f_nb = reinterpret_cast<double *>(base + mp.ml.f_nb);
  v.f_corr = mp.ml.pme ? reinterpret_cast<double *>(base + mp.ml.f_corr) : nullptr;
  v.f_rec = mp.ml.pme ? reinterpret_cast<double *>(base + mp.ml.f_rec) : nullptr;
  v.f_bond = reinterpret_cast<double *>(base + mp.ml.f_bond);
  v.energy = reinterpret_cast<double *>(base + mp.ml.energy);
  v.role = reinterpret_cast<uint8_t *>(base + mp.ml.role);
  v.md_status = reinterpret_cast<uint32_t *>(base + mp.ml.status);
  return v;
}

// Clears the MD scratch and marks the waters.
void setup(const MdPlan &mp, const Views &v, const nb_md_topology *topo, hipStream_t s) {
  const int64_t N = mp.p.N;
  const int ne = 5 * mp.p.B;
  hipLaunchKernelGGL(k_md_setup, dim3(blocks_for(std::max<int64_t>(N, ne))), dim3(kMdBlock), 0, s, v.role, v.f_bond,
                     v.energy, ne, v.md_status, N);
  if (topo->n_waters > 0)
    hipLaunchKernelGGL(k_md_roles, dim3(blocks_for(topo->n_waters)), dim3(kMdBlock), 0, s, v.role, topo->water_o,
                       topo->n_waters, v.d.desc, mp.p.B, N, v.md_status);
}

// The second stream of the reciprocal part and the two events that order it against the
// main stream: a fork after the integrator writes the positions, a join before the next
// integrator reads the forces.  Events are made per call and released when the call
// returns (HIP keeps them until the work they mark completes).
struct Aux {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  ~Aux() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
  }
  hipError_t open(hipStream_t aux, hipStream_t main, bool pme) {
    if (!aux || aux == main || !pme) return hipSuccess;
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e == hipSuccess) s = aux;
    return e;
  }
};

hipError_t launch_bonded(const MdPlan &mp, const Views &v, const nb_system *sys, const nb_md_topology *topo,
                         double *e_bond, hipStream_t s) {
  const int64_t nt = topo->n_bonds + topo->n_angles;
  if (nt == 0) return hipSuccess;
  BondedArgs a;
  a.pos = static_cast<const double *>(sys->pos);
  a.f = v.f_bond;
  a.energy = e_bond;
  a.bond_atoms = topo->bond_atoms;
  a.angle_atoms = topo->angle_atoms;
  a.bond_k = topo->bond_k;
  a.bond_r0 = topo->bond_r0;
  a.angle_k = topo->angle_k;
  a.angle_t0 = topo->angle_theta0;
  a.n_bonds = topo->n_bonds;
  a.n_angles = topo->n_angles;
  a.N = mp.p.N;
  a.desc = v.d.desc;
  a.B = mp.p.B;
  a.md_status = v.md_status;
  hipLaunchKernelGGL(k_md_bonded, dim3(blocks_for(nt)), dim3(kMdBlock), 0, s, a);
  return hipGetLastError();
}

// Every force part at the system's positions; energies into the accumulators when asked.
// With an auxiliary stream, the reciprocal part runs there beside the short-range work.
// The rest stays on the main stream, measured: the Ewald corrections beside the pair
// kernel made the step slower (0.137 against 0.128 ms on the 23.6k-atom box), and with
// the bonded terms on the second stream the first MD run of a process came out wrong
// (non-finite positions within 20 steps) for a reason not found.
hipError_t forces(const MdPlan &mp, const Views &v, const nb_system *sys, const nb_md_topology *topo, bool want_e,
                  hipStream_t s, const Aux &aux, std::string *err) {
  const int B = mp.p.B;
  double *e_nb = want_e ? v.energy : nullptr;
  double *e_corr = want_e ? v.energy + B : nullptr;
  double *e_rec = want_e ? v.energy + 2 * B : nullptr;
  double *e_bond = want_e ? v.energy + 3 * B : nullptr;
  const bool use_aux = aux.s != nullptr;  // only opened with a reciprocal part
  hipError_t e = hipSuccess;
  if (use_aux) {
    e = hipEventRecord(aux.fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(aux.s, aux.fork, 0);
    if (e == hipSuccess)
      e = launch_pme(mp.pl, sys, mp.p.beta, mp.p.ke, v.pme_ws, v.f_rec, e_rec, nullptr, aux.s, err);
  }
  if (e == hipSuccess && use_aux) e = hipEventRecord(aux.join, aux.s);
  if (e == hipSuccess) e = launch_build(mp.p, v.d, sys, s);
  if (e == hipSuccess) e = launch_forces(mp.p, v.d, sys, v.f_nb, e_nb, nullptr, s);
  if (e == hipSuccess && mp.ml.pme) e = launch_ewald(mp.p, v.d, sys, v.f_corr, e_corr, nullptr, s);
  if (e == hipSuccess && !use_aux && mp.ml.pme)
    e = launch_pme(mp.pl, sys, mp.p.beta, mp.p.ke, v.pme_ws, v.f_rec, e_rec, nullptr, s, err);
  if (e == hipSuccess) e = launch_bonded(mp, v, sys, topo, e_bond, s);
  if (e == hipSuccess && use_aux) e = hipStreamWaitEvent(s, aux.join, 0);
  return e;
}

}  // namespace

nb_status md_plan(const nb_system *sys, const nb_params *prm, const nb_md_params *md, MdPlan *mp, std::string *why) {
  nb_status st = make_plan(sys, prm, &mp->p);
  if (st != NB_OK) {
    *why = "";
    return st;
  }
  if (!md) {
    *why = "md params are NULL";
    return NB_ERR_ARG;
  }
  if (sys->pos_is_f64 != 1) {
    *why = "the MD state is double precision: pos_is_f64 must be 1";
    return NB_ERR_ARG;
  }
  if (!(md->dt > 0.0) || !std::isfinite(md->dt)) {
    *why = "dt must be positive and finite";
    return NB_ERR_ARG;
  }
  if (!(md->temperature >= 0.0) || !std::isfinite(md->temperature) || !(md->gamma >= 0.0) ||
      !std::isfinite(md->gamma)) {
    *why = "temperature and gamma must be >= 0 and finite";
    return NB_ERR_ARG;
  }
  const bool pme = md->pme_grid[0] != 0 || md->pme_grid[1] != 0 || md->pme_grid[2] != 0;
  MdLayout &ml = mp->ml;
  ml = MdLayout{};
  ml.pme = pme;
  size_t off = align256(mp->p.lay.total);
  if (pme) {
    if (!(prm->ewald_beta > 0.0)) {
      *why = "a PME grid needs ewald_beta > 0";
      return NB_ERR_ARG;
    }
    std::string w = pme_layout(mp->p.B, md->pme_grid, &mp->pl);
    if (!w.empty()) {
      *why = w;
      return NB_ERR_ARG;
    }
    w = pme_attach_plans(&mp->pl);
    if (!w.empty()) {
      *why = w;
      return NB_ERR_HIP;
    }
    ml.pme_ws = off;
    off = align256(off + mp->pl.total);
  }
  const size_t fbytes = align256(static_cast<size_t>(mp->p.N) * 3 * sizeof(double));
  ml.f_nb = off;
  off += fbytes;
  if (pme) {
    ml.f_corr = off;
    off += fbytes;
    ml.f_rec = off;
    off += fbytes;
  }
  ml.f_bond = off;
  off += fbytes;
  ml.energy = off;
  off += align256(5 * static_cast<size_t>(mp->p.B) * sizeof(double));
  ml.role = off;
  off += align256(static_cast<size_t>(mp->p.N));
  ml.status = off;
  off += 256;
  ml.total = off;
  return NB_OK;
}

std::string md_check_topology(const MdPlan &mp, const nb_md_topology *t) {
  if (!t) return "topology is NULL";
  if (mp.p.N > 0 && !t->mass) return "mass is required";
  if (t->n_waters < 0 || t->n_bonds < 0 || t->n_angles < 0) return "term counts must be >= 0";
  if (t->n_waters > mp.p.N / 3 || t->n_bonds > INT32_MAX || t->n_angles > INT32_MAX)
    return "more terms than the batch's atoms allow";
  if (t->n_waters > 0) {
    if (!t->water_o) return "water_o is required when n_waters > 0";
    if (!(t->water_r_oh > 0.0) || !(t->water_r_hh > 0.0) || !(t->water_r_hh < 2.0 * t->water_r_oh) ||
        !std::isfinite(t->water_r_oh) || !std::isfinite(t->water_r_hh))
      return "water lengths must be positive, finite and form a triangle (r_hh < 2 r_oh)";
  }
  if (t->n_bonds > 0 && (!t->bond_atoms || !t->bond_k || !t->bond_r0)) return "bond arrays are required";
  if (t->n_angles > 0 && (!t->angle_atoms || !t->angle_k || !t->angle_theta0)) return "angle arrays are required";
  return "";
}

hipError_t md_forces(const MdPlan &mp, const nb_system *sys, const nb_md_topology *topo, const nb_md_params *md,
                     void *ws, double *force, double *energy, hipStream_t s, std::string *err) {
  const Views v = views(mp, ws);
  Aux aux;
  hipError_t e = aux.open(md->aux_stream, s, mp.ml.pme);
  if (e != hipSuccess) return e;
  setup(mp, v, topo, s);
  e = forces(mp, v, sys, topo, energy != nullptr, s, aux, err);
  if (e != hipSuccess) return e;
  const int64_t n3 = 3 * mp.p.N;
  if (n3 > 0)
    hipLaunchKernelGGL(k_md_sum, dim3(blocks_for(n3)), dim3(kMdBlock), 0, s, force, v.f_nb, v.f_corr, v.f_rec,
                       v.f_bond, n3);
  if (energy)
    hipLaunchKernelGGL(k_md_pack, dim3(blocks_for(4 * mp.p.B)), dim3(kMdBlock), 0, s, energy, v.energy, mp.p.B, 4);
  hipLaunchKernelGGL(k_md_status, dim3(1), dim3(64), 0, s, v.d.status, v.md_status);
  return hipGetLastError();
}

hipError_t md_run(const MdPlan &mp, const nb_system *sys, const nb_md_topology *topo, const nb_md_params *md,
                  void *ws, double *vel, int64_t first_step, int64_t n_steps, double *energy, hipStream_t s,
                  std::string *err) {
  const Views v = views(mp, ws);
  Aux aux;
  hipError_t e = aux.open(md->aux_stream, s, mp.ml.pme);
  if (e != hipSuccess) return e;
  setup(mp, v, topo, s);
  e = forces(mp, v, sys, topo, energy != nullptr && n_steps == 0, s, aux, err);
  MdArgs k;
  k.pos = static_cast<double *>(const_cast<void *>(sys->pos));
  k.vel = vel;
  k.f_bond = v.f_bond;
  k.f_nb = v.f_nb;
  k.f_corr = v.f_corr;
  k.f_rec = v.f_rec;
  k.mass = topo->mass;
  k.role = v.role;
  k.desc = v.d.desc;
  k.B = mp.p.B;
  k.N = mp.p.N;
  k.dt = md->dt;
  k.c = std::exp(-0.5 * md->gamma * md->dt);
  k.noise_var = (1.0 - k.c * k.c) * kAccel * kBoltzmann * md->temperature;
  k.r_oh2 = topo->water_r_oh * topo->water_r_oh;
  k.r_hh2 = topo->water_r_hh * topo->water_r_hh;
  k.key0 = static_cast<uint32_t>(md->seed);
  k.key1 = static_cast<uint32_t>(md->seed >> 32);
  k.thermostat = md->gamma > 0.0 ? 1 : 0;
  k.water_o = topo->water_o;
  k.n_waters = topo->n_waters;
  constexpr int64_t kWatersPerBlock = kWatersPerWave * (kMdBlock / 64);
  const unsigned wb = static_cast<unsigned>((topo->n_waters + kWatersPerBlock - 1) / kWatersPerBlock);
  const dim3 g(wb + blocks_for(mp.p.N)), blk(kMdBlock);
  for (int64_t st = 0; st < n_steps && e == hipSuccess && mp.p.N > 0; ++st) {
    k.step_start = first_step + st;
    k.step_end = first_step + st - 1;
    if (st == 0) hipLaunchKernelGGL(k_md_integrate<kStart>, g, blk, 0, s, k, wb);
    else hipLaunchKernelGGL(k_md_integrate<kEndStart>, g, blk, 0, s, k, wb);
    e = hipGetLastError();
    if (e == hipSuccess) e = forces(mp, v, sys, topo, energy != nullptr && st == n_steps - 1, s, aux, err);
  }
  if (e != hipSuccess) return e;
  if (n_steps > 0 && mp.p.N > 0) {
    k.step_end = first_step + n_steps - 1;
    hipLaunchKernelGGL(k_md_integrate<kEnd>, g, blk, 0, s, k, wb);
  }
  if (energy) {
    if (mp.p.N > 0)
      hipLaunchKernelGGL(k_md_kinetic, dim3(blocks_for(mp.p.N)), blk, 0, s, vel, topo->mass, v.d.desc, mp.p.B, mp.p.N,
                         v.energy + 4 * mp.p.B);
    hipLaunchKernelGGL(k_md_pack, dim3(blocks_for(5 * mp.p.B)), dim3(kMdBlock), 0, s, energy, v.energy, mp.p.B, 5);
  }
  hipLaunchKernelGGL(k_md_status, dim3(1), dim3(64), 0, s, v.d.status, v.md_status);
  return hipGetLastError();
}

}  // namespace nb
