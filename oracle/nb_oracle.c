/*
 * nb_oracle.c -- FP64 brute-force reference for the short-range nonbonded
 * energy, forces, virial and parameter gradients.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header or constant generator
 * with the GPU library.
 *
 * What it computes (ACEMD paper, section 3: the non-bonded force term is the
 * full Lennard-Jones plus electrostatic interaction of every atom pair within the
 * cutoff R, with bonded pairs excluded; long-range electrostatics use PME, whose
 * short-range part is the Ewald real-space term):
 *
 *   d_ij = x_i - x_j - L * rint((x_i - x_j) / L)      per dimension (minimum image)
 *   a pair (i != j) counts iff |d_ij|^2 < R^2 and (i, j) is not excluded, where an
 *   exclusion listed in either atom's row excludes the pair both ways
 *   sigma_ij = (sigma_ti + sigma_tj) / 2,  eps_ij = sqrt(eps_ti * eps_tj)
 *   u_ij = 4 eps_ij [(sigma_ij/r)^12 - (sigma_ij/r)^6] + k_e q_i q_j erfc(beta r) / r
 *   F_i  = sum_j f_ij d_ij with
 *   f_ij = 24 eps_ij [2 (sigma_ij/r)^12 - (sigma_ij/r)^6] / r^2
 *        + k_e q_i q_j [erfc(beta r) / r^3 + (2 beta / sqrt(pi)) exp(-beta^2 r^2) / r^2]
 *
 * Force-field options (ACEMD paper, section 3, CHARMM/AMBER support; section 5, the
 * benchmark's cutoff "switched at 7.5 A"):
 *   - scaled 1-4 pairs: a pair listed in either atom's 1-4 row (and not excluded) has its
 *     Lennard-Jones term multiplied by s14_lj and its real-space Coulomb term by s14_c;
 *   - Lennard-Jones switching from r_on to R (sw_on = r_on > 0): u_LJ is multiplied by
 *     S(r) = (1 - x)^2 (1 + 2x), x = (r^2 - r_on^2)/(R^2 - r_on^2) clamped to [0, 1]
 *     (the CHARMM energy switch of Brooks et al., J. Comput. Chem. 4, 187 (1983)); the
 *     force is -d(S u_LJ)/dr; the Coulomb term is not switched.
 *
 * Force vector-Jacobian product (force matching): with a vector v_i per atom and
 * L = sum_i v_i . F_i = sum over ordered pairs of f_ij w_ij, w_ij = v_i . d_ij, the
 * derivatives of L with respect to the parameters are, per row i (full sums over j),
 *   dq2[i] = sum_j k_e w_c q_j gC_ij (v_i - v_j) . d_ij        (= dL/dq_i)
 *   a2[i]  = sum_j (1/2) df_ij/dsigma_ij (v_i - v_j) . d_ij    (sum over t_i = t: dL/dsigma_t)
 *   b2[i]  = sum_j (1/2) fLJ_ij (v_i - v_j) . d_ij             (sum over t_i = t, / eps_t: dL/deps_t)
 * with gC the Coulomb force factor per unit k_e q_i q_j and fLJ the LJ force factor (f =
 * fLJ + fC, F_i = sum_j f_ij d_ij).
 *
 * The evaluation is "row" based and deliberately plain: for every requested atom
 * i it loops over all N atoms j (an O(N) row, O(N^2) overall), so forces on a
 * subset of atoms (the sampled mode used for million-atom boxes) come from the
 * same code as a full evaluation.  Per-row outputs:
 *
 *   force[i]  = F_i
 *   energy[i] = (1/2) sum_j u_ij                        (per-atom energy split)
 *   phi[i]    = sum_j k_e q_j erfc(beta r)/r             (= dE/dq_i)
 *   a_sig[i]  = sum_j (1/2) du_ij/dsigma_ij              (sum over t_i = t gives dE/dsigma_t)
 *   b_eps[i]  = sum_j (1/2) u^LJ_ij                      (sum over t_i = t, / eps_t gives dE/deps_t)
 *   virial    = (1/2) sum_rows sum_j d_ij (x) F_ij       (9 entries, row-major a,b)
 *
 * Everything is IEEE double with libm erfc/exp; no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Symmetric closure of the exclusion CSR: row i of the result lists every j with
 * j in row(i) or i in row(j).  Returns 0 on success, -1 on bad input. */
static int sym_exclusions(int64_t n, const int32_t *off, const int32_t *idx,
                          int64_t **s_off_out, int32_t **s_idx_out) {
  int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -1;
  for (int64_t i = 0; i < n; ++i) {
    if (off[i + 1] < off[i]) { free(cnt); return -1; }
    for (int64_t k = off[i]; k < off[i + 1]; ++k) {
      int64_t j = idx[k];
      if (j < 0 || j >= n) { free(cnt); return -1; }
      cnt[i + 1]++;
      cnt[j + 1]++;
    }
  }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  int32_t *s_idx = malloc(sizeof(int32_t) * (size_t)(cnt[n] > 0 ? cnt[n] : 1));
  int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!s_idx || !fill) { free(cnt); free(s_idx); free(fill); return -1; }
  for (int64_t i = 0; i < n; ++i) fill[i] = cnt[i];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = off[i]; k < off[i + 1]; ++k) {
      int64_t j = idx[k];
      s_idx[fill[i]++] = (int32_t)j;
      s_idx[fill[j]++] = (int32_t)i;
    }
  free(fill);
  *s_off_out = cnt;
  *s_idx_out = s_idx;
  return 0;
}

/* CHARMM switch S(r) and dS/d(r^2) at squared distance r2 (r_on^2 = s_on, R^2 = rc2). */
static void lj_switch(double r2, double s_on, double rc2, double *S, double *dS_dr2) {
  double x = (r2 - s_on) / (rc2 - s_on);
  if (x <= 0.0) {
    *S = 1.0;
    *dS_dr2 = 0.0;
    return;
  }
  if (x > 1.0) x = 1.0;
  *S = (1.0 - x) * (1.0 - x) * (1.0 + 2.0 * x);
  *dS_dr2 = -6.0 * x * (1.0 - x) / (rc2 - s_on);
}

int nbo_rows_vjp(int64_t n, const double *pos, const double *q, const int32_t *type,
                 int32_t ntypes, const double *sigma, const double *eps,
                 const int32_t *excl_off, const int32_t *excl_idx, const double *box,
                 double cutoff, double beta, double ke,
                 const int32_t *p14_off, const int32_t *p14_idx, double s14_lj, double s14_c,
                 double sw_on, const double *vv,
                 int64_t n_rows, const int64_t *rows,
                 double *force, double *energy, double *phi, double *a_sig, double *b_eps,
                 double *dq2, double *a2, double *b2,
                 double *virial, double *e_lj_out, double *e_c_out, int64_t *pair_count_out,
                 int nthreads) {
  if (n < 0 || ntypes <= 0 || cutoff <= 0.0 || beta < 0.0) return -1;
  if (sw_on < 0.0 || sw_on >= cutoff) return -1;
  for (int a = 0; a < 3; ++a)
    if (!(box[a] > 0.0) || !(cutoff < 0.5 * box[a])) return -2;
  for (int64_t i = 0; i < n; ++i)
    if (type[i] < 0 || type[i] >= ntypes) return -3;
  int64_t *s_off = NULL;
  int32_t *s_idx = NULL;
  if (sym_exclusions(n, excl_off, excl_idx, &s_off, &s_idx) != 0) return -4;
  int64_t *p_off = NULL;
  int32_t *p_idx = NULL;
  if (p14_off && sym_exclusions(n, p14_off, p14_idx, &p_off, &p_idx) != 0) {
    free(s_off);
    free(s_idx);
    return -4;
  }
  const double s_on = sw_on * sw_on;
  const int64_t m = rows ? n_rows : n;
  const double rc2 = cutoff * cutoff;
  const double two_over_sqrt_pi = 2.0 / sqrt(acos(-1.0));
  double e_lj = 0.0, e_c = 0.0;
  double vir[9] = {0};
  int64_t pairs = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif

#pragma omp parallel reduction(+ : e_lj, e_c, pairs) reduction(+ : vir[:9])
  {
    /* stamp[j] == row + 1 marks j as excluded from the current row; stamp14[j] == row + 1
       marks j as a scaled 1-4 partner of it. */
    int64_t *stamp = calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t *stamp14 = calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
      const int64_t i = rows ? rows[r] : r;
      for (int64_t k = s_off[i]; k < s_off[i + 1]; ++k) stamp[s_idx[k]] = i + 1;
      if (p_off)
        for (int64_t k = p_off[i]; k < p_off[i + 1]; ++k) stamp14[p_idx[k]] = i + 1;
      double f[3] = {0, 0, 0};
      double ei = 0.0, ph = 0.0, as = 0.0, be = 0.0, cq2 = 0.0, ca2 = 0.0, cb2 = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        if (j == i || stamp[j] == i + 1) continue;
        double d[3];
        for (int a = 0; a < 3; ++a) {
          double t = pos[3 * i + a] - pos[3 * j + a];
          d[a] = t - box[a] * rint(t / box[a]);
        }
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < rc2)) continue;
        const double r = sqrt(r2);
        /* scale factors of a 1-4 pair, and the switch of the LJ term */
        const int scaled = p_off && stamp14[j] == i + 1;
        const double w_lj = scaled ? s14_lj : 1.0, w_c = scaled ? s14_c : 1.0;
        double S = 1.0, dS_dr2 = 0.0;
        if (sw_on > 0.0) lj_switch(r2, s_on, rc2, &S, &dS_dr2);
        /* Lennard-Jones 12-6 with Lorentz-Berthelot combination. */
        const double sij = 0.5 * (sigma[type[i]] + sigma[type[j]]);
        const double eij = sqrt(eps[type[i]] * eps[type[j]]);
        const double s2 = (sij * sij) / r2;
        const double s6 = s2 * s2 * s2;
        const double s12 = s6 * s6;
        const double u_lj0 = 4.0 * eij * (s12 - s6);
        /* u = w S u0: F = -du/dr d/r = w [S f0 - 2 u0 dS/d(r^2)] d */
        const double u_lj = w_lj * S * u_lj0;
        const double f_lj = w_lj * (S * 24.0 * eij * (2.0 * s12 - s6) / r2 - 2.0 * u_lj0 * dS_dr2);
        /* d u_lj / d sigma_ij = w S (4 eps / sigma)(12 s^12 - 6 s^6); zero if sigma_ij = 0. */
        const double du_dsig = sij > 0.0 ? w_lj * S * 4.0 * eij * (12.0 * s12 - 6.0 * s6) / sij : 0.0;
        /* Ewald real-space Coulomb. */
        const double erfc_br = erfc(beta * r);
        const double u_c = w_c * ke * q[i] * q[j] * erfc_br / r;
        const double f_c = w_c * ke * q[i] * q[j] *
                           (erfc_br / (r2 * r) + beta * two_over_sqrt_pi * exp(-beta * beta * r2) / r2);
        const double fs = f_lj + f_c;
        if (vv) {
          /* (v_i - v_j) . d_ij, and the parameter derivatives of this pair's force factor:
             f_LJ = w [S dd0/r^2 - 2 u0 dS/d(r^2)] with dd0 = 24 eps (2 s^12 - s^6); both
             terms scale as eps_ij, and d/dsigma_ij of dd0 is 24 eps (24 s^12 - 6 s^6)/sigma
             (of u0: dd0 / sigma) */
          double wv = 0.0;
          for (int a = 0; a < 3; ++a) wv += (vv[3 * i + a] - vv[3 * j + a]) * d[a];
          const double dd0_ds = sij > 0.0 ? 24.0 * eij * (24.0 * s12 - 6.0 * s6) / sij : 0.0;
          const double du0_ds = sij > 0.0 ? 4.0 * eij * (12.0 * s12 - 6.0 * s6) / sij : 0.0;
          const double dflj_ds = w_lj * (S * dd0_ds / r2 - 2.0 * du0_ds * dS_dr2);
          const double gc = w_c * (erfc_br / (r2 * r) + beta * two_over_sqrt_pi * exp(-beta * beta * r2) / r2);
          cq2 += ke * q[j] * gc * wv;
          ca2 += 0.5 * dflj_ds * wv;
          cb2 += 0.5 * f_lj * wv;
        }
        for (int a = 0; a < 3; ++a) f[a] += fs * d[a];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) vir[3 * a + b] += 0.5 * d[a] * fs * d[b];
        ei += 0.5 * (u_lj + u_c);
        e_lj += 0.5 * u_lj;
        e_c += 0.5 * u_c;
        ph += w_c * ke * q[j] * erfc_br / r;
        as += 0.5 * du_dsig;
        be += 0.5 * u_lj;
        pairs += 1;
      }
      if (force) for (int a = 0; a < 3; ++a) force[3 * r + a] = f[a];
      if (energy) energy[r] = ei;
      if (phi) phi[r] = ph;
      if (a_sig) a_sig[r] = as;
      if (b_eps) b_eps[r] = be;
      if (dq2) dq2[r] = cq2;
      if (a2) a2[r] = ca2;
      if (b2) b2[r] = cb2;
    }
    free(stamp);
    free(stamp14);
  }
  if (virial) for (int k = 0; k < 9; ++k) virial[k] = vir[k];
  if (e_lj_out) *e_lj_out = e_lj;
  if (e_c_out) *e_c_out = e_c;
  /* Every unordered pair was visited from both of its atoms when all rows ran. */
  if (pair_count_out) *pair_count_out = rows ? pairs : pairs / 2;
  free(s_off);
  free(s_idx);
  free(p_off);
  free(p_idx);
  return 0;
}

int nbo_rows_ff(int64_t n, const double *pos, const double *q, const int32_t *type,
                int32_t ntypes, const double *sigma, const double *eps,
                const int32_t *excl_off, const int32_t *excl_idx, const double *box,
                double cutoff, double beta, double ke,
                const int32_t *p14_off, const int32_t *p14_idx, double s14_lj, double s14_c,
                double sw_on,
                int64_t n_rows, const int64_t *rows,
                double *force, double *energy, double *phi, double *a_sig, double *b_eps,
                double *virial, double *e_lj_out, double *e_c_out, int64_t *pair_count_out,
                int nthreads) {
  return nbo_rows_vjp(n, pos, q, type, ntypes, sigma, eps, excl_off, excl_idx, box, cutoff, beta, ke, p14_off,
                      p14_idx, s14_lj, s14_c, sw_on, NULL, n_rows, rows, force, energy, phi, a_sig, b_eps, NULL,
                      NULL, NULL, virial, e_lj_out, e_c_out, pair_count_out, nthreads);
}

/* The plain interaction: no 1-4 list, no switch. */
int nbo_rows(int64_t n, const double *pos, const double *q, const int32_t *type,
             int32_t ntypes, const double *sigma, const double *eps,
             const int32_t *excl_off, const int32_t *excl_idx, const double *box,
             double cutoff, double beta, double ke,
             int64_t n_rows, const int64_t *rows,
             double *force, double *energy, double *phi, double *a_sig, double *b_eps,
             double *virial, double *e_lj_out, double *e_c_out, int64_t *pair_count_out,
             int nthreads) {
  return nbo_rows_ff(n, pos, q, type, ntypes, sigma, eps, excl_off, excl_idx, box, cutoff, beta, ke,
                     NULL, NULL, 1.0, 1.0, 0.0, n_rows, rows, force, energy, phi, a_sig, b_eps, virial,
                     e_lj_out, e_c_out, pair_count_out, nthreads);
}

/*
 * Ewald corrections around the real-space term (section 3: the electrostatics are
 * PME, whose real-space part is the pair term above; the reciprocal part counts every
 * pair, excluded ones included, and every charge with itself):
 *
 *   E_excl = - sum over excluded pairs {i, j} of k_e q_i q_j erf(beta r) / r
 *            - (1 - s14_c) sum over scaled 1-4 pairs (not excluded) of the same term
 *            (union of both rows, any distance, minimum image; at r = 0 the limit
 *            k_e q_i q_j 2 beta / sqrt(pi))
 *   E_self = - k_e beta / sqrt(pi) sum_i q_i^2
 *   F_i    = -dE_excl/dx_i = sum_j g_ij d_ij,
 *   g_ij   = k_e q_i q_j [(2 beta / sqrt(pi)) exp(-beta^2 r^2) / r^2 - erf(beta r) / r^3]
 *            (0 at r = 0)
 *   virial = sum over excluded pairs d_ij (x) g_ij d_ij
 *   energy[i] = (1/2) sum_j u_ij - k_e beta / sqrt(pi) q_i^2
 *
 * All rows; libm erf and exp.  Returns 0, or -1 / -2 / -4 on bad input.
 */
int nbo_ewald_corrections_ff(int64_t n, const double *pos, const double *q,
                             const int32_t *excl_off, const int32_t *excl_idx,
                             const int32_t *p14_off, const int32_t *p14_idx, double s14_c,
                             const double *box, double beta, double ke, double *force, double *energy,
                             double *virial, double *e_excl_out, double *e_self_out) {
  if (n < 0 || beta < 0.0) return -1;
  for (int a = 0; a < 3; ++a)
    if (!(box[a] > 0.0)) return -2;
  int64_t *s_off = NULL, *p_off = NULL;
  int32_t *s_idx = NULL, *p_idx = NULL;
  if (sym_exclusions(n, excl_off, excl_idx, &s_off, &s_idx) != 0) return -4;
  if (p14_off && sym_exclusions(n, p14_off, p14_idx, &p_off, &p_idx) != 0) {
    free(s_off);
    free(s_idx);
    return -4;
  }
  const double two_over_sqrt_pi = 2.0 / sqrt(acos(-1.0));
  int64_t *stamp = calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  double vir[9] = {0};
  double e_excl = 0.0, e_self = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double f[3] = {0, 0, 0};
    double ei = 0.0;
    /* pass 0: excluded partners (weight 1); pass 1: scaled 1-4 partners that are not also
       excluded (weight 1 - s14_c: the reciprocal part counts them in full, the real-space
       part with s14_c) */
    for (int pass = 0; pass < 2; ++pass) {
      const int64_t *o = pass == 0 ? s_off : p_off;
      const int32_t *x = pass == 0 ? s_idx : p_idx;
      const double w = pass == 0 ? 1.0 : 1.0 - s14_c;
      if (!o) continue;
      for (int64_t k = o[i]; k < o[i + 1]; ++k) {
        const int64_t j = x[k];
        if (j == i || stamp[j] == i + 1) continue;  /* the atom itself, or a repeated entry */
        stamp[j] = i + 1;
        double d[3];
        for (int a = 0; a < 3; ++a) {
          double t = pos[3 * i + a] - pos[3 * j + a];
          d[a] = t - box[a] * rint(t / box[a]);
        }
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double qq = w * ke * q[i] * q[j];
        double u, g;
        if (r2 > 0.0) {
          const double r = sqrt(r2);
          const double erf_br = erf(beta * r);
          u = -qq * erf_br / r;
          g = qq * (beta * two_over_sqrt_pi * exp(-beta * beta * r2) / r2 - erf_br / (r2 * r));
        } else {
          u = -qq * beta * two_over_sqrt_pi;
          g = 0.0;
        }
        for (int a = 0; a < 3; ++a) f[a] += g * d[a];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) vir[3 * a + b] += 0.5 * d[a] * g * d[b];
        ei += 0.5 * u;
        e_excl += 0.5 * u;
      }
    }
    const double si = -ke * beta * 0.5 * two_over_sqrt_pi * q[i] * q[i];
    e_self += si;
    if (force) for (int a = 0; a < 3; ++a) force[3 * i + a] = f[a];
    if (energy) energy[i] = ei + si;
  }
  if (virial) for (int k = 0; k < 9; ++k) virial[k] = vir[k];
  if (e_excl_out) *e_excl_out = e_excl;
  if (e_self_out) *e_self_out = e_self;
  free(stamp);
  free(s_off);
  free(s_idx);
  free(p_off);
  free(p_idx);
  return 0;
}

int nbo_ewald_corrections(int64_t n, const double *pos, const double *q,
                          const int32_t *excl_off, const int32_t *excl_idx, const double *box,
                          double beta, double ke, double *force, double *energy, double *virial,
                          double *e_excl_out, double *e_self_out) {
  return nbo_ewald_corrections_ff(n, pos, q, excl_off, excl_idx, NULL, NULL, 1.0, box, beta, ke, force,
                                  energy, virial, e_excl_out, e_self_out);
}
