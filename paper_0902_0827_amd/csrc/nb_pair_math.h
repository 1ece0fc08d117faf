// Pair arithmetic shared by the pair kernels (device code only).
//
// For a pair at distance r (r^2 < R^2, not excluded) with type-pair coefficients
// c6 = 4 eps_ij sigma_ij^6 and c12 = 4 eps_ij sigma_ij^12 and charge product qq
// (k_e already folded in):
//
//   u      = c12/r^12 - c6/r^6 + qq erfc(beta r)/r
//   f      = [12 c12/r^12 - 6 c6/r^6 + qq (erfc(beta r)/r + (2 beta/sqrt(pi)) exp(-beta^2 r^2))] / r^2
//
// so that the force on i from j is f * d_ij with d_ij = x_i - x_j (minimum image).
// The adjoint also needs du/dsigma_ij = (12 c12/r^12 - 6 c6/r^6) / sigma_ij.
#pragma once

#include <hip/hip_runtime.h>

namespace nb {

// erfc(x) = exp(-x^2) * t * P(t), t = 1/(1 + p x): Hastings' substitution (Abramowitz &
// Stegun 7.1.26) refitted to degree 8 by minimax on relative error over [0, 6]
// (gen_erfc_coeffs.py).  Fit error 6e-9; single-precision evaluation error ~3e-7.
constexpr float kErfcP = 0.47047f;
constexpr float kErfcC0 = 2.653190811e-01f;
constexpr float kErfcC1 = 2.676810699e-01f;
constexpr float kErfcC2 = 2.170464896e-01f;
constexpr float kErfcC3 = 2.685938874e-01f;
constexpr float kErfcC4 = -1.731834435e-01f;
constexpr float kErfcC5 = 5.340760566e-01f;
constexpr float kErfcC6 = -6.228106085e-01f;
constexpr float kErfcC7 = 2.961506389e-01f;
constexpr float kErfcC8 = -5.287316965e-02f;

// exp(x^2) erfc(x) for x >= 0 in single precision.
__device__ __forceinline__ float erfcx_f32(float x) {
  const float t = __builtin_amdgcn_rcpf(fmaf(kErfcP, x, 1.0f));
  float p = kErfcC8;
  p = fmaf(p, t, kErfcC7);
  p = fmaf(p, t, kErfcC6);
  p = fmaf(p, t, kErfcC5);
  p = fmaf(p, t, kErfcC4);
  p = fmaf(p, t, kErfcC3);
  p = fmaf(p, t, kErfcC2);
  p = fmaf(p, t, kErfcC1);
  p = fmaf(p, t, kErfcC0);
  return p * t;
}

struct PairF32 {
  float u_lj, u_c, f, dudsig_lj;  // energies, force factor, (12 c12/r^12 - 6 c6/r^6)
  float erfc_over_r;              // erfc(beta r)/r (for dE/dq)
};

// Single-precision pair terms.  beta, two_beta_sqrtpi = 2 beta/sqrt(pi) and
// mb2l2e = -beta^2 log2(e) are per-call constants.
__device__ __forceinline__ PairF32 pair_f32(float r2, float c6, float c12, float qq, float beta,
                                            float two_beta_sqrtpi, float mb2l2e) {
  // Products are fused into additions only within one expression, so that every kernel
  // this is inlined into rounds the pair terms alike.
#pragma clang fp contract(on)
  PairF32 o;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float rinv2 = rinv * rinv;
  const float rinv6 = rinv2 * rinv2 * rinv2;
  const float a = c12 * rinv6 * rinv6;
  const float b = c6 * rinv6;
  o.u_lj = a - b;
  o.dudsig_lj = fmaf(12.0f, a, -6.0f * b);
  const float r = r2 * rinv;
  const float e = __builtin_amdgcn_exp2f(r2 * mb2l2e);  // exp(-beta^2 r^2)
  const float erfc_br = erfcx_f32(beta * r) * e;
  o.erfc_over_r = erfc_br * rinv;
  o.u_c = qq * o.erfc_over_r;
  o.f = fmaf(qq, fmaf(two_beta_sqrtpi, e, o.erfc_over_r), o.dudsig_lj) * rinv2;
  return o;
}

// The same pair terms with the force-field options: the Lennard-Jones term weighted by
// w_lj (the 1-4 scale, else 1) and by the switch S(x) = (1 - x)^2 (1 + 2x),
// x = max((r^2 - sw_on2) sw_inv, 0) (the caller folds the 1-4 Coulomb scale into qq).
// With u0 and d0 = 12 a - 6 b the unswitched energy and its -r du/dr:
//   u_lj      = w S u0
//   dudsig_lj = w S d0                    (the sigma derivative at fixed r, for the adjoint)
//   f         = [w (S d0 + 12 x (1 - x) r^2 sw_inv u0) + qq (...)] / r^2
// the middle term being -2 r^2 u0 dS/d(r^2).  No switch: sw_inv = 0, so x = 0 and S = 1.
__device__ __forceinline__ PairF32 pair_f32_ff(float r2, float c6, float c12, float qq, float w_lj, float beta,
                                               float two_beta_sqrtpi, float mb2l2e, float sw_on2, float sw_inv) {
#pragma clang fp contract(on)
  PairF32 o;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float rinv2 = rinv * rinv;
  const float rinv6 = rinv2 * rinv2 * rinv2;
  const float a = c12 * rinv6 * rinv6;
  const float b = c6 * rinv6;
  const float u0 = a - b;
  const float d0 = fmaf(12.0f, a, -6.0f * b);
  const float x = fmaxf((r2 - sw_on2) * sw_inv, 0.0f);
  const float omx = 1.0f - x;
  const float ws = w_lj * (omx * omx * fmaf(2.0f, x, 1.0f));
  o.u_lj = ws * u0;
  o.dudsig_lj = ws * d0;
  const float dsw = w_lj * (12.0f * x * omx) * (r2 * sw_inv);
  const float d_force = fmaf(dsw, u0, o.dudsig_lj);
  const float r = r2 * rinv;
  const float e = __builtin_amdgcn_exp2f(r2 * mb2l2e);  // exp(-beta^2 r^2)
  const float erfc_br = erfcx_f32(beta * r) * e;
  o.erfc_over_r = erfc_br * rinv;
  o.u_c = qq * o.erfc_over_r;
  o.f = fmaf(qq, fmaf(two_beta_sqrtpi, e, o.erfc_over_r), d_force) * rinv2;
  return o;
}

// Parameter derivatives of the force factor, for the force VJP: the LJ force factor
// f_LJ = w [S d0 + 12 x (1 - x) r^2 sw_inv u0] / r^2 (as pair_f32_ff; S = 1 without a
// switch), sigma_ij df_LJ/dsigma_ij = w [S dd + 12 x (1 - x) r^2 sw_inv d0] / r^2 with
// dd = 144 a - 36 b (sigma d/dsigma takes u0 to d0 and d0 to dd), and the Coulomb force
// factor per unit qq, w_c [erfc(beta r)/r + (2 beta/sqrt(pi)) exp(-beta^2 r^2)] / r^2.
struct PairVjpF32 { float flj, dflj, gc; };
struct PairVjpF64 { double flj, dflj, gc; };

__device__ __forceinline__ PairVjpF32 pair_vjp_f32(float r2, float c6, float c12, float w_lj, float w_c, float beta,
                                                   float two_beta_sqrtpi, float mb2l2e, float sw_on2, float sw_inv) {
#pragma clang fp contract(on)
  PairVjpF32 o;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float rinv2 = rinv * rinv;
  const float rinv6 = rinv2 * rinv2 * rinv2;
  const float a = c12 * rinv6 * rinv6;
  const float b = c6 * rinv6;
  const float u0 = a - b;
  const float d0 = fmaf(12.0f, a, -6.0f * b);
  const float dd = fmaf(144.0f, a, -36.0f * b);
  const float x = fmaxf((r2 - sw_on2) * sw_inv, 0.0f);
  const float omx = 1.0f - x;
  const float sw = omx * omx * fmaf(2.0f, x, 1.0f);
  const float qs = (12.0f * x * omx) * (r2 * sw_inv);
  o.flj = w_lj * fmaf(qs, u0, sw * d0) * rinv2;
  o.dflj = w_lj * fmaf(qs, d0, sw * dd) * rinv2;
  const float r = r2 * rinv;
  const float e = __builtin_amdgcn_exp2f(r2 * mb2l2e);
  const float eor = erfcx_f32(beta * r) * e * rinv;
  o.gc = w_c * fmaf(two_beta_sqrtpi, e, eor) * rinv2;
  return o;
}

// Tabulated variant (section 3: the paper reads the radial parts of the electrostatic
// and van der Waals terms from linearly interpolated texture tables).  Node k of a table
// uniform in r (r = k h, h = R/n, nodes 0..n) holds
//   E12 = r^-12,  E6 = r^-6,  EC = erfc(beta r)/r,  FC = [erfc(beta r)/r + (2 beta/sqrt(pi)) exp(-beta^2 r^2)]/r^2
// (node 0 repeats node 1: no pair is that close).  TAB = 1: one float4 per node, linear
// interpolation; TAB = 2: per node the values and h times their r-derivatives (two float4),
// cubic Hermite interpolation.  Then u_LJ = c12 E12 - c6 E6, u_C = qq EC and
// f = (12 c12 E12 - 6 c6 E6)/r^2 + qq FC.
template <int TAB>
__device__ __forceinline__ PairF32 pair_f32_tab(float r2, float c6, float c12, float qq,
                                                const float4 *__restrict__ tab, float inv_h, float last) {
#pragma clang fp contract(on)
  PairF32 o;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float rinv2 = rinv * rinv;
  // lanes without a pair may hold any distance (or NaN at r = 0): the node index is
  // clamped to the table (fminf returns `last` for NaN) and their terms are discarded
  const float t = fminf(r2 * rinv * inv_h, last);
  const int k = static_cast<int>(t);
  const float u = t - static_cast<float>(k);
  float4 e;
  if constexpr (TAB == 1) {
    const float4 a = tab[k], b = tab[k + 1];
    e = make_float4(fmaf(u, b.x - a.x, a.x), fmaf(u, b.y - a.y, a.y), fmaf(u, b.z - a.z, a.z),
                    fmaf(u, b.w - a.w, a.w));
  } else {
    const float4 a = tab[2 * k], da = tab[2 * k + 1], b = tab[2 * k + 2], db = tab[2 * k + 3];
    const float omu = 1.0f - u;
    const float h00 = fmaf(2.0f, u, 1.0f) * omu * omu, h10 = u * omu * omu;
    const float h01 = u * u * fmaf(-2.0f, u, 3.0f), h11 = -u * u * omu;
    e = make_float4(fmaf(h00, a.x, fmaf(h10, da.x, fmaf(h01, b.x, h11 * db.x))),
                    fmaf(h00, a.y, fmaf(h10, da.y, fmaf(h01, b.y, h11 * db.y))),
                    fmaf(h00, a.z, fmaf(h10, da.z, fmaf(h01, b.z, h11 * db.z))),
                    fmaf(h00, a.w, fmaf(h10, da.w, fmaf(h01, b.w, h11 * db.w))));
  }
  const float a12 = c12 * e.x, b6 = c6 * e.y;
  o.u_lj = a12 - b6;
  o.dudsig_lj = fmaf(12.0f, a12, -6.0f * b6);
  o.erfc_over_r = e.z;
  o.u_c = qq * e.z;
  o.f = fmaf(o.dudsig_lj, rinv2, qq * e.w);
  return o;
}

// erfc(x) = exp(-x^2) * g(x) in double precision, with g a polynomial of degree 24 in
// s = (x - 3)/(x + 3), which maps x in [0, inf) onto [-1, 1): a Chebyshev interpolant
// of g converted to monomial form (gen_erfc_coeffs.py --f64).  Relative error of g
// below 4e-16 for 0 <= x <= 10 and below 3e-15 up to x = 30, with one reciprocal (hardware
// estimate and two Newton steps; x + 3 >= 3 has no special cases) and a Horner chain.
static __constant__ double kErfcxS[25] = {
    1.79001151181389956e-01,
    -3.26233560043037163e-01,
    2.45603801712330871e-01,
    -1.50115936500785557e-01,
    7.16658371979800313e-02,
    -2.43924993184123605e-02,
    4.26913633277677812e-03,
    7.07746435162920763e-04,
    -5.97061947532098215e-04,
    4.52553291283249557e-05,
    6.40565466645375150e-05,
    -1.28606511272684550e-05,
    -7.97808738953117245e-06,
    2.12050566308128781e-06,
    1.25236129992384039e-06,
    -2.94961939845765926e-07,
    -2.34395216015276363e-07,
    2.97949776303463178e-08,
    4.65820100294348347e-08,
    9.43754184607545609e-11,
    -8.64771944351097140e-09,
    -8.10395956093485400e-10,
    1.26827809481409217e-09,
    1.26390768337342988e-10,
    -1.04873117593991747e-10};

// a * b + c with c in a scalar register pair: one v_fma_f64.  (Left to itself the
// compiler copies c into the destination and uses the two-operand v_fmac_f64, three
// instructions per step of a Horner chain whose coefficients come from scalar loads.)
__device__ __forceinline__ double fma_s(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// The same g as a polynomial of degree 18 in s, interpolated on 0 <= x <= 4.2 only (to
// 4e-16 relative there): enough for every pair when beta R <= 4.2.
static __constant__ double kErfcxShort[19] = {
    1.79001151181389956e-01,
    -3.26233560043037218e-01,
    2.45603801712330816e-01,
    -1.50115936500776648e-01,
    7.16658371979928960e-02,
    -2.43924993186649779e-02,
    4.26913633168420764e-03,
    7.07746432994099325e-04,
    -5.97061928621600265e-04,
    4.52555777698059495e-05,
    6.40573859040072902e-05,
    -1.28618544324921400e-05,
    -7.99671182594526170e-06,
    2.04925522636487597e-06,
    1.09284090032394909e-06,
    -5.33848327689116094e-07,
    -4.80395335088038175e-07,
    -1.37166373609392244e-07,
    -1.50800419617872139e-08};
constexpr double kErfcxShortMax = 4.2;

__device__ __forceinline__ double erfcx_f64(double x, bool short_range) {
  // The coefficients are read from constant memory through a pointer the compiler
  // cannot treat as loop-invariant, so that they arrive by scalar loads where the
  // chain needs them instead of occupying 48 vector registers across the pair loop.
  using ConstF64 = const __attribute__((address_space(4))) double;
  ConstF64 *c = (ConstF64 *)(short_range ? kErfcxShort : kErfcxS);  // generic -> constant address space
  asm volatile("" : "+s"(c));
  // 1/(x + 3) from the hardware reciprocal and two Newton steps (x + 3 >= 3)
  const double b = x + 3.0;
  double y = __builtin_amdgcn_rcp(b);
  y = fma(fma(-b, y, 1.0), y, y);
  y = fma(fma(-b, y, 1.0), y, y);
  const double s = (x - 3.0) * y;
  double p;
  if (short_range) {  // wave-uniform: one choice per call
    p = c[18];
#pragma unroll
    for (int k = 17; k >= 0; --k) p = fma_s(p, s, c[k]);
  } else {
    p = c[24];
#pragma unroll
    for (int k = 23; k >= 0; --k) p = fma_s(p, s, c[k]);
  }
  return p;
}

struct PairF64 {
  double u_lj, u_c, f, dudsig_lj, erfc_over_r;
};

// exp(-y) for finite y >= 0 in double precision (Cody and Waite's argument reduction):
// y = n ln 2 + r with n = rint(y / ln 2) and |r| <= ln(2)/2, r formed with ln 2 split
// into a double and its remainder; exp(-r) by its Taylor series to degree 13
// (truncation error below 5e-18 relative), then exp(-y) = 2^-n exp(-r) by ldexp, which
// also takes results below the normal range to denormals and zero.
static __constant__ double kExpNegTaylor[14] = {
    1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040, 1.0 / 40320, 1.0 / 362880,
    1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600, 1.0 / 6227020800};
constexpr double kLn2Hi = 0.6931471805599453;      // ln 2 rounded to double
constexpr double kLn2Lo = 2.3190468138462996e-17;  // ln 2 - kLn2Hi
constexpr double kInvLn2 = 1.4426950408889634;

__device__ __forceinline__ double exp_neg_f64(double y) {
  using ConstF64 = const __attribute__((address_space(4))) double;
  ConstF64 *c = (ConstF64 *)(kExpNegTaylor);  // generic -> constant address space
  asm volatile("" : "+s"(c));                 // scalar loads where used (as in erfcx_f64)
  const double n = rint(y * kInvLn2);
  double r = fma(-n, kLn2Hi, y);
  r = fma(-n, kLn2Lo, r);  // y - n ln 2
  const double m = -r;
  double p = c[13];
#pragma unroll
  for (int k = 12; k >= 2; --k) p = fma_s(p, m, c[k]);
  p = fma(p, m, 1.0);
  p = fma(p, m, 1.0);
  return ldexp(p, -static_cast<int>(n));
}

// Double-precision pair terms: 1/r from the hardware reciprocal square root refined by
// Newton steps (each doubles the correct bits; two take it to double precision),
// exp(-beta^2 r^2) by exp_neg_f64, and erfc from that exponential (which the force
// needs anyway) times erfcx_f64.
__device__ __forceinline__ PairF64 pair_f64(double r2, double c6, double c12, double qq, double beta,
                                            double two_beta_sqrtpi, bool short_erfc) {
  PairF64 o;
  // 1/r from the hardware reciprocal square root and two Newton steps (r2 > 0 here)
  double rinv = __builtin_amdgcn_rsq(r2);
  rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
  rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
  const double r = r2 * rinv;
  const double rinv2 = rinv * rinv;
  const double rinv6 = rinv2 * rinv2 * rinv2;
  const double a = c12 * rinv6 * rinv6;
  const double b = c6 * rinv6;
  o.u_lj = a - b;
  o.dudsig_lj = 12.0 * a - 6.0 * b;
  const double e = exp_neg_f64(beta * beta * r2);  // exp(-(beta r)^2)
  const double erfc_br = erfcx_f64(beta * r, short_erfc) * e;
  o.erfc_over_r = erfc_br * rinv;
  o.u_c = qq * o.erfc_over_r;
  o.f = (o.dudsig_lj + qq * (o.erfc_over_r + two_beta_sqrtpi * e)) * rinv2;
  return o;
}

// Parameter derivatives of the force factor in double precision (as pair_vjp_f32).
__device__ __forceinline__ PairVjpF64 pair_vjp_f64(double r2, double c6, double c12, double w_lj, double w_c,
                                                   double beta, double two_beta_sqrtpi, bool short_erfc, double sw_on2,
                                                   double sw_inv) {
  PairVjpF64 o;
  double rinv = __builtin_amdgcn_rsq(r2);
  rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
  rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
  const double r = r2 * rinv;
  const double rinv2 = rinv * rinv;
  const double rinv6 = rinv2 * rinv2 * rinv2;
  const double a = c12 * rinv6 * rinv6;
  const double b = c6 * rinv6;
  const double u0 = a - b;
  const double d0 = 12.0 * a - 6.0 * b;
  const double dd = 144.0 * a - 36.0 * b;
  const double x = fmax((r2 - sw_on2) * sw_inv, 0.0);
  const double omx = 1.0 - x;
  const double sw = omx * omx * (1.0 + 2.0 * x);
  const double qs = (12.0 * x * omx) * (r2 * sw_inv);
  o.flj = w_lj * (sw * d0 + qs * u0) * rinv2;
  o.dflj = w_lj * (sw * dd + qs * d0) * rinv2;
  const double e = exp_neg_f64(beta * beta * r2);
  const double eor = erfcx_f64(beta * r, short_erfc) * e * rinv;
  o.gc = w_c * (eor + two_beta_sqrtpi * e) * rinv2;
  return o;
}

// The double-precision pair terms with the force-field options (as pair_f32_ff).
__device__ __forceinline__ PairF64 pair_f64_ff(double r2, double c6, double c12, double qq, double w_lj, double beta,
                                               double two_beta_sqrtpi, bool short_erfc, double sw_on2,
                                               double sw_inv) {
  PairF64 o;
  double rinv = __builtin_amdgcn_rsq(r2);
  rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
  rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
  const double r = r2 * rinv;
  const double rinv2 = rinv * rinv;
  const double rinv6 = rinv2 * rinv2 * rinv2;
  const double a = c12 * rinv6 * rinv6;
  const double b = c6 * rinv6;
  const double u0 = a - b;
  const double d0 = 12.0 * a - 6.0 * b;
  const double x = fmax((r2 - sw_on2) * sw_inv, 0.0);
  const double omx = 1.0 - x;
  const double ws = w_lj * (omx * omx * (1.0 + 2.0 * x));
  o.u_lj = ws * u0;
  o.dudsig_lj = ws * d0;
  const double d_force = o.dudsig_lj + w_lj * (12.0 * x * omx) * (r2 * sw_inv) * u0;
  const double e = exp_neg_f64(beta * beta * r2);  // exp(-(beta r)^2)
  const double erfc_br = erfcx_f64(beta * r, short_erfc) * e;
  o.erfc_over_r = erfc_br * rinv;
  o.u_c = qq * o.erfc_over_r;
  o.f = (d_force + qq * (o.erfc_over_r + two_beta_sqrtpi * e)) * rinv2;
  return o;
}

}  // namespace nb
