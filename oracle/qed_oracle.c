/*
 * qed_oracle.c -- plain FP64 CPU oracle of the per-particle strong-field QED step of
 * Gonoskov et al., arXiv:1412.6426.  TEST INFRASTRUCTURE ONLY (see qed_oracle.h).
 *
 * Everything here is scalar double precision with libm, built with -ffp-contract=off,
 * and follows the paper's equations in the paper's notation; no blocking, fusion or
 * reordering beyond what the equations state.  Equation numbers refer to the paper's
 * sequential numbering (Eq. (3) H_eff, (4) chi, (6) chi = gamma H_eff/E_S, (21) quantum
 * spectrum, (24) P(delta), (25) P_m, (29) dt requirement, (30) P_p, (31)-(32) chi_gamma,
 * (33) photon dt requirement).
 *
 * Readings of points where the paper is silent or ambiguous (each also listed in the
 * design notes of the repository):
 *  - modified generator photon energy is delta = f_m(r1) = r1^3 (Sec. IV.G);
 *  - the "<<" in Eqs. (29), (33) becomes dt_q = kappa * (bound), with n_sub = ceil(dt/dt_q);
 *  - n_sub and the fields are fixed once per step from the step-start state (Sec. IV.H);
 *  - inside a sub-step: Boris push, position update, chi, then the event decision;
 *  - children are stored at once but processed from the next step on;
 *  - emission recoil conserves momentum: k = delta*gamma*p/|p|, p <- p - k (Sec. IV.F);
 *  - pair split: electron r1*k, positron (1-r1)*k (Sec. V.A);
 *  - the rates are tabulated once and interpolated, as Sec. IV.F suggests:
 *    three 1-D tables in z = 2^u of e^z*F(z) for F = int K_{5/3}, K_{2/3}, int K_{1/3},
 *    4096 nodes uniform in u on [-20, 7], linear interpolation in u, a small-z series
 *    below z = 2^-20 and zero above z = 2^7.
 */
#include "qed_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* fine-structure constant, CODATA 2018 */
static const double OR_ALPHA = 7.2973525693e-3;
static const double OR_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with a Weyl key schedule.
 * Pinned by the published known-answer vectors of the generator.
 * ------------------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform number strictly inside (0,1) from two 32-bit words: the top 52 bits of the
 * 64-bit word hi:lo, plus one half, times 2^-52.  (The paper draws r in [0,1]; the open
 * interval keeps delta = r1^3 away from 0 and 1.) */
double or_uniform(uint32_t lo, uint32_t hi) {
  uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

/* ------------------------------------------------------------------------------------
 * Bessel-function integrals.  DLMF 10.32.9: K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt.
 * Integrating over z from z to infinity gives int_z^inf K_nu = int_0^inf exp(-z cosh t)
 * cosh(nu t)/cosh t dt.  Both are computed scaled by e^z, by the trapezoid rule in t,
 * which converges geometrically for these analytic, double-exponentially decaying
 * integrands.  cosh t - 1 is formed as 2 sinh^2(t/2) to keep relative accuracy near t=0.
 * Pinned against scipy.special.kv and against quadrature of kv (tests).
 * ------------------------------------------------------------------------------------ */
double or_kint_scaled(double nu, int over_cosh, double z) {
  double h = 1.0 / 32.0;
  if (z > 256.0) h = 0.5 / sqrt(z);
  double sum = 0.5; /* t = 0 term: exp(0) cosh(0) / cosh(0) = 1, half weight */
  double prev = 1.0;
  for (long k = 1; k < 2000000; ++k) {
    double t = (double)k * h;
    double sh = sinh(0.5 * t);
    double f = exp(-z * 2.0 * sh * sh) * cosh(nu * t);
    if (over_cosh) f /= cosh(t);
    sum += f;
    if (f <= prev && f < 1e-18 * sum) break;
    prev = f;
  }
  return sum * h;
}

double or_A(double z) { return or_kint_scaled(5.0 / 3.0, 1, z) * exp(-z); }
double or_B(double z) { return or_kint_scaled(2.0 / 3.0, 0, z) * exp(-z); }
double or_C(double z) { return or_kint_scaled(1.0 / 3.0, 1, z) * exp(-z); }
/* synchrotron functions of Sec. IV.E: F1(x) = x int_x^inf K_{5/3}, F2(x) = x K_{2/3}(x) */
double or_F1(double x) { return x * or_A(x); }
double or_F2(double x) { return x * or_B(x); }

/* ------------------------------------------------------------------------------------
 * Tables (tabulated once and interpolated, as Sec. IV.F suggests).
 * Small-z series (below z = 2^-20), from K_nu = (1/2)Gamma(nu)(z/2)^-nu (1 + (z/2)^2/(1-nu)
 * + ...) + (1/2)Gamma(-nu)(z/2)^nu (1 + ...) (DLMF 10.27.4 with 10.25.2) and
 * int_0^inf K_{1/3} = pi/sqrt(3) (DLMF 10.43.19):
 *   K_{2/3}(z)        = b0 z^-2/3 + b1 z^2/3 + (3/4) b0 z^4/3 + O(z^8/3)
 *   int_z^inf K_{1/3} = c0 - c1 z^2/3 - c2 z^4/3 + O(z^8/3)
 *   int_z^inf K_{5/3} = 2 K_{2/3} - int_z^inf K_{1/3}   (from K_{nu-1}+K_{nu+1} = -2K'_nu)
 * Pinned against the quadrature at small z (tests).
 * ------------------------------------------------------------------------------------ */
int or_tables_build(or_tables *t) {
  t->n = OR_TABLE_N;
  t->u_lo = OR_U_LO;
  t->u_hi = OR_U_HI;
  t->du = (OR_U_HI - OR_U_LO) / (double)(OR_TABLE_N - 1);
  t->gA = (double *)malloc(sizeof(double) * OR_TABLE_N);
  t->gB = (double *)malloc(sizeof(double) * OR_TABLE_N);
  t->gC = (double *)malloc(sizeof(double) * OR_TABLE_N);
  if (!t->gA || !t->gB || !t->gC) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < OR_TABLE_N; ++i) {
    double z = exp2(OR_U_LO + (double)i * t->du);
    t->gA[i] = or_kint_scaled(5.0 / 3.0, 1, z);
    t->gB[i] = or_kint_scaled(2.0 / 3.0, 0, z);
    t->gC[i] = or_kint_scaled(1.0 / 3.0, 1, z);
  }
  t->s_b0 = 0.5 * tgamma(2.0 / 3.0) * pow(2.0, 2.0 / 3.0);
  t->s_b1 = 0.5 * tgamma(-2.0 / 3.0) * pow(2.0, -2.0 / 3.0);
  t->s_c0 = OR_PI / sqrt(3.0);
  t->s_c1 = 0.5 * tgamma(1.0 / 3.0) * pow(2.0, 1.0 / 3.0) * 1.5;
  t->s_c2 = 0.5 * tgamma(-1.0 / 3.0) * pow(2.0, -1.0 / 3.0) * 0.75;
  return 0;
}

void or_tables_free(or_tables *t) {
  free(t->gA);
  free(t->gB);
  free(t->gC);
  t->gA = t->gB = t->gC = 0;
}

void or_eval_abc(const or_tables *t, int backend, double z, double *A, double *B, double *C) {
  if (!(z > 0.0)) { /* z <= 0 or NaN: no defined rate */
    *A = *B = *C = NAN;
    return;
  }
  if (backend == OR_EXACT) {
    *A = or_A(z);
    *B = or_B(z);
    *C = or_C(z);
    return;
  }
  if (z >= exp2(t->u_hi)) {
    *A = *B = *C = 0.0;
    return;
  }
  if (z < exp2(t->u_lo)) {
    double z23 = cbrt(z * z);
    double zm23 = 1.0 / z23;
    double z43 = z23 * z23;
    double b = t->s_b0 * zm23 + t->s_b1 * z23 + 0.75 * t->s_b0 * z43;
    double c = t->s_c0 - t->s_c1 * z23 - t->s_c2 * z43;
    *B = b;
    *C = c;
    *A = 2.0 * b - c;
    return;
  }
  double s = (log2(z) - t->u_lo) / t->du;
  int i = (int)floor(s);
  if (i < 0) i = 0;
  if (i > t->n - 2) i = t->n - 2;
  double f = s - (double)i;
  double e = exp(-z);
  *A = (t->gA[i] + f * (t->gA[i + 1] - t->gA[i])) * e;
  *B = (t->gB[i] + f * (t->gB[i + 1] - t->gB[i])) * e;
  *C = (t->gC[i] + f * (t->gC[i + 1] - t->gC[i])) * e;
}

/* ------------------------------------------------------------------------------------
 * Rates.  dtfac = Delta t * e^2 m c / hbar^2 = (sub-step duration) * alpha / eps_r.
 * ------------------------------------------------------------------------------------ */

/* Eq. (24): probability of emitting a photon with energy delta*m c^2*gamma during the
 * interval, with z_q of Eq. (21). */
double or_rate_emission(const or_tables *t, int backend, double delta, double chi, double gamma,
                        double dtfac) {
  if (!(chi > 0.0) || !(delta > 0.0) || !(delta < 1.0)) return 0.0;
  double zq = (2.0 / 3.0) * (1.0 / chi) * delta / (1.0 - delta);
  double A, B, C;
  or_eval_abc(t, backend, zq, &A, &B, &C);
  double F1 = zq * A;
  double F2 = zq * B;
  return dtfac * (sqrt(3.0) / (2.0 * OR_PI)) * (chi / gamma) * ((1.0 - delta) / delta) *
         (F1 + 1.5 * delta * chi * zq * F2);
}

/* Eq. (25) with f_m(x) = x^3 (Sec. IV.G): P_m(r1) = f_m'(r1) P(f_m(r1)). */
double or_rate_modified(const or_tables *t, int backend, double r1, double chi, double gamma,
                        double dtfac) {
  double delta = r1 * r1 * r1;
  return 3.0 * r1 * r1 * or_rate_emission(t, backend, delta, chi, gamma, dtfac);
}

/* Eq. (30): probability that a photon of energy kabs (units m c^2) creates a pair with
 * the electron taking the fraction delta_e.  Both (delta_e - 1) delta_e and the brace are
 * negative, so the product is positive; it is evaluated as printed. */
double or_rate_pair(const or_tables *t, int backend, double delta_e, double chi_g, double kabs,
                    double dtfac) {
  if (!(chi_g > 0.0) || !(delta_e > 0.0) || !(delta_e < 1.0)) return 0.0;
  double zp = (2.0 / 3.0) / (chi_g * (1.0 - delta_e) * delta_e);
  double A, B, C;
  or_eval_abc(t, backend, zp, &A, &B, &C);
  double F1 = zp * A;
  double F2 = zp * B;
  return dtfac * (sqrt(3.0) / (2.0 * OR_PI)) * (chi_g / kabs) * (delta_e - 1.0) * delta_e *
         (F1 - 1.5 * chi_g * zp * F2);
}

/* ------------------------------------------------------------------------------------
 * Kinematics.
 * ------------------------------------------------------------------------------------ */

/* Eq. (4) in normalised units: chi = eps_r sqrt((gamma E + p x B)^2 - (p.E)^2). */
double or_chi_lepton(const double p[3], const double E[3], const double B[3], double eps_r) {
  double gamma = sqrt(1.0 + p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  double v0 = gamma * E[0] + (p[1] * B[2] - p[2] * B[1]);
  double v1 = gamma * E[1] + (p[2] * B[0] - p[0] * B[2]);
  double v2 = gamma * E[2] + (p[0] * B[1] - p[1] * B[0]);
  double pe = p[0] * E[0] + p[1] * E[1] + p[2] * E[2];
  double r = v0 * v0 + v1 * v1 + v2 * v2 - pe * pe;
  if (r < 0.0) r = 0.0;
  return eps_r * sqrt(r);
}

/* Eqs. (31)-(32): chi_gamma = (hbar omega / m c^2) H_eff^gamma / E_S with
 * H_eff^gamma = sqrt((E + khat x B)^2 - (khat.E)^2). */
double or_chi_photon(const double k[3], const double E[3], const double B[3], double eps_r) {
  double kabs = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  if (!(kabs > 0.0)) return 0.0;
  double n0 = k[0] / kabs, n1 = k[1] / kabs, n2 = k[2] / kabs;
  double v0 = E[0] + (n1 * B[2] - n2 * B[1]);
  double v1 = E[1] + (n2 * B[0] - n0 * B[2]);
  double v2 = E[2] + (n0 * B[1] - n1 * B[0]);
  double ne = n0 * E[0] + n1 * E[1] + n2 * E[2];
  double r = v0 * v0 + v1 * v1 + v2 * v2 - ne * ne;
  if (r < 0.0) r = 0.0;
  double H = sqrt(r);
  return kabs * H * eps_r; /* H / E_S = H * eps_r */
}

/* Boris push (Appendix A): half step in E, rotation in B, half step in E; charge q. */
void or_boris(double p[3], double q, double h, const double E[3], const double B[3]) {
  double pm[3], t[3], pp[3], s[3];
  for (int i = 0; i < 3; ++i) pm[i] = p[i] + q * 0.5 * h * E[i];
  double g = sqrt(1.0 + pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2]);
  for (int i = 0; i < 3; ++i) t[i] = q * 0.5 * h * B[i] / g;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  pp[0] = pm[0] + (pm[1] * t[2] - pm[2] * t[1]);
  pp[1] = pm[1] + (pm[2] * t[0] - pm[0] * t[2]);
  pp[2] = pm[2] + (pm[0] * t[1] - pm[1] * t[0]);
  for (int i = 0; i < 3; ++i) s[i] = 2.0 * t[i] / (1.0 + t2);
  double pl[3];
  pl[0] = pm[0] + (pp[1] * s[2] - pp[2] * s[1]);
  pl[1] = pm[1] + (pp[2] * s[0] - pp[0] * s[2]);
  pl[2] = pm[2] + (pp[0] * s[1] - pp[1] * s[0]);
  for (int i = 0; i < 3; ++i) p[i] = pl[i] + q * 0.5 * h * E[i];
}

/* CIC (trilinear) interpolation of one Yee component whose nodes sit at
 * origin + (index + off) * dx, periodic in every direction. */
static double or_cic(const float *g, const int n[3], const double dx[3], const double org[3],
                     const double off[3], const double x[3]) {
  int i0[3];
  double fr[3];
  for (int d = 0; d < 3; ++d) {
    double s = (x[d] - org[d]) / dx[d] - off[d];
    double fl = floor(s);
    fr[d] = s - fl;
    long ii = (long)fl % n[d];
    if (ii < 0) ii += n[d];
    i0[d] = (int)ii;
  }
  double acc = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        int ii = (i0[0] + a) % n[0];
        int jj = (i0[1] + b) % n[1];
        int kk = (i0[2] + c) % n[2];
        double wgt = (a ? fr[0] : 1.0 - fr[0]) * (b ? fr[1] : 1.0 - fr[1]) *
                     (c ? fr[2] : 1.0 - fr[2]);
        acc += wgt * (double)g[((long)kk * n[1] + jj) * n[0] + ii];
      }
  return acc;
}

void or_field_at(const or_field *f, const double x[3], double t, double E[3], double B[3]) {
  switch (f->kind) {
    case OR_FIELD_UNIFORM:
      for (int i = 0; i < 3; ++i) {
        E[i] = f->e0[i];
        B[i] = f->b0[i];
      }
      break;
    case OR_FIELD_ROTATING_E: {
      double ph = f->omega * t + f->phase;
      E[0] = f->amp * cos(ph);
      E[1] = f->amp * sin(ph);
      E[2] = 0.0;
      B[0] = B[1] = B[2] = 0.0;
      break;
    }
    case OR_FIELD_CP_STANDING: {
      /* two counter-propagating circularly polarised waves of amplitude amp, k = omega */
      double ph = f->omega * t + f->phase;
      double ce = 2.0 * f->amp * cos(f->omega * x[0]);
      double cb = 2.0 * f->amp * sin(f->omega * x[0]);
      E[0] = 0.0;
      E[1] = ce * cos(ph);
      E[2] = ce * sin(ph);
      B[0] = 0.0;
      B[1] = cb * cos(ph);
      B[2] = cb * sin(ph);
      break;
    }
    case OR_FIELD_LP_STANDING: {
      /* two counter-propagating linearly polarised waves: E_y = amp sin(kx) cos(ph),
       * B_z = -amp cos(kx) sin(ph), k = omega (Sec. VII avalanche) */
      double ph = f->omega * t + f->phase;
      E[0] = E[2] = 0.0;
      E[1] = f->amp * sin(f->omega * x[0]) * cos(ph);
      B[0] = B[1] = 0.0;
      B[2] = -f->amp * cos(f->omega * x[0]) * sin(ph);
      break;
    }
    case OR_FIELD_YEE: {
      static const double off[6][3] = {{0.5, 0, 0},   {0, 0.5, 0},   {0, 0, 0.5},
                                       {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};
      for (int c = 0; c < 3; ++c) E[c] = or_cic(f->grid[c], f->n, f->dx, f->origin, off[c], x);
      for (int c = 0; c < 3; ++c)
        B[c] = or_cic(f->grid[3 + c], f->n, f->dx, f->origin, off[3 + c], x);
      break;
    }
    default:
      E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = NAN;
  }
}

/* Eq. (29) with the "<<" read as dt_q = kappa * 14 (lambda_C/c) (E_S/H_eff)^(2/3), and
 * H_eff/E_S = chi/gamma from Eq. (6); lambda_C/c = 2 pi eps_r in units of 1/w_r. */
double or_dtq_lepton(double chi, double gamma, double eps_r, double kappa) {
  double h_over_es = chi / gamma;
  return kappa * 14.0 * (2.0 * OR_PI * eps_r) * pow(1.0 / h_over_es, 2.0 / 3.0);
}

/* Eq. (33): dt_q = kappa * 130 (lambda_C/c) (E_S/H_eff^gamma), H^gamma/E_S = chi_g/kabs. */
double or_dtq_photon(double chi_g, double kabs, double eps_r, double kappa) {
  double h_over_es = chi_g / kabs;
  return kappa * 130.0 * (2.0 * OR_PI * eps_r) * (1.0 / h_over_es);
}

/* Sec. IV.H: divide dt into subintervals not greater than dt_q. */
int or_substeps(double dt, double dtq, int *near_int, int *clamped) {
  double r = dt / dtq;
  *near_int = 0;
  *clamped = 0;
  double nr = nearbyint(r);
  if (nr >= 1.0 && fabs(r - nr) <= 1e-12 * nr) *near_int = 1;
  if (!(r > 1.0)) return 1;
  double c = ceil(r);
  if (c > (double)OR_NSUB_MAX) {
    *clamped = 1;
    return OR_NSUB_MAX;
  }
  return (int)c;
}

uint64_t or_child_id(uint64_t parent, uint64_t seed, int64_t step, int substep, int purpose) {
  uint32_t ctr[4] = {(uint32_t)step, ((uint32_t)substep & 0xFFFFu) | ((uint32_t)purpose << 16),
                     (uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t key[2] = {(uint32_t)parent, (uint32_t)(parent >> 32)};
  uint32_t o[4];
  or_philox4x32_10(ctr, key, o);
  uint64_t id = (((uint64_t)o[1] << 32) | (uint64_t)o[0]) | (1ull << 63);
  if (id == OR_ID_DEAD) id = OR_ID_DEAD - 1;
  return id;
}

/* The decision draw (r1, r2) of a sub-step, counter (step, substep, seed lo, seed hi); run
 * r > 0 of the reverse mode (Sec. VI) puts r in the top byte of the second word. */
static void or_draw_run(uint64_t id, uint64_t seed, int64_t step, int substep, int run,
                        double *r1, double *r2) {
  uint32_t ctr[4] = {(uint32_t)step, ((uint32_t)substep & 0xFFFFu) | ((uint32_t)run << 24),
                     (uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t key[2] = {(uint32_t)id, (uint32_t)(id >> 32)};
  uint32_t o[4];
  or_philox4x32_10(ctr, key, o);
  *r1 = or_uniform(o[0], o[1]);
  *r2 = or_uniform(o[2], o[3]);
}

/* Sec. VI, tunable generator factor: are the children of an event that fired created?  With
 * f_g > 1 the generator runs with probability 1/f_g (its own draw, purpose 5 or 6). */
static int or_generator_runs(uint64_t parent, uint64_t seed, int64_t step, int substep,
                             int purpose, double fg) {
  if (!(fg > 1.0)) return 1;
  uint32_t ctr[4] = {(uint32_t)step, ((uint32_t)substep & 0xFFFFu) | ((uint32_t)purpose << 16),
                     (uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t key[2] = {(uint32_t)parent, (uint32_t)(parent >> 32)};
  uint32_t o[4];
  or_philox4x32_10(ctr, key, o);
  return or_uniform(o[0], o[1]) < 1.0 / fg;
}

/* The weight factor of children created by a generator with factor fg. */
static double or_generator_weight(double fg) { return fg > 1.0 ? fg : 1.0; }

/* Sec. VI, the deterministic form: the generator runs once every F occasions.  The parent's
 * phase phi in [0, F) comes from its own draw (purpose 12, step word 0, so it is the same at
 * every step); its event number e makes children iff (e + phi) mod F == 0. */
static int or_generator_every(uint64_t parent, uint64_t seed, uint32_t e, int F) {
  uint32_t ctr[4] = {0u, 12u << 16, (uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t key[2] = {(uint32_t)parent, (uint32_t)(parent >> 32)};
  uint32_t o[4];
  or_philox4x32_10(ctr, key, o);
  uint64_t phi = ((uint64_t)o[0] * (uint64_t)F) >> 32;
  return ((uint64_t)e + phi) % (uint64_t)F == 0;
}

/* Are the children of this event created (every rule of Sec. VI that thins them)? */
static int or_children_made(const or_params *p, double fg, uint64_t parent, int64_t step,
                            int substep, int purpose, uint32_t e) {
  if (!(fg > 1.0)) return 1;
  if (p->f_every) return or_generator_every(parent, p->seed, e, (int)fg);
  return or_generator_runs(parent, p->seed, step, substep, purpose, fg);
}

/* ------------------------------------------------------------------------------------
 * The step.
 * ------------------------------------------------------------------------------------ */
typedef struct {
  double x[3], p[3], w;
  uint64_t id, parent;
  uint32_t birth;
  int species;
  double tau;        /* rest of the birth step after the event */
  double E[3], B[3]; /* the parent's frozen fields, inherited */
} or_child;

/* What a particle is advanced through in this step: the whole step from its state at the
 * step start, with the fields evaluated once at its position and t_n (Sec. IV.H), or, for a
 * child in its birth step, the rest of the step with its parent's fields. */
typedef struct {
  double T;
  int inherited;
  double E[3], B[3];
} or_span;

typedef struct {
  or_child *v;
  int64_t n, cap;
} or_childbuf;

static void or_push_child(or_childbuf *b, const or_child *c) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? 2 * b->cap : 1024;
    or_child *nv = (or_child *)realloc(b->v, sizeof(or_child) * (size_t)nc);
    if (!nv) abort();
    b->v = nv;
    b->cap = nc;
  }
  b->v[b->n++] = *c;
}

static void or_note_decision(or_stats *s, double P, double r2, int is_pair) {
  if (!isfinite(P)) {
    s->nonfinite++;
    return;
  }
  if (is_pair) {
    /* only decisions that made a pair: every probability >= 1 is among them */
    if (r2 < P && P > s->max_p_pair) s->max_p_pair = P;
  } else {
    if (P > s->max_p_emit) s->max_p_emit = P;
  }
  if (P >= 1.0) s->saturated++;
  if (fabs(r2 - P) < 1e-12) s->near_threshold++;
}

static void or_stats_merge(or_stats *a, const or_stats *b) {
  for (int i = 0; i < 3; ++i) {
    a->n_start[i] += b->n_start[i];
    a->advanced[i] += b->advanced[i];
  }
  a->emitted += b->emitted;
  a->pairs += b->pairs;
  a->dropped += b->dropped;
  a->saturated += b->saturated;
  a->near_threshold += b->near_threshold;
  a->nsub_near_int += b->nsub_near_int;
  a->nsub_clamped += b->nsub_clamped;
  a->nonfinite += b->nonfinite;
  a->substeps += b->substeps;
  a->nsub_refined += b->nsub_refined;
  a->children_advanced += b->children_advanced;
  a->deferred += b->deferred;
  a->photon_energy += b->photon_energy;
  if (b->max_p_emit > a->max_p_emit) a->max_p_emit = b->max_p_emit;
  if (b->max_p_pair > a->max_p_pair) a->max_p_pair = b->max_p_pair;
  for (int i = 0; i < OR_NSUB_HIST; ++i) a->nsub_hist[i] += b->nsub_hist[i];
  for (int i = 0; i < OR_SPECTRUM_BINS; ++i) a->photon_hist[i] += b->photon_hist[i];
}

static void or_lepton_advance(const or_tables *t, or_store *st, int species, int64_t j,
                              const or_field *f, const or_params *p, double tn,
                              const or_span *span, or_childbuf *cb, or_stats *s) {
  double q = (species == 0) ? -1.0 : 1.0;
  double x[3] = {st->x[j], st->y[j], st->z[j]};
  double mom[3] = {st->px[j], st->py[j], st->pz[j]};
  uint64_t id = st->id[j];
  double E[3], B[3];
  if (span->inherited) {
    for (int d = 0; d < 3; ++d) {
      E[d] = span->E[d];
      B[d] = span->B[d];
    }
  } else {
    or_field_at(f, x, tn, E, B); /* once per step (Sec. IV.H) */
  }
  double gamma = sqrt(1.0 + mom[0] * mom[0] + mom[1] * mom[1] + mom[2] * mom[2]);
  double chi = or_chi_lepton(mom, E, B, p->eps_r);
  int nsub = 1, near_int = 0, clamped = 0;
  if (p->forced_substeps > 0) {
    nsub = p->forced_substeps;
  } else if (p->adaptive && chi > 0.0) {
    nsub = or_substeps(span->T, or_dtq_lepton(chi, gamma, p->eps_r, p->kappa), &near_int,
                       &clamped);
  }
  if (!isfinite(chi)) s->nonfinite++;
  s->nsub_near_int += near_int;
  s->nsub_clamped += clamped;
  if (!span->inherited) {
    s->nsub_hist[nsub < OR_NSUB_HIST ? nsub : OR_NSUB_HIST - 1]++;
    s->advanced[species]++;
  }
  /* Sub-steps of length h, `left` of them still to go (the current one included).  Sec.
   * IV.H asks every sub-interval to satisfy Eq. (29); the lepton's effective field can grow
   * within the step (the field slows it down, or it has just radiated most of its energy), so
   * a sub-step is kept only if h <= dt_q in the state it ends in, where its event is decided.
   * Otherwise the rest of the step is cut into twice as many sub-steps of half the length and
   * the sub-step is taken again from its start (at most OR_NSUB_MAX sub-steps in all). */
  double h = span->T / (double)nsub;
  const int refine = p->forced_substeps <= 0 && p->adaptive;
  int left = nsub, k = 0;
  uint32_t nev = st->n_events ? st->n_events[j] : 0;
  while (left > 0) {
    double pn[3] = {mom[0], mom[1], mom[2]};
    or_boris(pn, q, h, E, B);
    double gn = sqrt(1.0 + pn[0] * pn[0] + pn[1] * pn[1] + pn[2] * pn[2]);
    double chin = or_chi_lepton(pn, E, B, p->eps_r);
    if (refine && chin > 0.0) {
      double dtq = or_dtq_lepton(chin, gn, p->eps_r, p->kappa);
      if (fabs(h / dtq - 1.0) <= 1e-12) s->nsub_near_int++;
      if (h > dtq) {
        if (k + 2 * left <= OR_NSUB_MAX) {
          h *= 0.5;
          left *= 2;
          s->nsub_refined++;
          continue;
        }
        s->nsub_clamped++;
      }
    }
    for (int d = 0; d < 3; ++d) mom[d] = pn[d];
    gamma = gn;
    chi = chin;
    for (int d = 0; d < 3; ++d) x[d] += h * mom[d] / gamma;
    s->substeps++;
    const int kk = k++;
    --left;
    if (!p->emission) continue;
    double dtfac = h * OR_ALPHA / p->eps_r;
    /* the generator runs R times (R > 1 in the reverse mode of Sec. VI), each run with its
     * own draw, from the momentum the lepton has before the sub-step's events */
    const int R = p->runs_photon > 1 ? p->runs_photon : 1;
    const double wrun = st->w[j] / (double)R;
    double rec[3] = {0.0, 0.0, 0.0};
    int fired = 0;
    for (int r = 0; r < R; ++r) {
      double r1, r2;
      or_draw_run(id, p->seed, p->step, kk, r, &r1, &r2);
      double Pm = or_rate_modified(t, p->backend, r1, chi, gamma, dtfac);
      or_note_decision(s, Pm, r2, 0);
      if (!(r2 < Pm)) continue;
      double delta = r1 * r1 * r1;
      double eps = delta * gamma; /* photon energy, units m c^2 */
      double pabs = sqrt(mom[0] * mom[0] + mom[1] * mom[1] + mom[2] * mom[2]);
      if (!(pabs > 0.0)) {
        s->nonfinite++;
        continue;
      }
      or_child c;
      for (int d = 0; d < 3; ++d) {
        c.p[d] = (eps / pabs) * mom[d];
        c.x[d] = x[d];
      }
      /* the lepton recoils at every event, whether or not the photon is created */
      if (R == 1) {
        for (int d = 0; d < 3; ++d) mom[d] = mom[d] - c.p[d];
      } else {
        for (int d = 0; d < 3; ++d) rec[d] = rec[d] + c.p[d];
        fired = 1;
      }
      const uint32_t e = nev++;
      s->photon_energy += wrun * eps;
      double bin = floor(10.0 * (log10(eps) + 8.0));
      if (bin >= 0.0 && bin < (double)OR_SPECTRUM_BINS) s->photon_hist[(int)bin]++;
      if (or_children_made(p, p->f_photon, id, p->step, kk, 5, e)) {
        c.w = R > 1 ? wrun : st->w[j] * or_generator_weight(p->f_photon);
        c.id = or_child_id(id, p->seed, p->step, kk, 1 | (r << 8));
        c.parent = id;
        c.birth = (uint32_t)(((uint64_t)(p->step + 1) << 14) | (uint32_t)kk);
        c.species = 2;
        c.tau = (double)(left) * h; /* the sub-steps after this one */
        for (int d = 0; d < 3; ++d) {
          c.E[d] = E[d];
          c.B[d] = B[d];
        }
        or_push_child(cb, &c);
        s->emitted++;
      }
    }
    /* reverse mode: the mean recoil of the R runs */
    if (fired)
      for (int d = 0; d < 3; ++d) mom[d] = mom[d] - rec[d] / (double)R;
  }
  st->x[j] = x[0];
  st->y[j] = x[1];
  st->z[j] = x[2];
  st->px[j] = mom[0];
  st->py[j] = mom[1];
  st->pz[j] = mom[2];
  if (st->n_events) st->n_events[j] = nev;
}

static void or_photon_advance(const or_tables *t, or_store *st, int64_t j, const or_field *f,
                              const or_params *p, double tn, const or_span *span,
                              or_childbuf *cb, or_stats *s) {
  uint64_t id = st->id[j];
  if (id == OR_ID_DEAD) return;
  double x[3] = {st->x[j], st->y[j], st->z[j]};
  double k[3] = {st->px[j], st->py[j], st->pz[j]};
  double kabs = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  if (!(kabs > 0.0) || !isfinite(kabs)) {
    s->nonfinite++;
    return;
  }
  if (!span->inherited) s->advanced[2]++;
  double E[3], B[3];
  if (span->inherited) {
    for (int d = 0; d < 3; ++d) {
      E[d] = span->E[d];
      B[d] = span->B[d];
    }
  } else {
    or_field_at(f, x, tn, E, B);
  }
  double chi_g = or_chi_photon(k, E, B, p->eps_r);
  int nsub = 1, near_int = 0, clamped = 0;
  if (p->forced_substeps > 0) {
    nsub = p->forced_substeps;
  } else if (p->adaptive && chi_g > 0.0) {
    nsub = or_substeps(span->T, or_dtq_photon(chi_g, kabs, p->eps_r, p->kappa), &near_int,
                       &clamped);
  }
  if (!isfinite(chi_g)) s->nonfinite++;
  s->nsub_near_int += near_int;
  s->nsub_clamped += clamped;
  double h = span->T / (double)nsub;
  double dtfac = h * OR_ALPHA / p->eps_r;
  int dead = 0;
  /* reverse mode (Sec. VI): the photon stands for R copies of weight w / R */
  const int R = p->runs_pair > 1 ? p->runs_pair : 1;
  double wcur = st->w[j];
  for (int kk = 0; kk < nsub; ++kk) {
    if (p->push_photons)
      for (int d = 0; d < 3; ++d) x[d] += h * (k[d] / kabs); /* photons move at c along k */
    chi_g = or_chi_photon(k, E, B, p->eps_r);
    s->substeps++;
    if (!p->pairs) continue;
    /* R runs of the pair generator (R = 1 but in the reverse mode of Sec. VI), each with
     * its own draw; every run that fires makes a pair of weight wcur / R */
    const double wc = R > 1 ? wcur / (double)R : wcur;
    int m = 0;
    for (int r = 0; r < R; ++r) {
      double r1, r2;
      or_draw_run(id, p->seed, p->step, kk, r, &r1, &r2);
      double Pp = or_rate_pair(t, p->backend, r1, chi_g, kabs, dtfac);
      or_note_decision(s, Pp, r2, 1);
      if (!(r2 < Pp)) continue;
      ++m;
      /* the photon decays at every event, whether or not the pair is created */
      if (R == 1 && !or_children_made(p, p->f_pair, id, p->step, kk, 6, 0u)) continue;
      or_child e, pos;
      for (int d = 0; d < 3; ++d) {
        e.x[d] = x[d];
        pos.x[d] = x[d];
        e.p[d] = r1 * k[d];
        pos.p[d] = (1.0 - r1) * k[d];
      }
      e.w = pos.w = R > 1 ? wc : wc * or_generator_weight(p->f_pair);
      e.parent = pos.parent = id;
      e.birth = pos.birth = (uint32_t)(((uint64_t)(p->step + 1) << 14) | (uint32_t)kk);
      e.id = or_child_id(id, p->seed, p->step, kk, 2 | (r << 8));
      pos.id = or_child_id(id, p->seed, p->step, kk, 3 | (r << 8));
      e.species = 0;
      pos.species = 1;
      e.tau = pos.tau = (double)(nsub - kk - 1) * h;
      for (int d = 0; d < 3; ++d) {
        e.E[d] = pos.E[d] = E[d];
        e.B[d] = pos.B[d] = B[d];
      }
      or_push_child(cb, &e);
      or_push_child(cb, &pos);
      s->pairs++;
    }
    if (m == R) { /* every copy decayed */
      dead = 1;
      break;
    }
    if (m > 0) wcur = wc * (double)(R - m);
  }
  st->x[j] = x[0];
  st->y[j] = x[1];
  st->z[j] = x[2];
  if (dead) st->id[j] = OR_ID_DEAD;
  else if (wcur != st->w[j]) st->w[j] = wcur;
}

/* Appends a child to its store; returns its slot, or -1 when the store is full. */
static int64_t or_append(or_store *st, const or_child *c, or_stats *s) {
  or_store *d = &st[c->species];
  if (d->count >= d->capacity) {
    s->dropped++;
    return -1;
  }
  int64_t i = d->count++;
  d->x[i] = c->x[0];
  d->y[i] = c->x[1];
  d->z[i] = c->x[2];
  d->px[i] = c->p[0];
  d->py[i] = c->p[1];
  d->pz[i] = c->p[2];
  d->w[i] = c->w;
  d->id[i] = c->id;
  d->parent[i] = c->parent;
  d->birth[i] = c->birth;
  if (d->n_events) d->n_events[i] = 0;
  return i;
}

/* A child appended in this step that is still to be advanced through the rest of it. */
typedef struct {
  int species;
  int64_t slot;
  or_span span;
} or_pending;

/* Appends every thread's children in thread order.  With `next` non-NULL the appended
 * children with time left in the step are listed there; `*n_next` counts them, and
 * `*n_later` counts every child created with time left (appended or dropped). */
static int or_append_all(or_store *st, or_childbuf *bufs, int nthreads, or_stats *s,
                         or_pending **next, int64_t *n_next, int64_t *n_later) {
  int64_t total = 0, m = 0, later = 0;
  for (int i = 0; i < nthreads; ++i) total += bufs[i].n;
  or_pending *list = NULL;
  if (next && total > 0) {
    list = (or_pending *)malloc(sizeof(or_pending) * (size_t)total);
    if (!list) return -1;
  }
  for (int i = 0; i < nthreads; ++i) {
    for (int64_t c = 0; c < bufs[i].n; ++c) {
      const or_child *ch = &bufs[i].v[c];
      if (ch->tau > 0.0) ++later;
      int64_t slot = or_append(st, ch, s);
      if (list && slot >= 0 && ch->tau > 0.0) {
        or_pending *q = &list[m++];
        q->species = ch->species;
        q->slot = slot;
        q->span.T = ch->tau;
        q->span.inherited = 1;
        for (int d = 0; d < 3; ++d) {
          q->span.E[d] = ch->E[d];
          q->span.B[d] = ch->B[d];
        }
      }
    }
    bufs[i].n = 0;
  }
  if (next) {
    *next = list;
    *n_next = m;
  }
  if (n_later) *n_later = later;
  return 0;
}

int or_step(const or_tables *t, or_store *st, const or_field *f, const or_params *p,
            or_stats *s) {
  memset(s, 0, sizeof(*s));
  /* the forms of Sec. VI that do not combine: a factor and the reverse mode on one
   * generator, a deterministic factor that is no integer, more than 64 runs */
  if ((p->f_photon > 1.0 && p->runs_photon > 1) || (p->f_pair > 1.0 && p->runs_pair > 1) ||
      p->runs_photon > 64 || p->runs_pair > 64)
    return -2;
  if (p->f_every && ((p->f_photon > 1.0 && (p->f_photon != floor(p->f_photon) ||
                                            p->f_photon > 2147483647.0)) ||
                     (p->f_pair > 1.0 && (p->f_pair != floor(p->f_pair) ||
                                          p->f_pair > 2147483647.0))))
    return -2;
  const int64_t n0[3] = {st[0].count, st[1].count, st[2].count};
  for (int i = 0; i < 3; ++i) s->n_start[i] = n0[i];
  const double tn = p->t0 + (double)p->step * p->dt;
  const int G = p->same_step_generations > 0 ? p->same_step_generations : 0;
  const int photons = p->push_photons || p->pairs;
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  or_childbuf *bufs = (or_childbuf *)calloc((size_t)nthreads, sizeof(or_childbuf));
  or_stats *ts = (or_stats *)calloc((size_t)nthreads, sizeof(or_stats));
  if (!bufs || !ts) return -1;
  const or_span whole = {p->dt, 0, {0, 0, 0}, {0, 0, 0}};
  /* the particles alive at the step start, through the whole step */
#pragma omp parallel num_threads(nthreads)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    for (int sp = 0; sp < 2; ++sp) {
#pragma omp for schedule(static)
      for (int64_t j = 0; j < n0[sp]; ++j)
        or_lepton_advance(t, &st[sp], sp, j, f, p, tn, &whole, &bufs[tid], &ts[tid]);
    }
    if (photons) {
#pragma omp for schedule(static)
      for (int64_t j = 0; j < n0[2]; ++j)
        or_photon_advance(t, &st[2], j, f, p, tn, &whole, &bufs[tid], &ts[tid]);
    }
  }
  for (int i = 0; i < nthreads; ++i) {
    or_stats_merge(s, &ts[i]);
    memset(&ts[i], 0, sizeof(or_stats));
  }
  or_pending *list = NULL;
  int64_t n_list = 0, n_later = 0;
  int rc = or_append_all(st, bufs, nthreads, s, G > 0 ? &list : NULL, &n_list, &n_later);
  /* children through the rest of their birth step, one generation at a time */
  for (int g = 1; rc == 0 && g <= G && n_list > 0; ++g) {
    s->children_advanced += n_list;
#pragma omp parallel num_threads(nthreads)
    {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
      for (int64_t c = 0; c < n_list; ++c) {
        const or_pending *q = &list[c];
        if (q->species == 2) {
          if (photons)
            or_photon_advance(t, &st[2], q->slot, f, p, tn, &q->span, &bufs[tid], &ts[tid]);
        } else {
          or_lepton_advance(t, &st[q->species], q->species, q->slot, f, p, tn, &q->span,
                            &bufs[tid], &ts[tid]);
        }
      }
    }
    for (int i = 0; i < nthreads; ++i) {
      or_stats_merge(s, &ts[i]);
      memset(&ts[i], 0, sizeof(or_stats));
    }
    free(list);
    list = NULL;
    n_list = 0;
    rc = or_append_all(st, bufs, nthreads, s, &list, &n_list, &n_later);
    if (g == G) s->deferred += n_later; /* generation G + 1: advanced from the next step */
  }
  free(list);
  for (int i = 0; i < nthreads; ++i) free(bufs[i].v);
  free(bufs);
  free(ts);
  return rc;
}

/* ------------------------------------------------------------------------------------
 * Thinning (Sec. VI, global even redistribution): remove random super-particles and share
 * their weight among all the remaining ones by the factor sum f / (sum f - f_r).
 * ------------------------------------------------------------------------------------ */
int or_thin(or_store *s, int64_t trigger, int64_t target, uint64_t seed, int64_t step,
            or_thin_record *rec) {
  rec->live_before = rec->kept = 0;
  rec->weight_before = rec->weight_after = 0.0;
  rec->factor = 1.0;
  if (s->count <= trigger) return 0; /* not examined */
  int64_t live = 0;
  double w_live = 0.0;
  for (int64_t i = 0; i < s->count; ++i)
    if (s->id[i] != OR_ID_DEAD) {
      ++live;
      w_live += s->w[i];
    }
  rec->live_before = live;
  rec->weight_before = w_live;
  rec->kept = live;
  rec->weight_after = w_live;
  rec->factor = 1.0;
  if (target >= live) return 0;
  const double q = (double)target / (double)live;
  /* which particles stay: u < q with u from the particle's own draw */
  int64_t kept = 0;
  double w_kept = 0.0;
  unsigned char *keep = (unsigned char *)malloc((size_t)(s->count > 0 ? s->count : 1));
  if (!keep) return -1;
  for (int64_t i = 0; i < s->count; ++i) {
    keep[i] = 0;
    if (s->id[i] == OR_ID_DEAD) continue;
    uint32_t ctr[4] = {(uint32_t)step, 4u << 16, (uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t key[2] = {(uint32_t)s->id[i], (uint32_t)(s->id[i] >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    if (or_uniform(o[0], o[1]) < q) {
      keep[i] = 1;
      ++kept;
      w_kept += s->w[i];
    }
  }
  /* the removed weight goes to every survivor in proportion to its own weight */
  const double factor = kept > 0 ? w_live / w_kept : 0.0;
  int64_t j = 0;
  for (int64_t i = 0; i < s->count; ++i) {
    if (!keep[i]) continue;
    s->x[j] = s->x[i];
    s->y[j] = s->y[i];
    s->z[j] = s->z[i];
    s->px[j] = s->px[i];
    s->py[j] = s->py[i];
    s->pz[j] = s->pz[i];
    s->w[j] = s->w[i] * factor;
    s->id[j] = s->id[i];
    s->parent[j] = s->parent[i];
    s->birth[j] = s->birth[i];
    if (s->n_events) s->n_events[j] = s->n_events[i];
    ++j;
  }
  free(keep);
  s->count = kept;
  rec->kept = kept;
  rec->factor = factor;
  double w_after = 0.0;
  for (int64_t i = 0; i < kept; ++i) w_after += s->w[i];
  rec->weight_after = w_after;
  return 1;
}

/* ------------------------------------------------------------------------------------
 * Thinning per cell: Sec. VI's global even redistribution applied within each block of
 * cells, to the groups holding more than max_per_cell particles.
 * ------------------------------------------------------------------------------------ */
typedef struct {
  int64_t key, slot;
} or_keyed;

static int or_keyed_cmp(const void *a, const void *b) {
  const or_keyed *u = (const or_keyed *)a, *v = (const or_keyed *)b;
  if (u->key != v->key) return u->key < v->key ? -1 : 1;
  return u->slot < v->slot ? -1 : (u->slot > v->slot ? 1 : 0);
}

/* The block of a position, or -1 for a non-finite coordinate. */
static int64_t or_block_of(const double x[3], const int n[3], const double dx[3],
                           const double origin[3], int shift, const int64_t nb[3]) {
  int64_t b[3];
  for (int d = 0; d < 3; ++d) {
    if (!isfinite(x[d])) return -1;
    const double fl = floor((x[d] - origin[d]) / dx[d]);
    double c = fmod(fl, (double)n[d]); /* exact for integers below 2^53 */
    if (c < 0.0) c += (double)n[d];
    b[d] = (int64_t)c >> shift;
  }
  return (b[2] * nb[1] + b[1]) * nb[0] + b[0];
}

int or_thin_cells(or_store *s, int is_photon, const int n[3], const double dx[3],
                  const double origin[3], int64_t max_per_cell, uint64_t seed, int64_t step,
                  or_thin_cells_record *rec) {
  memset(rec, 0, sizeof(*rec));
  /* the coarsest grouping that still numbers every block below 2^24 - 2 */
  int shift = 0;
  int64_t nb[3];
  for (;; ++shift) {
    int64_t blocks = 1;
    for (int d = 0; d < 3; ++d) {
      nb[d] = ((int64_t)n[d] + ((int64_t)1 << shift) - 1) >> shift;
      blocks *= nb[d];
    }
    if (blocks <= ((int64_t)1 << 24) - 2) break;
  }
  const int64_t nonfinite = nb[0] * nb[1] * nb[2]; /* after every block */
  or_keyed *order = (or_keyed *)malloc(sizeof(or_keyed) * (size_t)(s->count > 0 ? s->count : 1));
  double *u = (double *)malloc(sizeof(double) * (size_t)(s->count > 0 ? s->count : 1));
  unsigned char *keep = (unsigned char *)malloc((size_t)(s->count > 0 ? s->count : 1));
  double *factor = (double *)malloc(sizeof(double) * (size_t)(s->count > 0 ? s->count : 1));
  if (!order || !u || !keep || !factor) {
    free(order), free(u), free(keep), free(factor);
    return -1;
  }
  int64_t live = 0;
  for (int64_t i = 0; i < s->count; ++i) {
    if (is_photon && s->id[i] == OR_ID_DEAD) continue;
    const double x[3] = {s->x[i], s->y[i], s->z[i]};
    const int64_t b = or_block_of(x, n, dx, origin, shift, nb);
    order[live].key = b < 0 ? nonfinite : b;
    order[live].slot = i;
    ++live;
  }
  qsort(order, (size_t)live, sizeof(or_keyed), or_keyed_cmp);
  rec->live_before = live;
  for (int64_t a = 0; a < live;) {
    int64_t e = a;
    while (e < live && order[e].key == order[a].key) ++e;
    const int64_t m = e - a;
    double W = 0.0;
    for (int64_t j = a; j < e; ++j) W += s->w[order[j].slot];
    rec->groups += 1;
    rec->weight_before += W;
    if (m <= max_per_cell) {
      for (int64_t j = a; j < e; ++j) {
        keep[j] = 1;
        factor[j] = 1.0;
      }
      rec->weight_after += W;
    } else {
      rec->groups_thinned += 1;
      const double q = (double)max_per_cell / (double)m;
      double K = 0.0;
      int64_t kept = 0, first_min = a;
      for (int64_t j = a; j < e; ++j) {
        const uint64_t id = s->id[order[j].slot];
        uint32_t ctr[4] = {(uint32_t)step, 11u << 16, (uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t key[2] = {(uint32_t)id, (uint32_t)(id >> 32)};
        uint32_t o[4];
        or_philox4x32_10(ctr, key, o);
        u[j] = or_uniform(o[0], o[1]);
        keep[j] = u[j] < q;
        if (keep[j]) {
          ++kept;
          K += s->w[order[j].slot];
        }
        if (u[j] < u[first_min]) first_min = j;
      }
      if (kept == 0) { /* the group keeps its weight in its smallest draw */
        keep[first_min] = 1;
        K = s->w[order[first_min].slot];
      }
      const double f = W / K;
      double Wa = 0.0;
      for (int64_t j = a; j < e; ++j) {
        factor[j] = f;
        if (keep[j]) Wa += s->w[order[j].slot] * f;
      }
      rec->weight_after += Wa;
    }
    a = e;
  }
  /* survivors in group order; the columns are copied out first, since the order moves
   * particles both ways */
  or_store t = *s;
  const size_t nn = (size_t)(s->count > 0 ? s->count : 1);
  double *cp = (double *)malloc(sizeof(double) * nn * 7);
  uint64_t *cu = (uint64_t *)malloc(sizeof(uint64_t) * nn * 2);
  uint32_t *cb = (uint32_t *)malloc(sizeof(uint32_t) * nn * 2);
  if (!cp || !cu || !cb) {
    free(order), free(u), free(keep), free(factor), free(cp), free(cu), free(cb);
    return -1;
  }
  for (int64_t i = 0; i < s->count; ++i) {
    cp[7 * i + 0] = t.x[i], cp[7 * i + 1] = t.y[i], cp[7 * i + 2] = t.z[i];
    cp[7 * i + 3] = t.px[i], cp[7 * i + 4] = t.py[i], cp[7 * i + 5] = t.pz[i];
    cp[7 * i + 6] = t.w[i];
    cu[2 * i] = t.id[i], cu[2 * i + 1] = t.parent[i];
    cb[2 * i] = t.birth[i], cb[2 * i + 1] = t.n_events ? t.n_events[i] : 0u;
  }
  int64_t k = 0;
  for (int64_t j = 0; j < live; ++j) {
    if (!keep[j]) continue;
    const int64_t i = order[j].slot;
    s->x[k] = cp[7 * i + 0], s->y[k] = cp[7 * i + 1], s->z[k] = cp[7 * i + 2];
    s->px[k] = cp[7 * i + 3], s->py[k] = cp[7 * i + 4], s->pz[k] = cp[7 * i + 5];
    s->w[k] = cp[7 * i + 6] * factor[j];
    s->id[k] = cu[2 * i], s->parent[k] = cu[2 * i + 1];
    s->birth[k] = cb[2 * i];
    if (s->n_events) s->n_events[k] = cb[2 * i + 1];
    ++k;
  }
  s->count = k;
  rec->kept = k;
  free(order), free(u), free(keep), free(factor), free(cp), free(cu), free(cb);
  return rec->groups_thinned > 0 ? 1 : 0;
}

/* ------------------------------------------------------------------------------------
 * The cap on the children of one parent in one iteration (Sec. VII).
 * ------------------------------------------------------------------------------------ */
typedef struct {
  uint64_t parent;
  int64_t slot;
} or_by_parent;

static int or_by_parent_cmp(const void *a, const void *b) {
  const or_by_parent *u = (const or_by_parent *)a, *v = (const or_by_parent *)b;
  if (u->parent != v->parent) return u->parent < v->parent ? -1 : 1;
  return u->slot < v->slot ? -1 : (u->slot > v->slot ? 1 : 0);
}

int or_thin_children(or_store *s, int is_photon, int64_t max_per_parent, uint64_t seed,
                     int64_t step, or_thin_children_record *rec) {
  memset(rec, 0, sizeof(*rec));
  const size_t nn = (size_t)(s->count > 0 ? s->count : 1);
  or_by_parent *kids = (or_by_parent *)malloc(sizeof(or_by_parent) * nn);
  unsigned char *keep = (unsigned char *)malloc(nn);
  double *u = (double *)malloc(sizeof(double) * nn);
  if (!kids || !keep || !u) {
    free(kids), free(keep), free(u);
    return -1;
  }
  int64_t nk = 0;
  for (int64_t i = 0; i < s->count; ++i) {
    keep[i] = 1;
    if (is_photon && s->id[i] == OR_ID_DEAD) continue;
    if ((int64_t)(s->birth[i] >> 14) != step) continue;
    if (s->parent[i] == OR_NO_PARENT) continue; /* Schwinger pairs: no particle made them */
    kids[nk].parent = s->parent[i];
    kids[nk].slot = i;
    ++nk;
    rec->weight_before += s->w[i];
  }
  rec->children = nk;
  qsort(kids, (size_t)nk, sizeof(or_by_parent), or_by_parent_cmp);
  for (int64_t a = 0; a < nk;) {
    int64_t e = a;
    while (e < nk && kids[e].parent == kids[a].parent) ++e;
    const int64_t n = e - a;
    rec->groups += 1;
    if (n > max_per_parent) {
      rec->groups_thinned += 1;
      const double q = (double)max_per_parent / (double)n;
      int64_t K = 0;
      double umin = 2.0;
      for (int64_t j = a; j < e; ++j) {
        const int64_t i = kids[j].slot;
        const uint64_t id = s->id[i];
        uint32_t ctr[4] = {(uint32_t)step, 13u << 16, (uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t key[2] = {(uint32_t)id, (uint32_t)(id >> 32)};
        uint32_t o[4];
        or_philox4x32_10(ctr, key, o);
        u[i] = or_uniform(o[0], o[1]);
        keep[i] = u[i] < q;
        K += keep[i];
        if (u[i] < umin) umin = u[i];
      }
      if (K == 0) /* the group keeps its weight in its smallest draw */
        for (int64_t j = a; j < e; ++j) {
          const int64_t i = kids[j].slot;
          if (u[i] == umin) {
            keep[i] = 1;
            ++K;
          }
        }
      const double f = (double)n / (double)K;
      for (int64_t j = a; j < e; ++j)
        if (keep[kids[j].slot]) s->w[kids[j].slot] *= f;
    }
    a = e;
  }
  /* the survivors and every other particle in store order */
  int64_t k = 0;
  for (int64_t i = 0; i < s->count; ++i) {
    if (!keep[i]) continue;
    if (is_photon && s->id[i] == OR_ID_DEAD) {
      /* removed photons stay where they are among the others */
    } else if ((int64_t)(s->birth[i] >> 14) == step && s->parent[i] != OR_NO_PARENT) {
      rec->kept += 1;
      rec->weight_after += s->w[i];
    }
    if (k != i) {
      s->x[k] = s->x[i], s->y[k] = s->y[i], s->z[k] = s->z[i];
      s->px[k] = s->px[i], s->py[k] = s->py[i], s->pz[k] = s->pz[i];
      s->w[k] = s->w[i];
      s->id[k] = s->id[i], s->parent[k] = s->parent[i];
      s->birth[k] = s->birth[i];
      if (s->n_events) s->n_events[k] = s->n_events[i];
    }
    ++k;
  }
  s->count = k;
  free(kids), free(keep), free(u);
  return rec->groups_thinned > 0 ? 1 : 0;
}

/* ------------------------------------------------------------------------------------
 * Non-perturbative pair production (Sec. V.B): per grid cell and step, a pair with
 * probability R_S V c dt from the cell's field.
 * ------------------------------------------------------------------------------------ */
static double or_grid_at(const float *g, const int n[3], int64_t i, int64_t j, int64_t k) {
  i = ((i % n[0]) + n[0]) % n[0];
  j = ((j % n[1]) + n[1]) % n[1];
  k = ((k % n[2]) + n[2]) % n[2];
  return (double)g[i + (int64_t)n[0] * (j + (int64_t)n[1] * k)];
}

int or_schwinger(or_store *st, const or_field *f, double dt, double eps_r, double weight,
                 uint64_t seed, int64_t step, or_schwinger_record *rec) {
  memset(rec, 0, sizeof(*rec));
  const double vol = f->dx[0] * f->dx[1] * f->dx[2];
  const double pref = vol * dt / (4.0 * OR_PI * OR_PI * OR_PI * pow(eps_r, 4.0));
  for (int64_t k = 0; k < f->n[2]; ++k)
    for (int64_t j = 0; j < f->n[1]; ++j)
      for (int64_t i = 0; i < f->n[0]; ++i) {
        const uint64_t c = (uint64_t)(i + (int64_t)f->n[0] * (j + (int64_t)f->n[1] * k));
        rec->cells++;
        /* the cell's field: each component the mean of its four samples on the cell */
        const double ex = 0.25 * (or_grid_at(f->grid[0], f->n, i, j, k) +
                                  or_grid_at(f->grid[0], f->n, i, j + 1, k) +
                                  or_grid_at(f->grid[0], f->n, i, j, k + 1) +
                                  or_grid_at(f->grid[0], f->n, i, j + 1, k + 1));
        const double ey = 0.25 * (or_grid_at(f->grid[1], f->n, i, j, k) +
                                  or_grid_at(f->grid[1], f->n, i + 1, j, k) +
                                  or_grid_at(f->grid[1], f->n, i, j, k + 1) +
                                  or_grid_at(f->grid[1], f->n, i + 1, j, k + 1));
        const double ez = 0.25 * (or_grid_at(f->grid[2], f->n, i, j, k) +
                                  or_grid_at(f->grid[2], f->n, i + 1, j, k) +
                                  or_grid_at(f->grid[2], f->n, i, j + 1, k) +
                                  or_grid_at(f->grid[2], f->n, i + 1, j + 1, k));
        const double e = sqrt(ex * ex + ey * ey + ez * ez) * eps_r; /* E / E_S */
        if (!(e > 0.0)) continue;
        const double P = pref * e * e * exp(-OR_PI / e);
        rec->expected += P < 1.0 ? P : 1.0;
        if (P >= 1.0) rec->saturated++;
        uint32_t key[2] = {(uint32_t)c, (uint32_t)(c >> 32)};
        uint32_t ctr[4] = {(uint32_t)step, 7u << 16, (uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t o[4];
        or_philox4x32_10(ctr, key, o);
        if (!(or_uniform(o[0], o[1]) < P)) continue;
        ctr[1] = 8u << 16;
        or_philox4x32_10(ctr, key, o);
        const double u[3] = {((double)o[0] + 0.5) * 0x1p-32, ((double)o[1] + 0.5) * 0x1p-32,
                             ((double)o[2] + 0.5) * 0x1p-32};
        or_child e_, p_;
        const int64_t cell[3] = {i, j, k};
        for (int d = 0; d < 3; ++d) {
          e_.x[d] = p_.x[d] = f->origin[d] + ((double)cell[d] + u[d]) * f->dx[d];
          e_.p[d] = p_.p[d] = 0.0;
        }
        e_.w = p_.w = weight;
        e_.parent = p_.parent = OR_NO_PARENT;
        e_.birth = p_.birth = (uint32_t)((uint64_t)(step + 1) << 14);
        e_.id = or_child_id(c, seed, step, 0, 9);
        p_.id = or_child_id(c, seed, step, 0, 10);
        e_.species = 0;
        p_.species = 1;
        e_.tau = p_.tau = 0.0;
        or_stats s;
        memset(&s, 0, sizeof(s));
        or_append(st, &e_, &s);
        or_append(st, &p_, &s);
        rec->dropped += s.dropped;
        rec->pairs++;
      }
  return 0;
}

/* ------------------------------------------------------------------------------------
 * Generator trials for the statistical pins: trial i draws (r1, r2) from Philox with
 * counter (i, i>>32, 0, 0) and the given key, then applies the generator decision.
 * ------------------------------------------------------------------------------------ */
int64_t or_emission_trials(const or_tables *t, int backend, double chi, double gamma, double dtfac,
                           uint64_t key, int64_t n, double *delta_out) {
  int64_t m = 0;
  uint32_t kk[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u}, o[4];
    or_philox4x32_10(ctr, kk, o);
    double r1 = or_uniform(o[0], o[1]);
    double r2 = or_uniform(o[2], o[3]);
    if (r2 < or_rate_modified(t, backend, r1, chi, gamma, dtfac)) delta_out[m++] = r1 * r1 * r1;
  }
  return m;
}

/* ------------------------------------------------------------------------------------
 * The three emission generators of Sec. IV.G as independent trials (the setting of the
 * paper's comparison of their spectra).
 *
 * W(x) of the standard generator (Eq. (23)) is integrated in u = log2 z, with
 * z = (2/3) delta / (chi (1 - delta)) the argument of Eq. (21)'s functions, so
 *   delta(u) = q / (1 + q),  q = 1.5 chi 2^u,  d delta / du = ln 2 delta (1 - delta).
 * The panels are the rate table's own intervals in u (the integrand is smooth inside each,
 * the interpolation's kinks sit on the panel ends), each integrated by 5-point
 * Gauss-Legendre; above z = 2^u_hi the rate is zero.  W at the panel ends is summed once,
 * as the paper suggests tabulating W, and Eq. (22)'s root is found by bisection in u inside
 * the panel that holds it.
 * ------------------------------------------------------------------------------------ */
typedef struct {
  const or_tables *t;
  int backend;
  double chi, gamma, dtfac;
} or_w_args;

static double or_w_integrand(const or_w_args *a, double u) {
  const double q = 1.5 * a->chi * exp2(u);
  const double d = q / (1.0 + q);
  return or_rate_emission(a->t, a->backend, d, a->chi, a->gamma, a->dtfac) * log(2.0) * d /
         (1.0 + q);
}

/* 5-point Gauss-Legendre on [lo, hi]: nodes 0, +-sqrt(5 -+ 2 sqrt(10/7)) / 3 */
static double or_gl5(const or_w_args *a, double lo, double hi) {
  const double x1 = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0;
  const double x2 = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
  const double w0 = 128.0 / 225.0;
  const double w1 = (322.0 + 13.0 * sqrt(70.0)) / 900.0;
  const double w2 = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
  const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
  return h * (w0 * or_w_integrand(a, c) +
              w1 * (or_w_integrand(a, c - h * x1) + or_w_integrand(a, c + h * x1)) +
              w2 * (or_w_integrand(a, c - h * x2) + or_w_integrand(a, c + h * x2)));
}

typedef struct {
  int n;         /* panels */
  double *edge;  /* n + 1 panel ends in u */
  double *cum;   /* W at the panel ends */
} or_w_table;

/* panels from u(delta_min) to u_hi on the table's grid u_lo + k du (continued below u_lo) */
static int or_w_table_build(const or_w_args *a, double delta_min, or_w_table *w) {
  const or_tables *t = a->t;
  const double u0 = log2((2.0 / 3.0) * delta_min / (a->chi * (1.0 - delta_min)));
  const double top = t->u_hi;
  w->n = 0;
  w->edge = w->cum = NULL;
  if (!(u0 < top)) return 0; /* no rate above delta_min */
  const double k0 = floor((u0 - t->u_lo) / t->du) + 1.0; /* first grid point above u0 */
  const int n = 1 + (int)ceil((top - (t->u_lo + k0 * t->du)) / t->du);
  w->edge = (double *)malloc((size_t)(n + 1) * sizeof(double));
  w->cum = (double *)malloc((size_t)(n + 1) * sizeof(double));
  if (!w->edge || !w->cum) return -1;
  w->edge[0] = u0;
  for (int k = 1; k <= n; ++k) {
    const double e = t->u_lo + (k0 + k - 1) * t->du;
    w->edge[k] = e < top ? e : top;
  }
  w->cum[0] = 0.0;
  for (int k = 0; k < n; ++k) w->cum[k + 1] = w->cum[k] + or_gl5(a, w->edge[k], w->edge[k + 1]);
  w->n = n;
  return 0;
}

static void or_w_table_free(or_w_table *w) {
  free(w->edge);
  free(w->cum);
}

/* W at u, inside the table's range */
static double or_w_at(const or_w_args *a, const or_w_table *w, double u) {
  if (w->n == 0 || u <= w->edge[0]) return 0.0;
  if (u >= w->edge[w->n]) return w->cum[w->n];
  int k = 0;
  while (w->edge[k + 1] <= u) ++k;
  return w->cum[k] + or_gl5(a, w->edge[k], u);
}

double or_standard_w(const or_tables *t, int backend, double chi, double gamma, double dtfac,
                     double delta_min, double x) {
  const or_w_args a = {t, backend, chi, gamma, dtfac};
  or_w_table w;
  if (or_w_table_build(&a, delta_min, &w) != 0) return NAN;
  const double r = or_w_at(&a, &w, log2((2.0 / 3.0) * x / (chi * (1.0 - x))));
  or_w_table_free(&w);
  return r;
}

int64_t or_generator_trials(const or_tables *t, int backend, int generator, double chi,
                            double gamma, double dtfac, double delta_min, uint64_t key,
                            int64_t first, int64_t n, double *delta_out) {
  if (generator < OR_GEN_MODIFIED || generator > OR_GEN_STANDARD) return -1;
  if (generator == OR_GEN_STANDARD && !(delta_min > 0.0 && delta_min < 1.0)) return -1;
  const or_w_args a = {t, backend, chi, gamma, dtfac};
  or_w_table wt = {0, NULL, NULL};
  if (generator == OR_GEN_STANDARD && or_w_table_build(&a, delta_min, &wt) != 0) return -1;
  const double w1 = wt.n ? wt.cum[wt.n] : 0.0; /* W(1), the total probability */
  int64_t m = 0;
  const uint32_t kk[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : m)
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t trial = (uint64_t)(first + i);
    uint32_t ctr[4] = {(uint32_t)trial, (uint32_t)(trial >> 32), 0u, 0u}, o[4];
    or_philox4x32_10(ctr, kk, o);
    const double r1 = or_uniform(o[0], o[1]);
    const double r2 = or_uniform(o[2], o[3]);
    double delta = 0.0;
    if (generator == OR_GEN_MODIFIED) {
      if (r2 < or_rate_modified(t, backend, r1, chi, gamma, dtfac)) delta = r1 * r1 * r1;
    } else if (generator == OR_GEN_ALTERNATIVE) {
      if (r2 < or_rate_emission(t, backend, r1, chi, gamma, dtfac)) delta = r1;
    } else if (r1 < w1) {
      /* the panel with W(edge k) <= r2 W(1) < W(edge k+1), then bisection in u inside it */
      const double target = r2 * w1;
      int lo_k = 0, hi_k = wt.n;
      while (hi_k - lo_k > 1) {
        const int mid = (lo_k + hi_k) / 2;
        if (wt.cum[mid] <= target) lo_k = mid; else hi_k = mid;
      }
      double lo = wt.edge[lo_k], hi = wt.edge[lo_k + 1];
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break; /* the bracket is down to adjacent doubles */
        if (wt.cum[lo_k] + or_gl5(&a, wt.edge[lo_k], mid) <= target) lo = mid; else hi = mid;
      }
      const double q = 1.5 * chi * exp2(0.5 * (lo + hi));
      delta = q / (1.0 + q);
    }
    delta_out[i] = delta;
    m += delta > 0.0 ? 1 : 0;
  }
  or_w_table_free(&wt);
  return m;
}

int64_t or_pair_trials(const or_tables *t, int backend, double chi_g, double kabs, double dtfac,
                       uint64_t key, int64_t n, double *delta_out) {
  int64_t m = 0;
  uint32_t kk[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u}, o[4];
    or_philox4x32_10(ctr, kk, o);
    double r1 = or_uniform(o[0], o[1]);
    double r2 = or_uniform(o[2], o[3]);
    if (r2 < or_rate_pair(t, backend, r1, chi_g, kabs, dtfac)) delta_out[m++] = r1;
  }
  return m;
}
