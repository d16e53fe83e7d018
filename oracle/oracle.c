/*
 * Plain FP64 CPU oracle — TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Each function follows the passage of the paper named in its comment and is
 * written for reading, not for speed: scalar loops, fixed summation order,
 * no blocking, no fusion.  Compile with -O2 -ffp-contract=off.  Loops whose
 * iterations are independent (per particle, per cell, per mesh plane) carry an
 * OpenMP pragma; every sum over them stays serial, so the results do not
 * depend on the thread count.
 *
 * Pins (tests/test_oracle_*.py) check this file against what the paper and the
 * mathematics fix: numpy's Philox, closed forms, conservation laws, quadrature of
 * the defining integrals, brute force on tiny inputs and the expected orders of
 * accuracy.  The shape of the paper's example cross section (Fig. 1a) is not in
 * the text; only its maximum is pinned (through Table 1): "parity unpinned" for
 * the sigma_n values themselves.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define PI_D 3.14159265358979323846264338327950288
#define TWO_PI_D 6.28318530717958647692528676655900577

enum { TAG_INIT = 1, TAG_COLL = 2, TAG_REDRAW = 3, TAG_NPAIRS = 4 };

/* ======================================================================== */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11, "Parallel random       */
/* numbers: as easy as 1, 2, 3"): ten rounds of two 64x64->128 multiplies,   */
/* Weyl key schedule.                                                       */
/* ======================================================================== */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
/* (w >> 12) + 1/2 needs at most 53 bits, so the map is exact and never reaches 0 or 1 */
double orc_u01_open(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1.0p-52; }

/* floor(U * n) for U = (w >> 11) 2^-53, done exactly in integers (Algorithm 1,
 * "floor(rand_num() * N_p^cell)", 0-based). */
int64_t orc_index_below(uint64_t w, int64_t n) {
  unsigned __int128 p = (unsigned __int128)(w >> 11) * (unsigned __int128)(uint64_t)n;
  return (int64_t)(p >> 53);
}

static void rng_block(uint64_t seed, uint32_t rep, uint64_t entity, uint64_t step,
                      uint64_t tag, uint64_t call, uint64_t k, uint64_t block, uint64_t out[4]) {
  uint64_t ctr[4] = {entity, step, (tag << 56) | (call << 48) | k, block};
  uint64_t key[2] = {seed, (uint64_t)rep};
  orc_philox4x64_10(ctr, key, out);
}

/* Sec. 3.2: N_p uniform samples per coordinate, fixed for the whole run. */
void orc_init_uniforms(uint64_t seed, uint32_t rep, int64_t id, double xi[6]) {
  uint64_t b0[4], b1[4];
  rng_block(seed, rep, (uint64_t)id, 0, TAG_INIT, 0, 0, 0, b0);
  rng_block(seed, rep, (uint64_t)id, 0, TAG_INIT, 0, 0, 1, b1);
  xi[0] = orc_u01_open(b0[0]);
  xi[1] = orc_u01_open(b0[1]);
  xi[2] = orc_u01_open(b0[2]);
  xi[3] = orc_u01_open(b1[0]);
  xi[4] = orc_u01_open(b1[1]);
  xi[5] = orc_u01_open(b1[2]);
}

/* ======================================================================== */
/* Root solve of a monotone CDF: safeguarded Newton with bisection fallback. */
/* ======================================================================== */
typedef double (*cdf_fn)(double x, const void* ctx, double* density);

static double solve_cdf(cdf_fn F, const void* ctx, double target, double lo, double hi,
                        double x) {
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 400; ++it) {
    double dens;
    double r = F(x, ctx, &dens) - target;
    if (r == 0.0) return x;
    if (r > 0.0) hi = x; else lo = x;
    double xn = (dens > 0.0) ? x - r / dens : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (xn == lo || xn == hi) return xn;
    if (fabs(xn - x) <= 2.0 * DBL_EPSILON * fabs(xn)) return xn;
    x = xn;
  }
  return x;
}

/* ======================================================================== */
/* Manufactured solution, paper family (Sec. 5.2) and configuration family. */
/* ======================================================================== */
static const double PHI_SHIFT[3] = {1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0};

typedef struct {
  const orc_problem* P;
  int dim;
  double t;
  double a; /* cfg family z: amplitude A sin(2 pi x/L) sin(2 pi y/L) */
} cdf_ctx;

/* Sec. 5.2, f_x, f_y, f_z and their CDFs (integrals from 0). */
static double paper_fx1(const orc_problem* P, int dim, double x, double t) {
  double L = P->L[dim], e = exp(t / P->T), s = x / L;
  if (dim == 0) return (1.0 + (e / 5.0) * sin(TWO_PI_D * s)) / L;
  if (dim == 1) return (1.0 + (1.0 / 5.0) * sin(TWO_PI_D * (s - 3.0 * e / 20.0))) / L;
  return (1.0 - (e / 6.0) * sin(TWO_PI_D * (s + e / 15.0))) / L;
}

static double paper_Fx1(const orc_problem* P, int dim, double x, double t) {
  double L = P->L[dim], e = exp(t / P->T), s = x / L;
  if (dim == 0) return s + (e / 5.0) * (1.0 - cos(TWO_PI_D * s)) / TWO_PI_D;
  if (dim == 1) {
    double c = 3.0 * e / 20.0;
    return s + (cos(TWO_PI_D * c) - cos(TWO_PI_D * (s - c))) / (10.0 * PI_D);
  }
  double b = e / 15.0;
  return s - (e / (12.0 * PI_D)) * (cos(TWO_PI_D * b) - cos(TWO_PI_D * (s + b)));
}

/* d/dt of the CDF at fixed x (numerator of xdot^M in Sec. 3.2). */
static double paper_dFdt1(const orc_problem* P, int dim, double x, double t) {
  double L = P->L[dim], T = P->T, e = exp(t / T), s = x / L;
  if (dim == 0) return (e / (5.0 * T)) * (1.0 - cos(TWO_PI_D * s)) / TWO_PI_D;
  if (dim == 1) {
    double c = 3.0 * e / 20.0, cdot = c / T;
    /* d/dt (cos 2 pi c - cos 2 pi (s - c)) / (10 pi) */
    return (-TWO_PI_D * cdot * sin(TWO_PI_D * c) - TWO_PI_D * cdot * sin(TWO_PI_D * (s - c))) /
           (10.0 * PI_D);
  }
  double b = e / 15.0, bdot = b / T, edot = e / T;
  double bracket = cos(TWO_PI_D * b) - cos(TWO_PI_D * (s + b));
  double dbracket = -TWO_PI_D * bdot * sin(TWO_PI_D * b) + TWO_PI_D * bdot * sin(TWO_PI_D * (s + b));
  return -(edot / (12.0 * PI_D)) * bracket - (e / (12.0 * PI_D)) * dbracket;
}

static double paper_pos_cdf(double x, const void* vctx, double* dens) {
  const cdf_ctx* c = (const cdf_ctx*)vctx;
  *dens = paper_fx1(c->P, c->dim, x, c->t);
  return paper_Fx1(c->P, c->dim, x, c->t);
}

/* Configuration family: density (N/V)(1 + A sin sin sin) on the box; the x and y
 * marginals are uniform and z given (x, y) has CDF
 * z/L + a (1 - cos 2 pi z/L)/(2 pi), a = A sin(2 pi x/L) sin(2 pi y/L). */
static double cfg_z_cdf(double z, const void* vctx, double* dens) {
  const cdf_ctx* c = (const cdf_ctx*)vctx;
  double L = c->P->L[2], s = z / L;
  *dens = (1.0 + c->a * sin(TWO_PI_D * s)) / L;
  return s + c->a * (1.0 - cos(TWO_PI_D * s)) / TWO_PI_D;
}

/* Eq. fv integrated: G(a) = (1 + erf a)/2 - a exp(-a^2)/sqrt(pi), a = v / vhat. */
static double paper_G(double a, const void* vctx, double* dens) {
  (void)vctx;
  double ea = exp(-a * a);
  *dens = (2.0 / sqrt(PI_D)) * a * a * ea;
  return 0.5 * (1.0 + erf(a)) - a * ea / sqrt(PI_D);
}

static double gauss_Phi(double z, const void* vctx, double* dens) {
  (void)vctx;
  *dens = exp(-0.5 * z * z) / sqrt(TWO_PI_D);
  return 0.5 * erfc(-z / sqrt(2.0));
}

/* Starting guess for the standard normal quantile: Abramowitz & Stegun 26.2.23. */
static double normal_quantile_guess(double p) {
  double pp = (p < 0.5) ? p : 1.0 - p;
  double t = sqrt(-2.0 * log(pp));
  double z = t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                     (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t);
  return (p < 0.5) ? -z : z;
}

/* Both velocity densities are even, so F^{-1}(xi) = -F^{-1}(1 - xi); the root is
 * taken on the lower half, where F - xi keeps its relative accuracy (near
 * F = 1 the residual would lose the digits of the tail).  1 - xi is exact for
 * the sampled xi. */
static double paper_a_of_xi(double xi) {
  double pp = (xi < 0.5) ? xi : 1.0 - xi;
  double a0 = cbrt(1.5 * sqrt(PI_D) * (pp - 0.5));
  double a = solve_cdf(paper_G, NULL, pp, -30.0, 0.0, a0);
  return (xi < 0.5) ? a : -a;
}

static double gauss_z_of_xi(double xi) {
  double pp = (xi < 0.5) ? xi : 1.0 - xi;
  double z = solve_cdf(gauss_Phi, NULL, pp, -40.0, 0.0, normal_quantile_guess(pp));
  return (xi < 0.5) ? z : -z;
}

/* Sec. 5.2: vhat_u, vhat_v, vhat_w and their time derivatives. */
void orc_vhat(const orc_problem* P, double t, double vh[3]) {
  double T = P->T, vb = P->vbar;
  if (P->family == ORC_FAM_CFG) {
    vh[0] = vh[1] = vh[2] = vb;
    return;
  }
  vh[0] = (1.0 + 0.2 * sin(PI_D * t / (2.0 * T))) * vb;
  vh[1] = (1.0 + 0.2 * cos(PI_D * t / T)) * vb;
  vh[2] = (1.0 + 0.2 * sin(3.0 * PI_D * t / (2.0 * T))) * vb;
}

static void vhat_dot(const orc_problem* P, double t, double vd[3]) {
  double T = P->T, vb = P->vbar;
  if (P->family == ORC_FAM_CFG) {
    vd[0] = vd[1] = vd[2] = 0.0;
    return;
  }
  vd[0] = 0.2 * (PI_D / (2.0 * T)) * cos(PI_D * t / (2.0 * T)) * vb;
  vd[1] = -0.2 * (PI_D / T) * sin(PI_D * t / T) * vb;
  vd[2] = 0.2 * (3.0 * PI_D / (2.0 * T)) * cos(3.0 * PI_D * t / (2.0 * T)) * vb;
}

/* Eq. mms_sol for positions. */
void orc_xM(const orc_problem* P, const double xi[3], double t, double x[3]) {
  if (P->family == ORC_FAM_CFG) {
    x[0] = P->L[0] * xi[0];
    x[1] = P->L[1] * xi[1];
    cdf_ctx c = {P, 2, t, 0.0};
    c.a = P->rho_amp * sin(TWO_PI_D * x[0] / P->L[0]) * sin(TWO_PI_D * x[1] / P->L[1]);
    x[2] = solve_cdf(cfg_z_cdf, &c, xi[2], 0.0, P->L[2], P->L[2] * xi[2]);
    return;
  }
  for (int d = 0; d < 3; ++d) {
    cdf_ctx c = {P, d, t, 0.0};
    x[d] = solve_cdf(paper_pos_cdf, &c, xi[d], 0.0, P->L[d], P->L[d] * xi[d]);
  }
}

/* Sec. 3.2: xdot^M = -(d/dt F_x)(x^M, t) / f_x(x^M, t). */
void orc_xdotM(const orc_problem* P, const double xm[3], double t, double xd[3]) {
  if (P->family == ORC_FAM_CFG) {
    xd[0] = xd[1] = xd[2] = 0.0;
    return;
  }
  for (int d = 0; d < 3; ++d)
    xd[d] = -paper_dFdt1(P, d, xm[d], t) / paper_fx1(P, d, xm[d], t);
}

/* Eq. mms_sol for velocities.  Paper family: F_v(v, t) = G(v / vhat(t)), so
 * v^M(t) = vhat(t) G^{-1}(xi).  Configuration family: N(0, vbar^2) per component. */
void orc_vM(const orc_problem* P, const double xi[3], double t, double v[3]) {
  if (P->family == ORC_FAM_CFG) {
    for (int d = 0; d < 3; ++d) v[d] = P->vbar * gauss_z_of_xi(xi[d]);
    return;
  }
  double vh[3];
  orc_vhat(P, t, vh);
  for (int d = 0; d < 3; ++d) v[d] = vh[d] * paper_a_of_xi(xi[d]);
}

/* Sec. 3.2: vdot^M; with F_v = G(v/vhat) this is vhat'(t) G^{-1}(xi). */
void orc_vdotM(const orc_problem* P, const double xi[3], double t, double vd[3]) {
  if (P->family == ORC_FAM_CFG) {
    vd[0] = vd[1] = vd[2] = 0.0;
    return;
  }
  double hd[3];
  vhat_dot(P, t, hd);
  for (int d = 0; d < 3; ++d) vd[d] = hd[d] * paper_a_of_xi(xi[d]);
}

/* Eq. fx: number density f_x(x, t) (integrates to N over the box). */
double orc_fx(const orc_problem* P, const double x[3], double t) {
  if (P->family == ORC_FAM_CFG) {
    double V = P->L[0] * P->L[1] * P->L[2];
    double s = sin(TWO_PI_D * x[0] / P->L[0]) * sin(TWO_PI_D * x[1] / P->L[1]) *
               sin(TWO_PI_D * x[2] / P->L[2]);
    return (P->nphys / V) * (1.0 + P->rho_amp * s);
  }
  return P->nphys * paper_fx1(P, 0, x[0], t) * paper_fx1(P, 1, x[1], t) *
         paper_fx1(P, 2, x[2], t);
}

/* Sec. 5.2: phi^M = phibar e^{t/(2T)} prod_d sin(2 pi (x_d/L_d - c_d)). */
double orc_phiM(const orc_problem* P, const double x[3], double t) {
  double r = P->phibar * exp(t / (2.0 * P->T));
  for (int d = 0; d < 3; ++d) r *= sin(TWO_PI_D * (x[d] / P->L[d] - PHI_SHIFT[d]));
  return r;
}

/* E^M = -grad phi^M (eq. potential). */
void orc_EM(const orc_problem* P, const double x[3], double t, double E[3]) {
  double amp = P->phibar * exp(t / (2.0 * P->T));
  double s[3], c[3];
  for (int d = 0; d < 3; ++d) {
    double arg = TWO_PI_D * (x[d] / P->L[d] - PHI_SHIFT[d]);
    s[d] = sin(arg);
    c[d] = cos(arg);
  }
  E[0] = -amp * (TWO_PI_D / P->L[0]) * c[0] * s[1] * s[2];
  E[1] = -amp * (TWO_PI_D / P->L[1]) * s[0] * c[1] * s[2];
  E[2] = -amp * (TWO_PI_D / P->L[2]) * s[0] * s[1] * c[2];
}

double orc_lapphiM(const orc_problem* P, const double x[3], double t) {
  double k2 = 0.0;
  for (int d = 0; d < 3; ++d) k2 += (TWO_PI_D / P->L[d]) * (TWO_PI_D / P->L[d]);
  return -k2 * orc_phiM(P, x, t);
}

/* sigma(g) g: eq. sigma_ms times g, or variable hard sphere
 * sigma_ref (g/g_ref)^(1 - 2 omega) times g. */
double orc_sigma_g(const orc_problem* P, double g) {
  if (P->sigma_model == ORC_SIGMA_POLY) {
    double r = 0.0, g2n = 1.0;
    for (int n = 0; n < P->n_sigma; ++n) {
      r += P->sigma_n[n] * g2n;
      g2n *= g * g;
    }
    return r;
  }
  return P->sigma_ref * pow(P->g_ref, 2.0 * P->omega - 1.0) * pow(g, 2.0 - 2.0 * P->omega);
}

/* Sec. 5.2: (sigma g)_max over [0, g_max]. */
double orc_sigma_g_max(const orc_problem* P) {
  if (P->sigma_model == ORC_SIGMA_VHS) {
    /* nondecreasing in g for omega <= 1 */
    return orc_sigma_g(P, P->g_max);
  }
  /* polynomial in G = g^2 of degree n_sigma - 1 <= 2: candidates are the ends
   * and the interior critical point of the quadratic. */
  double best = orc_sigma_g(P, 0.0);
  double e = orc_sigma_g(P, P->g_max);
  if (e > best) best = e;
  if (P->n_sigma == 3 && P->sigma_n[2] != 0.0) {
    double G = -P->sigma_n[1] / (2.0 * P->sigma_n[2]);
    if (G > 0.0 && G < P->g_max * P->g_max) {
      double c = orc_sigma_g(P, sqrt(G));
      if (c > best) best = c;
    }
  }
  return best;
}

/* Hard-sphere integral for a Gaussian f_v with variance s^2 per component:
 * int g (v_q - v_p) f_v dv_q = -s^2 K(|v_p|/s) v_p/|v_p|, with
 * K(l) = [(l^4 + 2 l^2 - 1) erf(l/sqrt 2) + 2 l (l^2 + 1) phi_N(l)] / l^2.
 * For small l the same expression is summed as its Taylor series. */
double orc_hs_K(double lam) {
  if (lam < 0.5) {
    /* erf(l/sqrt2) = sqrt(2/pi) sum a_n l^(2n+1), 2 l phi_N(l) = sqrt(2/pi) sum b_n l^(2n+1),
     * a_n = (-1)^n / (2^n n! (2n+1)),  b_n = (-1)^n / (2^n n!). */
    double a[40], b[40];
    double fact = 1.0, pow2 = 1.0;
    for (int n = 0; n < 40; ++n) {
      if (n > 0) { fact *= n; pow2 *= 2.0; }
      double sgn = (n % 2) ? -1.0 : 1.0;
      b[n] = sgn / (pow2 * fact);
      a[n] = b[n] / (2.0 * n + 1.0);
    }
    double sum = 0.0;
    for (int j = 1; j < 38; ++j) {
      double c = (j >= 2 ? a[j - 2] : 0.0) + 2.0 * a[j - 1] - a[j] + b[j - 1] + b[j];
      sum += c * pow(lam, 2.0 * j - 1.0);
    }
    return sqrt(2.0 / PI_D) * sum;
  }
  double l2 = lam * lam;
  double phiN = exp(-0.5 * l2) / sqrt(TWO_PI_D);
  return ((l2 * l2 + 2.0 * l2 - 1.0) * erf(lam / sqrt(2.0)) + 2.0 * lam * (l2 + 1.0) * phiN) / l2;
}

/* Eq. vel_change_1c without its prefactor: int sigma(g) g (v_q - v_p) f_v(v_q, t) dv_q.
 * Polynomial cross section: sum_n sigma_n f_n (eq. vel_change_3, eq. fn), with the
 * paper's printed f_0, f_1, f_2 for the paper f_v and the same moments expansion
 * for the Gaussian (m2 = s^2, m4 = 3 s^4 per component). */
int orc_source_integral(const orc_problem* P, const double vp[3], double t, double out[3]) {
  if (P->sigma_model == ORC_SIGMA_VHS) {
    if (P->omega == 1.0) { /* Maxwell molecules: sigma g = sigma_ref g_ref; E[v_q] = 0 */
      double c = P->sigma_ref * P->g_ref;
      for (int i = 0; i < 3; ++i) out[i] = -c * vp[i];
      return 0;
    }
    if (P->omega == 0.5 && P->family == ORC_FAM_CFG) { /* hard sphere */
      double s = P->vbar;
      double sp = sqrt(vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2]);
      if (sp == 0.0) {
        out[0] = out[1] = out[2] = 0.0;
        return 0;
      }
      double K = orc_hs_K(sp / s);
      for (int i = 0; i < 3; ++i) out[i] = -P->sigma_ref * s * s * K * vp[i] / sp;
      return 0;
    }
    return -1;
  }
  double fn[3][3];
  double u2 = vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2];
  if (P->family == ORC_FAM_PAPER) {
    double vh[3];
    orc_vhat(P, t, vh);
    double vh2[3] = {vh[0] * vh[0], vh[1] * vh[1], vh[2] * vh[2]};
    double V2 = vh2[0] + vh2[1] + vh2[2];
    double cross = vh2[0] * vp[0] * vp[0] + vh2[1] * vp[1] * vp[1] + vh2[2] * vp[2] * vp[2];
    for (int i = 0; i < 3; ++i) {
      double prod_other = 1.0;
      for (int j = 0; j < 3; ++j)
        if (j != i) prod_other *= vh2[j];
      fn[0][i] = -vp[i];
      fn[1][i] = -0.5 * (3.0 * V2 + 6.0 * vh2[i] + 2.0 * u2) * vp[i];
      fn[2][i] = -0.25 *
                 (15.0 * V2 * V2 + 36.0 * vh2[i] * vh2[i] + 24.0 * u2 * vh2[i] + 4.0 * u2 * u2 +
                  24.0 * vh2[i] * V2 + 12.0 * u2 * V2 + 24.0 * cross - 12.0 * prod_other) *
                 vp[i];
    }
  } else {
    double m2 = P->vbar * P->vbar, m4 = 3.0 * m2 * m2;
    for (int i = 0; i < 3; ++i) {
      double ui = vp[i];
      double s1 = 0.0, s2 = 0.0, pr = 1.0;
      for (int j = 0; j < 3; ++j) {
        if (j == i) continue;
        double uj2 = vp[j] * vp[j];
        s1 += m2 + uj2;
        s2 += m4 + 6.0 * uj2 * m2 + uj2 * uj2;
        pr *= m2 + uj2;
      }
      fn[0][i] = -ui;
      fn[1][i] = -ui * (3.0 * m2 + ui * ui + s1);
      fn[2][i] = -ui * (5.0 * m4 + 10.0 * ui * ui * m2 + ui * ui * ui * ui + s2 + 2.0 * pr +
                        2.0 * (3.0 * m2 + ui * ui) * s1);
    }
  }
  for (int i = 0; i < 3; ++i) {
    double r = 0.0;
    for (int n = 0; n < P->n_sigma; ++n) r += P->sigma_n[n] * fn[n][i];
    out[i] = r;
  }
  return 0;
}

/* ======================================================================== */
/* Mesh: nodes x_i = i h (periodic), cells [i h, (i+1) h).                  */
/* ======================================================================== */
static int64_t nnodes(const orc_disc* D) { return (int64_t)D->nc[0] * D->nc[1] * D->nc[2]; }

static int64_t node_index(const orc_disc* D, int i, int j, int k) {
  i = ((i % D->nc[0]) + D->nc[0]) % D->nc[0];
  j = ((j % D->nc[1]) + D->nc[1]) % D->nc[1];
  k = ((k % D->nc[2]) + D->nc[2]) % D->nc[2];
  return ((int64_t)k * D->nc[1] + j) * D->nc[0] + i;
}

/* Cell index and offset in cell units of a position in [0, L). */
static void locate(const orc_problem* P, const orc_disc* D, const double x[3], int c[3],
                   double o[3]) {
  for (int d = 0; d < 3; ++d) {
    double inv_h = (double)D->nc[d] / P->L[d];
    double s = x[d] * inv_h;
    int i = (int)floor(s);
    if (i < 0) i = 0;
    if (i > D->nc[d] - 1) i = D->nc[d] - 1;
    c[d] = i;
    o[d] = s - (double)i;
  }
}

/* Cloud-in-cell weight of corner (a, b, c) of the particle's cell. */
static double cic_weight(const double o[3], int a, int b, int c) {
  double wx = a ? o[0] : 1.0 - o[0];
  double wy = b ? o[1] : 1.0 - o[1];
  double wz = c ? o[2] : 1.0 - o[2];
  return wx * wy * wz;
}

void orc_cell_keys(const orc_problem* P, const orc_disc* D, int64_t np, const double* x,
                   int32_t* key) {
#pragma omp parallel for
  for (int64_t p = 0; p < np; ++p) {
    double xp[3] = {x[p], x[np + p], x[2 * np + p]};
    int c[3];
    double o[3];
    locate(P, D, xp, c, o);
    key[p] = (int32_t)node_index(D, c[0], c[1], c[2]);
  }
}

/* Stable counting sort by cell key: count, exclusive prefix sum, place in order. */
void orc_stable_sort(int64_t np, int32_t ncell, const int32_t* key, int64_t* perm,
                     int64_t* cell_start) {
  int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
  for (int32_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
  for (int64_t p = 0; p < np; ++p) cell_start[key[p] + 1] += 1;
  for (int32_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
  for (int64_t p = 0; p < np; ++p) {
    int32_t c = key[p];
    perm[cell_start[c] + fill[c]] = p;
    fill[c] += 1;
  }
  free(fill);
}

/* Sec. 2: cloud-in-cell charge deposition, rho_i = (q w / dV) sum_p W_i(x_p). */
void orc_deposit(const orc_problem* P, const orc_disc* D, int64_t np, const double* x,
                 double* rho) {
  int64_t nn = nnodes(D);
  for (int64_t i = 0; i < nn; ++i) rho[i] = 0.0;
  for (int64_t p = 0; p < np; ++p) {
    double xp[3] = {x[p], x[np + p], x[2 * np + p]};
    int c[3];
    double o[3];
    locate(P, D, xp, c, o);
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx)
          rho[node_index(D, c[0] + cx, c[1] + cy, c[2] + cz)] += cic_weight(o, cx, cy, cz);
  }
  double dV = (P->L[0] / D->nc[0]) * (P->L[1] / D->nc[1]) * (P->L[2] / D->nc[2]);
  double w = P->nphys / (double)D->np;
  double scale = P->q * w / dV;
  for (int64_t i = 0; i < nn; ++i) rho[i] *= scale;
}

static void node_position(const orc_problem* P, const orc_disc* D, int64_t n, double x[3]) {
  int i = (int)(n % D->nc[0]);
  int j = (int)((n / D->nc[0]) % D->nc[1]);
  int k = (int)(n / ((int64_t)D->nc[0] * D->nc[1]));
  x[0] = i * (P->L[0] / D->nc[0]);
  x[1] = j * (P->L[1] / D->nc[1]);
  x[2] = k * (P->L[2] / D->nc[2]);
}

/* Eq. poisson_mms at the nodes, spatial mean removed (Sec. 2).
 * 7-point form: b_i = lap phi^M(x_i) - (rho_i - q f_x(x_i)) / eps0, pointwise.
 * Q1 form (Galerkin, divided by the cell volume): the particle charge enters as
 * rho_i = (q w / dV) sum_p N_i(x_p), which is exactly (1/dV) int rho N_i for
 * point charges; the manufactured terms m = lap phi^M + q f_x / eps0 enter as
 * (1/dV) (M m)_i with the consistent Q1 mass matrix M applied to their nodal
 * values: the tensor product of (1, 4, 1) / 6 along each axis. */
void orc_rhs(const orc_problem* P, const orc_disc* D, const double* rho, double t, double* b) {
  int64_t nn = nnodes(D);
  double* m = (double*)malloc(sizeof(double) * (size_t)nn);
  for (int64_t n = 0; n < nn; ++n) {
    double xn[3];
    node_position(P, D, n, xn);
    double v = orc_lapphiM(P, xn, t);
    if (P->particles_to_field) v += P->q * orc_fx(P, xn, t) / P->eps0;
    m[n] = v;
  }
  double sum = 0.0;
  for (int k = 0; k < D->nc[2]; ++k)
    for (int j = 0; j < D->nc[1]; ++j)
      for (int i = 0; i < D->nc[0]; ++i) {
        int64_t n = node_index(D, i, j, k);
        double v;
        if (D->poisson_op == ORC_OP_Q1) {
          static const double w1[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
          v = 0.0;
          for (int c = -1; c <= 1; ++c)
            for (int bb = -1; bb <= 1; ++bb)
              for (int a = -1; a <= 1; ++a)
                v += w1[a + 1] * w1[bb + 1] * w1[c + 1] * m[node_index(D, i + a, j + bb, k + c)];
        } else {
          v = m[n];
        }
        if (P->particles_to_field) v -= rho[n] / P->eps0;
        b[n] = v;
        sum += v;
      }
  free(m);
  double mean = sum / (double)nn;
  for (int64_t n = 0; n < nn; ++n) b[n] -= mean;
}

/* Periodic Laplacian L of the field discretization.  7-point: the second
 * differences (phi_{i-1} - 2 phi_i + phi_{i+1}) / h^2 summed over the axes.
 * Q1 (minus the trilinear stiffness divided by the cell volume, Sec. 4.2):
 * along each axis d the second difference in d times the 1-D mass weights
 * (1, 4, 1) / 6 in the two other axes, summed over d (27 points). */
void orc_laplacian(const orc_disc* D, const orc_problem* P, const double* phi, double* out) {
  double ih2[3];
  for (int d = 0; d < 3; ++d) {
    double h = P->L[d] / D->nc[d];
    ih2[d] = 1.0 / (h * h);
  }
  if (D->poisson_op == ORC_OP_Q1) {
    static const double w1[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    static const double d2[3] = {1.0, -2.0, 1.0};
#pragma omp parallel for
    for (int k = 0; k < D->nc[2]; ++k)
      for (int j = 0; j < D->nc[1]; ++j)
        for (int i = 0; i < D->nc[0]; ++i) {
          double v = 0.0;
          for (int c = -1; c <= 1; ++c)
            for (int bb = -1; bb <= 1; ++bb)
              for (int a = -1; a <= 1; ++a) {
                double f = phi[node_index(D, i + a, j + bb, k + c)];
                double wx = d2[a + 1] * ih2[0] * w1[bb + 1] * w1[c + 1];
                double wy = w1[a + 1] * d2[bb + 1] * ih2[1] * w1[c + 1];
                double wz = w1[a + 1] * w1[bb + 1] * d2[c + 1] * ih2[2];
                v += (wx + wy + wz) * f;
              }
          out[node_index(D, i, j, k)] = v;
        }
    return;
  }
#pragma omp parallel for
  for (int k = 0; k < D->nc[2]; ++k)
    for (int j = 0; j < D->nc[1]; ++j)
      for (int i = 0; i < D->nc[0]; ++i) {
        double c = phi[node_index(D, i, j, k)];
        double lx = (phi[node_index(D, i + 1, j, k)] - 2.0 * c + phi[node_index(D, i - 1, j, k)]);
        double ly = (phi[node_index(D, i, j + 1, k)] - 2.0 * c + phi[node_index(D, i, j - 1, k)]);
        double lz = (phi[node_index(D, i, j, k + 1)] - 2.0 * c + phi[node_index(D, i, j, k - 1)]);
        out[node_index(D, i, j, k)] = lx * ih2[0] + ly * ih2[1] + lz * ih2[2];
      }
}

static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Conjugate gradients (Hestenes and Stiefel, textbook form) on A = -L_h, which
 * is SPD on zero-mean fields: A phi = -b.  The paper names no solver (Sec. 4.1
 * fixes only a second-order operator), so this is the plain method:
 *   r_0 = -b - A x_0, p_0 = r_0;
 *   alpha_i = r_i.r_i / p_i.A p_i, x_{i+1} = x_i + alpha_i p_i,
 *   r_{i+1} = r_i - alpha_i A p_i, beta_i = r_{i+1}.r_{i+1} / r_i.r_i,
 *   p_{i+1} = r_{i+1} + beta_i p_i.
 * Stops when ||r||_2 <= tol ||b||_2.  phi holds the initial guess on entry;
 * the result is projected to zero mean (Sec. 2). */
int orc_cg(const orc_disc* D, const orc_problem* P, const double* b, double* phi, double tol,
           int max_iter, int* iters, double* relres) {
  int64_t n = nnodes(D);
  double* r = (double*)malloc(sizeof(double) * n);
  double* p = (double*)malloc(sizeof(double) * n);
  double* Ap = (double*)malloc(sizeof(double) * n);
  double* rhs = (double*)malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; ++i) rhs[i] = -b[i];
  orc_laplacian(D, P, phi, Ap); /* Ap = L phi, so A phi = -Ap */
  for (int64_t i = 0; i < n; ++i) r[i] = rhs[i] + Ap[i];
  for (int64_t i = 0; i < n; ++i) p[i] = r[i];
  double bnorm = sqrt(dot(n, rhs, rhs));
  double rr = dot(n, r, r);
  int it = 0, status = 0;
  if (bnorm == 0.0) {
    for (int64_t i = 0; i < n; ++i) phi[i] = 0.0;
    rr = 0.0;
  } else {
    while (sqrt(rr) > tol * bnorm) {
      if (it >= max_iter) {
        status = -3;
        break;
      }
      orc_laplacian(D, P, p, Ap);
#pragma omp parallel for
      for (int64_t i = 0; i < n; ++i) Ap[i] = -Ap[i];
      double alpha = rr / dot(n, p, Ap);
#pragma omp parallel for
      for (int64_t i = 0; i < n; ++i) {
        phi[i] += alpha * p[i];
        r[i] -= alpha * Ap[i];
      }
      double rr_new = dot(n, r, r);
      double beta = rr_new / rr;
#pragma omp parallel for
      for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
      rr = rr_new;
      ++it;
    }
  }
  double mean = 0.0;
  for (int64_t i = 0; i < n; ++i) mean += phi[i];
  mean /= (double)n;
  for (int64_t i = 0; i < n; ++i) phi[i] -= mean;
  *iters = it;
  *relres = (bnorm == 0.0) ? 0.0 : sqrt(rr) / bnorm;
  free(r); free(p); free(Ap); free(rhs);
  return status;
}

/* E = -grad phi by central differences (Sec. 4.1, second-order gradient). */
void orc_gradient(const orc_problem* P, const orc_disc* D, const double* phi, double* E) {
  int64_t nn = nnodes(D);
  double h[3];
  for (int d = 0; d < 3; ++d) h[d] = P->L[d] / D->nc[d];
#pragma omp parallel for
  for (int k = 0; k < D->nc[2]; ++k)
    for (int j = 0; j < D->nc[1]; ++j)
      for (int i = 0; i < D->nc[0]; ++i) {
        int64_t n = node_index(D, i, j, k);
        E[n] = -(phi[node_index(D, i + 1, j, k)] - phi[node_index(D, i - 1, j, k)]) / (2.0 * h[0]);
        E[nn + n] = -(phi[node_index(D, i, j + 1, k)] - phi[node_index(D, i, j - 1, k)]) / (2.0 * h[1]);
        E[2 * nn + n] =
            -(phi[node_index(D, i, j, k + 1)] - phi[node_index(D, i, j, k - 1)]) / (2.0 * h[2]);
      }
}

/* Interpolation of nodal E to the particles with the deposition weights. */
void orc_gather(const orc_problem* P, const orc_disc* D, const double* E, int64_t np,
                const double* x, double* Ep) {
  int64_t nn = nnodes(D);
#pragma omp parallel for
  for (int64_t p = 0; p < np; ++p) {
    double xp[3] = {x[p], x[np + p], x[2 * np + p]};
    int c[3];
    double o[3];
    locate(P, D, xp, c, o);
    double e[3] = {0.0, 0.0, 0.0};
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          int64_t n = node_index(D, c[0] + cx, c[1] + cy, c[2] + cz);
          double wgt = cic_weight(o, cx, cy, cz);
          for (int d = 0; d < 3; ++d) e[d] += wgt * E[d * nn + n];
        }
    for (int d = 0; d < 3; ++d) Ep[d * np + p] = e[d];
  }
}

/* ======================================================================== */
/* Algorithm 1 (no-time-counter binary elastic collisions), run navg times   */
/* from the same pre-collision velocities and averaged (eq. avg_outcome).    */
/* v and dv_avg are SoA over the n particles of the cell: v[d * n + j].      */
/* ======================================================================== */
static uint64_t redraw_word(uint64_t seed, uint32_t rep, int64_t cell, int64_t step, int call,
                            int k, int64_t m, const uint64_t wb[4], int r) {
  if (r < 3) return wb[1 + r];
  int64_t j = (r - 3) / 4;
  uint64_t blk[4];
  rng_block(seed, rep, (uint64_t)cell, (uint64_t)step, TAG_REDRAW, (uint64_t)call, (uint64_t)k,
            ((uint64_t)m << 16) | (uint64_t)j, blk);
  return blk[(r - 3) % 4];
}

/* ---- scattering-angle recovery (eq. angle_recovery and the empirical-CDF
 * errors that follow it) ---- */
static struct {
  double* buf;
  int64_t cap, n;
} angle_rec = {NULL, 0, 0};

void orc_angle_record_start(double* buf, int64_t cap) {
  angle_rec.buf = buf;
  angle_rec.cap = cap;
  angle_rec.n = 0;
}

int64_t orc_angle_record_stop(void) {
  int64_t n = angle_rec.n;
  angle_rec.buf = NULL;
  angle_rec.cap = 0;
  return n;
}

/* chi = acos(g'_z / g), eps = atan2(g'_y, g'_x) in [0, 2 pi), from the
 * post-collision relative velocity g' and the pre-collision speed g. */
static void record_angles(double gx, double gy, double gz, double g) {
  if (!angle_rec.buf) return;
  double cz = gz / g;
  if (cz > 1.0) cz = 1.0;
  if (cz < -1.0) cz = -1.0;
  double eps = atan2(gy, gx);
  if (eps < 0.0) eps += TWO_PI_D;
  if (angle_rec.n < angle_rec.cap) {
    angle_rec.buf[2 * angle_rec.n] = acos(cz);
    angle_rec.buf[2 * angle_rec.n + 1] = eps;
  }
  ++angle_rec.n;
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Polar angle from the uniform xi, returned as cos chi.
 *   isotropic (eq. chi_iso): cos chi = 1 - 2 xi.
 *   manufactured anisotropy (Sec. 5.2, eq. fpiv_ms): with u = sin^2(chi/2)
 *     the CDF is F(u) = (13 u + 96 u^2 - 160 u^3 + 80 u^4) / 29, inverted in
 *     closed form through a(xi) and b(xi); cos chi = 1 - 2 u.
 *   variable soft sphere (eq. vss): F(chi) = 1 - cos^(2 alpha)(chi/2), whose
 *     exact inverse is cos(chi/2) = (1 - xi)^(1/(2 alpha)) (the printed
 *     xi^(1/(2 alpha)) is the same law with xi -> 1 - xi); cos chi =
 *     2 cos^2(chi/2) - 1. */
double orc_cos_chi(int chi_model, double chi_alpha, double xi) {
  if (chi_model == ORC_CHI_MMS) {
    double inner = 298924665.0 + 55680.0 * xi * (376377.0 + 2320.0 * xi * (-429.0 + 290.0 * xi));
    double a = cbrt(81909.0 - 83520.0 * xi + sqrt(inner)) / (40.0 * pow(3.0, 2.0 / 3.0));
    double b = 0.2 + a + (161.0 - 290.0 * xi) / (600.0 * a);
    double sb = sqrt(b);
    double u = 0.5 * (1.0 - sb + sqrt(0.6 - b + 29.0 / (40.0 * sb)));
    return 1.0 - 2.0 * u;
  }
  if (chi_model == ORC_CHI_VSS) return 2.0 * pow(1.0 - xi, 1.0 / chi_alpha) - 1.0;
  return 1.0 - 2.0 * xi;
}

/* F_pchi(chi) of the polar-angle model: (1 - cos chi)/2; sin^2(chi/2) -
 * (3 + 5 cos 2 chi) sin^2(chi) / 58 (Sec. 5.2); 1 - cos^(2 alpha)(chi/2). */
double orc_chi_cdf(int chi_model, double chi_alpha, double chi) {
  if (chi_model == ORC_CHI_MMS) {
    double s2 = sin(0.5 * chi), sc = sin(chi);
    return s2 * s2 - (3.0 + 5.0 * cos(2.0 * chi)) * sc * sc / 58.0;
  }
  if (chi_model == ORC_CHI_VSS) return 1.0 - pow(cos(0.5 * chi), 2.0 * chi_alpha);
  return 0.5 * (1.0 - cos(chi));
}

/* e_r = F(alpha_r) - F^M(alpha_r) with the empirical CDF F(alpha) =
 * (1/N) sum_r theta(alpha - alpha_r), theta(0) = 1, and the analytic CDFs
 * F^M_chi of the polar-angle model and F^M_eps = eps / (2 pi):
 * out = {eps_2 chi, eps_inf chi, eps_2 eps, eps_inf eps}. */
void orc_angle_errors(const double* rec, int64_t n, int chi_model, double chi_alpha,
                      double out[4]) {
  double* a = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int which = 0; which < 2; ++which) {
    for (int64_t r = 0; r < n; ++r) a[r] = rec[2 * r + which];
    qsort(a, (size_t)n, sizeof(double), cmp_double);
    double s2 = 0.0, mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      int64_t j = i;  /* theta(0) = 1: equal values share the largest rank */
      while (j + 1 < n && a[j + 1] == a[i]) ++j;
      double fm = which == 0 ? orc_chi_cdf(chi_model, chi_alpha, a[i]) : a[i] / TWO_PI_D;
      double e = (double)(j + 1) / (double)n - fm;
      s2 += e * e;
      if (fabs(e) > mx) mx = fabs(e);
    }
    out[2 * which] = n > 0 ? sqrt(s2 / (double)n) : 0.0;
    out[2 * which + 1] = mx;
  }
  free(a);
}

int orc_collide_cell(const orc_problem* P, const orc_disc* D, uint64_t seed, uint32_t rep,
                     int64_t step, int call, int64_t cell, int64_t n, const double* v,
                     double* dv_avg, orc_pair* log, int64_t log_cap, int64_t* log_n,
                     int64_t* n_accepted, int64_t* n_gmax) {
  for (int64_t j = 0; j < 3 * n; ++j) dv_avg[j] = 0.0;
  if (n < 2) return 0;
  double dV = (P->L[0] / D->nc[0]) * (P->L[1] / D->nc[1]) * (P->L[2] / D->nc[2]);
  double w = P->nphys / (double)D->np;
  double sgmax = orc_sigma_g_max(P);
  /* Algorithm 1: P_coll,max = (sigma g)_max w dt / dV */
  double pmax = sgmax * w * D->dt / dV;
  double* u = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  for (int k = 0; k < D->navg; ++k) {
    for (int64_t j = 0; j < 3 * n; ++j) u[j] = v[j];
    /* the N_pairs uniform of outcome k: word k mod 4 of the NPAIRS block of
     * outcome group k / 4 (four outcomes share one block) */
    uint64_t w0[4];
    rng_block(seed, rep, (uint64_t)cell, (uint64_t)step, TAG_NPAIRS, (uint64_t)call,
              (uint64_t)(k >> 2), 0, w0);
    /* N_pairs = floor(N (N - 1) P_max / 2 + rand) */
    int64_t npairs =
        (int64_t)floor((double)n * (double)(n - 1) * pmax / 2.0 + orc_u01(w0[k & 3]));
    for (int64_t m = 0; m < npairs; ++m) {
      uint64_t wa[4], wb[4];
      rng_block(seed, rep, (uint64_t)cell, (uint64_t)step, TAG_COLL, (uint64_t)call, (uint64_t)k,
                (uint64_t)(1 + 2 * m), wa);
      rng_block(seed, rep, (uint64_t)cell, (uint64_t)step, TAG_COLL, (uint64_t)call, (uint64_t)k,
                (uint64_t)(2 + 2 * m), wb);
      int64_t p = orc_index_below(wa[0], n);
      int64_t q = orc_index_below(wa[1], n);
      int r = 0;
      while (q == p) {
        if (r >= 3 + 4 * 65536) { /* budget exhausted: deterministic fallback */
          q = (p + 1) % n;
          break;
        }
        q = orc_index_below(redraw_word(seed, rep, cell, step, call, k, m, wb, r), n);
        ++r;
      }
      double dx = u[p] - u[q], dy = u[n + p] - u[n + q], dz = u[2 * n + p] - u[2 * n + q];
      double g = sqrt(dx * dx + dy * dy + dz * dz);
      if (g > P->g_max) ++*n_gmax;
      double u_acc = orc_u01(wa[2]), ratio = orc_sigma_g(P, g) / sgmax;
      int accepted = u_acc < ratio;
      if (accepted) {
        ++*n_accepted;
        double eps = TWO_PI_D * orc_u01(wa[3]);
        double cchi = orc_cos_chi(P->chi_model, P->chi_alpha, orc_u01(wb[0]));
        double schi = sqrt(fmax(0.0, (1.0 - cchi) * (1.0 + cchi)));
        double nv[3] = {cos(eps) * schi, sin(eps) * schi, cchi}; /* eq. n */
        if (P->coding_error == 2) {
          if (orc_u01(wb[0]) < 0.5) {
            for (int d = 0; d < 3; ++d) {
              double tmp = u[d * n + p];
              u[d * n + p] = u[d * n + q];
              u[d * n + q] = tmp;
            }
          }
        } else {
          for (int d = 0; d < 3; ++d) {
            double up = u[d * n + p], uq = u[d * n + q];
            double vcm = (P->coding_error == 1) ? 0.5 * (up - uq) : 0.5 * (up + uq);
            u[d * n + p] = vcm + 0.5 * g * nv[d];
            u[d * n + q] = vcm - 0.5 * g * nv[d];
          }
        }
        record_angles(u[p] - u[q], u[n + p] - u[n + q], u[2 * n + p] - u[2 * n + q], g);
      }
      if (log && *log_n < log_cap) {
        orc_pair rec = {cell, call, k, m, p, q, accepted, u_acc, ratio};
        log[*log_n] = rec;
      }
      if (log) ++*log_n;
    }
    for (int64_t j = 0; j < 3 * n; ++j) dv_avg[j] += u[j] - v[j];
  }
  for (int64_t j = 0; j < 3 * n; ++j) dv_avg[j] /= (double)D->navg;
  free(u);
  return 0;
}

/* ======================================================================== */
/* Whole simulation: eq. velocity_verlet with the collision calls of          */
/* eq. avg_outcome and the sources of eq. eom_mms.                           */
/* ======================================================================== */
struct orc_sim {
  orc_problem P;
  orc_disc D;
  uint64_t seed;
  uint32_t rep;
  int64_t np, nn;
  double *x, *v, *tmp;
  int64_t* id;
  int64_t* id_tmp;
  int32_t* key;
  int64_t *perm, *cell_start;
  double *rho, *phi, *E, *b, *Ep, *DA, *SA;
  int64_t step;
  int cg_iters;
  double cg_relres;
  int64_t n_acc, n_gmax;
};

orc_sim* orc_create(const orc_problem* P, const orc_disc* D, uint64_t seed, uint32_t rep) {
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->P = *P;
  s->D = *D;
  s->seed = seed;
  s->rep = rep;
  s->np = D->np;
  s->nn = nnodes(D);
  size_t np = (size_t)s->np, nn = (size_t)s->nn;
  s->x = (double*)calloc(3 * np, sizeof(double));
  s->v = (double*)calloc(3 * np, sizeof(double));
  s->tmp = (double*)calloc(3 * np, sizeof(double));
  s->id = (int64_t*)calloc(np, sizeof(int64_t));
  s->id_tmp = (int64_t*)calloc(np, sizeof(int64_t));
  s->key = (int32_t*)calloc(np, sizeof(int32_t));
  s->perm = (int64_t*)calloc(np, sizeof(int64_t));
  s->cell_start = (int64_t*)calloc(nn + 1, sizeof(int64_t));
  s->rho = (double*)calloc(nn, sizeof(double));
  s->phi = (double*)calloc(nn, sizeof(double));
  s->b = (double*)calloc(nn, sizeof(double));
  s->E = (double*)calloc(3 * nn, sizeof(double));
  s->Ep = (double*)calloc(3 * np, sizeof(double));
  s->DA = (double*)calloc(3 * np, sizeof(double));
  s->SA = (double*)calloc(3 * np, sizeof(double));
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  free(s->x); free(s->v); free(s->tmp); free(s->id); free(s->id_tmp); free(s->key);
  free(s->perm); free(s->cell_start); free(s->rho); free(s->phi); free(s->b); free(s->E);
  free(s->Ep); free(s->DA); free(s->SA);
  free(s);
}

/* Stable sort of the particle arrays by their current cell. */
static void sim_sort(orc_sim* s) {
  int64_t np = s->np;
  orc_cell_keys(&s->P, &s->D, np, s->x, s->key);
  orc_stable_sort(np, (int32_t)s->nn, s->key, s->perm, s->cell_start);
  double* arrs[2] = {s->x, s->v};
  for (int a = 0; a < 2; ++a) {
#pragma omp parallel for
    for (int64_t i = 0; i < np; ++i)
      for (int d = 0; d < 3; ++d) s->tmp[d * np + i] = arrs[a][d * np + s->perm[i]];
    memcpy(arrs[a], s->tmp, sizeof(double) * 3 * (size_t)np);
  }
  for (int64_t i = 0; i < np; ++i) s->id_tmp[i] = s->id[s->perm[i]];
  memcpy(s->id, s->id_tmp, sizeof(int64_t) * (size_t)np);
}

/* deposit -> RHS -> CG (warm start from the previous phi) -> E */
static int sim_field(orc_sim* s, double t) {
  orc_deposit(&s->P, &s->D, s->np, s->x, s->rho);
  orc_rhs(&s->P, &s->D, s->rho, t, s->b);
  int st = orc_cg(&s->D, &s->P, s->b, s->phi, s->D.cg_tol, s->D.cg_max_iter, &s->cg_iters,
                  &s->cg_relres);
  orc_gradient(&s->P, &s->D, s->phi, s->E);
  return st;
}

int orc_init(orc_sim* s) {
#pragma omp parallel for
  for (int64_t p = 0; p < s->np; ++p) {
    double xi[6], xm[3], vm[3];
    orc_init_uniforms(s->seed, s->rep, p, xi);
    orc_xM(&s->P, xi, 0.0, xm);
    orc_vM(&s->P, xi + 3, 0.0, vm);
    for (int d = 0; d < 3; ++d) {
      s->x[d * s->np + p] = xm[d];
      s->v[d * s->np + p] = vm[d];
    }
    s->id[p] = p;
  }
  sim_sort(s);
  for (int64_t i = 0; i < s->nn; ++i) s->phi[i] = 0.0;
  s->step = 0;
  s->n_acc = s->n_gmax = 0;
  return sim_field(s, 0.0);
}

/* One collision call over all cells: dv_avg = <dv> (eq. avg_outcome) and
 * dv_src = <dv^M> = (w dt (N - 1) / (2 dV)) * integral (eq. vel_change_1c). */
static int sim_collide(orc_sim* s, int call, double t, double* dv_avg, double* dv_src,
                       orc_pair* log, int64_t log_cap, int64_t* log_n) {
  int64_t np = s->np;
  double dV = (s->P.L[0] / s->D.nc[0]) * (s->P.L[1] / s->D.nc[1]) * (s->P.L[2] / s->D.nc[2]);
  double w = s->P.nphys / (double)s->D.np;
  int64_t maxn = 0;
  for (int64_t c = 0; c < s->nn; ++c) {
    int64_t n = s->cell_start[c + 1] - s->cell_start[c];
    if (n > maxn) maxn = n;
  }
  /* cells are independent; the pair log and the angle records keep the serial
   * cell order, so they run on one thread */
  const int serial = log != NULL || angle_rec.buf != NULL;
  int64_t acc = 0, gmx = 0;
  int bad = 0;
#pragma omp parallel if (!serial) reduction(+ : acc, gmx) reduction(| : bad)
  {
    double* vc = (double*)malloc(sizeof(double) * 3 * (size_t)(maxn + 1));
    double* dc = (double*)malloc(sizeof(double) * 3 * (size_t)(maxn + 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < s->nn; ++c) {
      int64_t b = s->cell_start[c], n = s->cell_start[c + 1] - b;
      for (int d = 0; d < 3; ++d)
        for (int64_t j = 0; j < n; ++j) vc[d * n + j] = s->v[d * np + b + j];
      orc_collide_cell(&s->P, &s->D, s->seed, s->rep, s->step, call, c, n, vc, dc, log, log_cap,
                       log_n, &acc, &gmx);
      double coef = (w * s->D.dt * (double)(n - 1)) / (2.0 * dV);
      for (int64_t j = 0; j < n; ++j) {
        double vp[3] = {vc[j], vc[n + j], vc[2 * n + j]}, I[3];
        if (orc_source_integral(&s->P, vp, t, I) != 0) bad = 1;
        for (int d = 0; d < 3; ++d) {
          dv_avg[d * np + b + j] = dc[d * n + j];
          dv_src[d * np + b + j] = (n >= 2) ? coef * I[d] : 0.0;
        }
      }
    }
    free(vc);
    free(dc);
  }
  s->n_acc += acc;
  s->n_gmax += gmx;
  return bad ? -1 : 0;
}

int orc_collide(orc_sim* s, int call, double t, double* dv_avg, double* dv_src, orc_pair* log,
                int64_t log_cap, int64_t* log_n) {
  if (log_n) *log_n = 0;
  int64_t dummy = 0;
  return sim_collide(s, call, t, dv_avg, dv_src, log, log_cap, log_n ? log_n : &dummy);
}

static double wrap_periodic(double x, double L) {
  if (x < 0.0) x += L;
  if (x >= L) x -= L;
  return x;
}

/* Half kick of eq. velocity_verlet at time t (E at the current positions),
 * collision terms D - S, and the manufactured term: 0.5 dt vdot^M(t), or, in the
 * isolation mode of Sec. 5.4.1, v^M(t_other) - v^M(t) (sign by direction). */
static int sim_kick(orc_sim* s, double t, double t_iso_from, double t_iso_to, const double* Dc,
                    const double* Sc) {
  int64_t np = s->np;
  orc_gather(&s->P, &s->D, s->E, np, s->x, s->Ep);
  double qm = s->P.field_to_particles ? s->P.q / s->P.m : 0.0;
  double dt = s->D.dt;
#pragma omp parallel for
  for (int64_t p = 0; p < np; ++p) {
    double xi[6], xp[3], EM[3], h[3];
    orc_init_uniforms(s->seed, s->rep, s->id[p], xi);
    for (int d = 0; d < 3; ++d) xp[d] = s->x[d * np + p];
    orc_EM(&s->P, xp, t, EM);
    if (s->P.isolate) {
      double va[3], vb[3];
      orc_vM(&s->P, xi + 3, t_iso_from, va);
      orc_vM(&s->P, xi + 3, t_iso_to, vb);
      for (int d = 0; d < 3; ++d) h[d] = vb[d] - va[d];
    } else {
      double vd[3];
      orc_vdotM(&s->P, xi + 3, t, vd);
      for (int d = 0; d < 3; ++d) h[d] = 0.5 * dt * vd[d];
    }
    for (int d = 0; d < 3; ++d) {
      double acc = dt * qm * (s->Ep[d * np + p] - EM[d]);
      double coll = Dc ? Dc[d * np + p] - Sc[d * np + p] : 0.0;
      s->v[d * np + p] = s->v[d * np + p] + 0.5 * (acc + coll) + h[d];
    }
  }
  return 0;
}

/* Drift of eq. velocity_verlet: x += dt (v + xdot^M - v^M)^{n+1/2}, with the
 * isolation substitution dt xdot^M -> x^M(t^{n+1}) - x^M(t^n). */
static void sim_drift(orc_sim* s, double t0, double th, double t1) {
  int64_t np = s->np;
  double dt = s->D.dt;
#pragma omp parallel for
  for (int64_t p = 0; p < np; ++p) {
    double xi[6], vm[3], h[3];
    orc_init_uniforms(s->seed, s->rep, s->id[p], xi);
    orc_vM(&s->P, xi + 3, th, vm);
    if (s->P.isolate) {
      double xa[3], xb[3];
      orc_xM(&s->P, xi, t0, xa);
      orc_xM(&s->P, xi, t1, xb);
      for (int d = 0; d < 3; ++d) h[d] = xb[d] - xa[d];
    } else {
      double xm[3], xd[3];
      orc_xM(&s->P, xi, th, xm);
      orc_xdotM(&s->P, xm, th, xd);
      for (int d = 0; d < 3; ++d) h[d] = dt * xd[d];
    }
    for (int d = 0; d < 3; ++d) {
      double xn = s->x[d * np + p] + dt * (s->v[d * np + p] - vm[d]) + h[d];
      s->x[d * np + p] = wrap_periodic(xn, s->P.L[d]);
    }
  }
}

int orc_step(orc_sim* s, int nsteps) {
  int st = 0;
  for (int it = 0; it < nsteps; ++it) {
    int64_t n = s->step;
    double dt = s->D.dt;
    double t0 = (double)n * dt, th = ((double)n + 0.5) * dt, t1 = ((double)n + 1.0) * dt;
    int64_t dummy = 0;
    if (s->P.collisions)
      if (sim_collide(s, 0, t0, s->DA, s->SA, NULL, 0, &dummy) != 0) st = -1;
    sim_kick(s, t0, t0, th, s->P.collisions ? s->DA : NULL, s->SA);
    sim_drift(s, t0, th, t1);
    sim_sort(s);
    int fs = sim_field(s, t1);
    if (fs != 0) st = fs;
    if (s->P.collisions)
      if (sim_collide(s, 1, th, s->DA, s->SA, NULL, 0, &dummy) != 0) st = -1;
    sim_kick(s, t1, th, t1, s->P.collisions ? s->DA : NULL, s->SA);
    s->step = n + 1;
  }
  return st;
}

/* Sec. 4.3 norms at the current time; positions by minimum image. */
int orc_errors(orc_sim* s, double out[14]) {
  int64_t np = s->np;
  double t = (double)s->step * s->D.dt;
  double sq[7] = {0}, mx[7] = {0};
  for (int64_t p = 0; p < np; ++p) {
    double xi[6], xm[3], vm[3];
    orc_init_uniforms(s->seed, s->rep, s->id[p], xi);
    orc_xM(&s->P, xi, t, xm);
    orc_vM(&s->P, xi + 3, t, vm);
    for (int d = 0; d < 3; ++d) {
      double L = s->P.L[d];
      double e = s->x[d * np + p] - xm[d];
      if (e >= 0.5 * L) e -= L;
      if (e < -0.5 * L) e += L;
      double ev = s->v[d * np + p] - vm[d];
      sq[d] += e * e;
      sq[3 + d] += ev * ev;
      if (fabs(e) > mx[d]) mx[d] = fabs(e);
      if (fabs(ev) > mx[3 + d]) mx[3 + d] = fabs(ev);
    }
  }
  for (int64_t n = 0; n < s->nn; ++n) {
    double xn[3];
    node_position(&s->P, &s->D, n, xn);
    double e = s->phi[n] - orc_phiM(&s->P, xn, t);
    sq[6] += e * e;
    if (fabs(e) > mx[6]) mx[6] = fabs(e);
  }
  for (int a = 0; a < 6; ++a) out[a] = sqrt(sq[a] / (double)np);
  out[6] = sqrt(sq[6] / (double)s->nn);
  for (int a = 0; a < 7; ++a) out[7 + a] = mx[a];
  return 0;
}

int orc_get(orc_sim* s, int what, void* dst) {
  size_t np = (size_t)s->np, nn = (size_t)s->nn;
  switch (what) {
    case ORC_X: memcpy(dst, s->x, 3 * np * sizeof(double)); return 0;
    case ORC_V: memcpy(dst, s->v, 3 * np * sizeof(double)); return 0;
    case ORC_ID: memcpy(dst, s->id, np * sizeof(int64_t)); return 0;
    case ORC_CELL_START: memcpy(dst, s->cell_start, (nn + 1) * sizeof(int64_t)); return 0;
    case ORC_RHO: memcpy(dst, s->rho, nn * sizeof(double)); return 0;
    case ORC_PHI: memcpy(dst, s->phi, nn * sizeof(double)); return 0;
    case ORC_E: memcpy(dst, s->E, 3 * nn * sizeof(double)); return 0;
    case ORC_EP:
      orc_gather(&s->P, &s->D, s->E, s->np, s->x, s->Ep);
      memcpy(dst, s->Ep, 3 * np * sizeof(double));
      return 0;
  }
  return -1;
}

/* Replace the particle positions or velocities (component-major, in the
 * current cell-sorted order).  New positions are wrapped into [0, L), the
 * particles are stable-sorted by their new cells from the current order, and
 * the field is deposited and solved at the current time, as at
 * initialisation; the CG starts from the current phi.  Returns the field
 * solve's status, or -1 for an unknown item. */
int orc_set(orc_sim* s, int what, const void* src) {
  size_t np = (size_t)s->np;
  if (what == ORC_V) {
    memcpy(s->v, src, 3 * np * sizeof(double));
    return 0;
  }
  if (what != ORC_X) return -1;
  memcpy(s->x, src, 3 * np * sizeof(double));
  for (int d = 0; d < 3; ++d)
    for (size_t p = 0; p < np; ++p) {
      double L = s->P.L[d], x = s->x[d * np + p];
      x -= floor(x / L) * L;
      if (!(x >= 0.0 && x < L)) x = 0.0;  /* rounding up to L, or non-finite */
      s->x[d * np + p] = x;
    }
  sim_sort(s);
  return sim_field(s, (double)s->step * s->D.dt);
}

int64_t orc_step_index(orc_sim* s) { return s->step; }
double orc_time(orc_sim* s) { return (double)s->step * s->D.dt; }
int orc_cg_iters(orc_sim* s) { return s->cg_iters; }
double orc_cg_relres(orc_sim* s) { return s->cg_relres; }
int64_t orc_accepted(orc_sim* s) { return s->n_acc; }
int64_t orc_gmax_events(orc_sim* s) { return s->n_gmax; }

/* Threads of the independent loops (results do not depend on it). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
