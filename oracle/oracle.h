/*
 * Plain FP64 CPU oracle for the manufactured-solution PIC/DSMC time step of
 * Freno, McDoniel, Moore & Matula, "Code-Verification Techniques for
 * Particle-in-Cell Simulations with Direct Simulation Monte Carlo Collisions".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library; the only common ground is the published
 * definition of Philox4x64-10 and the stream layout stated below, which each
 * side implements on its own.
 *
 * Everything is scalar FP64, compiled with -ffp-contract=off, and written to be
 * checked against the paper by eye.  Independent per-particle and per-cell
 * loops run on OpenMP threads; sums stay serial, so results are bitwise the
 * same for any thread count.
 *
 * Random stream layout (the paper's Algorithm 1 only says "rand_num()"):
 *   generator  Philox4x64-10, key = (seed, replicate)
 *   counter    c0 = entity (particle id or linear cell index)
 *              c1 = time step n
 *              c2 = tag << 56 | call << 48 | outcome k
 *              c3 = block index
 *   tag 1 INIT   particle id, n = 0: block 0 -> (xi_x, xi_y, xi_z, -),
 *                block 1 -> (xi_u, xi_v, xi_w, -); uniforms on (0,1)
 *   tag 4 NPAIRS cell, step, call (0 = first kick, 1 = second kick), outcome
 *                field k / 4, block 0: word k mod 4 -> the N_pairs uniform of
 *                outcome k (four consecutive outcomes share one block)
 *   tag 2 COLL   cell, step, call, outcome k: pair m uses blocks
 *                1+2m -> (p, q, U_acc, U_eps) and 2+2m -> (U_chi, q-redraw 1..3);
 *                block 0 is not used
 *   tag 3 REDRAW same entity/step/call/outcome, c3 = m << 16 | j: four further
 *                q-redraws per block j of pair m
 *   uniform on [0,1): (w >> 11) * 2^-53; on (0,1): ((w >> 12) + 1/2) * 2^-52;
 *   index below N: floor((w >> 11) * N / 2^53) in exact integer arithmetic.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FAM_PAPER = 0, ORC_FAM_CFG = 1 };
enum { ORC_SIGMA_POLY = 0, ORC_SIGMA_VHS = 1 };
/* Polar scattering angle: isotropic (eq. chi_iso), the manufactured
 * anisotropy fitted to VSS alpha = 2 (eq. pchi_ms with C_0 = 1/2, C_1 = 12/29,
 * inverse eq. fpiv_ms), variable soft sphere with exponent alpha (eq. vss). */
enum { ORC_CHI_ISO = 0, ORC_CHI_MMS = 1, ORC_CHI_VSS = 2 };

typedef struct {
  int family;              /* ORC_FAM_PAPER (Sec. 5.2 functions) or ORC_FAM_CFG */
  double L[3];             /* box lengths */
  double nphys;            /* N, physical particles in the box (eq. fx) */
  double q, m, eps0;       /* species charge, mass; permittivity */
  double T;                /* manufactured time scale */
  double vbar;             /* velocity scale: paper vbar, or Gaussian sigma_v */
  double phibar;           /* manufactured potential amplitude */
  double rho_amp;          /* cfg family: density 1 + rho_amp*sin*sin*sin */
  int sigma_model;         /* ORC_SIGMA_POLY (eq. sigma_ms) or ORC_SIGMA_VHS */
  int n_sigma;             /* number of polynomial terms, <= 3 */
  double sigma_n[3];       /* sigma(g) = sum_n sigma_n g^(2n-1) */
  double sigma_ref, g_ref, omega; /* VHS: sigma = sigma_ref (g/g_ref)^(1-2 omega) */
  double g_max;            /* (sigma g)_max is taken over [0, g_max] */
  int chi_model;           /* ORC_CHI_ISO, ORC_CHI_MMS or ORC_CHI_VSS */
  int field_to_particles;  /* 0 => q/m = 0 in the push */
  int particles_to_field;  /* 0 => q = 0 in the Poisson source */
  int collisions;          /* 0 => no DSMC */
  int isolate;             /* 1 => exact-difference substitution of Sec. 5.4.1 */
  int coding_error;        /* 0 none; 1 = v_cm sign error; 2 = swap w.p. 1/2 */
  double chi_alpha;        /* VSS exponent alpha in [1, 2] (ORC_CHI_VSS) */
} orc_problem;

typedef struct {
  int nc[3];               /* cells (= nodes, periodic) per dimension */
  int64_t np;              /* computational particles */
  double dt;
  int navg;                /* averaged independent collision outcomes */
  double cg_tol;           /* relative residual tolerance */
  int cg_max_iter;
  int poisson_op;          /* ORC_OP_FD7 or ORC_OP_Q1 */
} orc_disc;

/* Field discretization: the periodic 7-point finite-difference Laplacian with
 * a pointwise right-hand side, or the trilinear (Q1) finite elements of
 * Sec. 4.2 (27-point stiffness, Galerkin right-hand side), both divided by the
 * cell volume so that the system reads L phi = b in either case. */
enum { ORC_OP_FD7 = 0, ORC_OP_Q1 = 1 };

typedef struct orc_sim orc_sim;

/* ---- Philox and uniforms ---- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double orc_u01(uint64_t w);          /* [0,1) */
double orc_u01_open(uint64_t w);     /* (0,1) */
int64_t orc_index_below(uint64_t w, int64_t n);
void orc_init_uniforms(uint64_t seed, uint32_t rep, int64_t id, double xi[6]);

/* ---- manufactured solution (Sec. 3 and Sec. 5.2) ---- */
void orc_xM(const orc_problem* P, const double xi[3], double t, double x[3]);
void orc_vM(const orc_problem* P, const double xi[3], double t, double v[3]);
void orc_xdotM(const orc_problem* P, const double xm[3], double t, double xd[3]);
void orc_vdotM(const orc_problem* P, const double xi[3], double t, double vd[3]);
double orc_fx(const orc_problem* P, const double x[3], double t);  /* number density */
double orc_phiM(const orc_problem* P, const double x[3], double t);
void orc_EM(const orc_problem* P, const double x[3], double t, double E[3]);
double orc_lapphiM(const orc_problem* P, const double x[3], double t);
void orc_vhat(const orc_problem* P, double t, double vh[3]);
double orc_sigma_g(const orc_problem* P, double g);       /* sigma(g) * g */
double orc_sigma_g_max(const orc_problem* P);
/* int sigma(g) g (v_q - v_p) f_v(v_q, t) dv_q  (eq. vel_change_1c without prefactor) */
int orc_source_integral(const orc_problem* P, const double vp[3], double t, double out[3]);
double orc_hs_K(double lam);

/* ---- mesh stages ---- */
void orc_deposit(const orc_problem* P, const orc_disc* D, int64_t np, const double* x,
                 double* rho);
void orc_rhs(const orc_problem* P, const orc_disc* D, const double* rho, double t, double* b);
int orc_cg(const orc_disc* D, const orc_problem* P, const double* b, double* phi,
           double tol, int max_iter, int* iters, double* relres);
void orc_laplacian(const orc_disc* D, const orc_problem* P, const double* phi, double* out);
void orc_gradient(const orc_problem* P, const orc_disc* D, const double* phi, double* E);
void orc_gather(const orc_problem* P, const orc_disc* D, const double* E, int64_t np,
                const double* x, double* Ep);
void orc_cell_keys(const orc_problem* P, const orc_disc* D, int64_t np, const double* x,
                   int32_t* key);
void orc_stable_sort(int64_t np, int32_t ncell, const int32_t* key, int64_t* perm,
                     int64_t* cell_start);

/* ---- one cell, one collision call: Algorithm 1 run navg times, averaged ---- */
/* One candidate pair of Algorithm 1: where it was drawn, the pair, whether it
 * was accepted, and the two numbers the accept test compared (U < ratio with
 * ratio = sigma(g) g / (sigma g)_max). */
typedef struct {
  int64_t cell, call, k, m, p, q, accepted;
  double u_acc, ratio;
} orc_pair;
int orc_collide_cell(const orc_problem* P, const orc_disc* D, uint64_t seed, uint32_t rep,
                     int64_t step, int call, int64_t cell, int64_t n, const double* v,
                     double* dv_avg, orc_pair* log, int64_t log_cap, int64_t* log_n,
                     int64_t* n_accepted, int64_t* n_gmax);

/* Scattering-angle records (chi, eps) of every accepted collision between
 * start and stop (eq. angle_recovery); stop returns the number of collisions
 * (records beyond cap are counted, not stored). */
void orc_angle_record_start(double* buf, int64_t cap);
int64_t orc_angle_record_stop(void);
/* Empirical-CDF errors of n records against the isotropic analytic CDFs:
 * {eps_2 chi, eps_inf chi, eps_2 eps, eps_inf eps}. */
/* cos chi = cos F_pchi^{-1}(xi) of the polar-angle model (eq. chi_iso,
 * eq. fpiv_ms, eq. vss) and the model's CDF F_pchi(chi). */
double orc_cos_chi(int chi_model, double chi_alpha, double xi);
double orc_chi_cdf(int chi_model, double chi_alpha, double chi);
void orc_angle_errors(const double* rec, int64_t n, int chi_model, double chi_alpha,
                      double out[4]);

/* ---- whole simulation ---- */
orc_sim* orc_create(const orc_problem* P, const orc_disc* D, uint64_t seed, uint32_t rep);
void orc_destroy(orc_sim* s);
int orc_init(orc_sim* s);
int orc_step(orc_sim* s, int nsteps);
int orc_collide(orc_sim* s, int call, double t, double* dv_avg, double* dv_src,
                orc_pair* log, int64_t log_cap, int64_t* log_n);
/* out: l2[x,y,z,u,v,w,phi] then linf[...]; 14 doubles, at the sim's current time */
int orc_errors(orc_sim* s, double out[14]);

enum { ORC_X = 0, ORC_V = 1, ORC_ID = 2, ORC_CELL_START = 3, ORC_RHO = 4, ORC_PHI = 5,
       ORC_E = 6, ORC_EP = 7 };
int orc_get(orc_sim* s, int what, void* dst);
/* Replace positions (then wrap, stable re-sort, deposit and field solve at the
 * current time) or velocities; component-major, current sorted order. */
int orc_set(orc_sim* s, int what, const void* src);
int64_t orc_step_index(orc_sim* s);
double orc_time(orc_sim* s);
int orc_cg_iters(orc_sim* s);
double orc_cg_relres(orc_sim* s);
int64_t orc_accepted(orc_sim* s);
int64_t orc_gmax_events(orc_sim* s);
void orc_set_threads(int n);
int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
