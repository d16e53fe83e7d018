/*
 * pic.h — C ABI of the MI355X (gfx950) manufactured-solution PIC/DSMC time step.
 *
 * Method: Freno, McDoniel, Moore & Matula, "Code-Verification Techniques for
 * Particle-in-Cell Simulations with Direct Simulation Monte Carlo Collisions".
 * One species on a periodic box, electrostatic field (Sec. 2, eq. eom_full,
 * eq. poisson), binary elastic collisions by the no-time-counter algorithm
 * (Algorithm 1) averaged over N_avg independent outcomes (eq. avg_outcome),
 * manufactured positions and velocities by inverse-CDF queries (eq. mms_sol)
 * with the modified equations of motion (eq. eom_mms) integrated by velocity
 * Verlet (eq. velocity_verlet), and direct error norms (Sec. 4.3).
 *
 * Conventions for every entry point:
 *  - Return value: PIC_OK (0) on success, a negative PIC_E* code on error, a
 *    positive PIC_WARN_* code when the call succeeded with a warning.  No
 *    exception crosses the boundary.  The text of the last error of a context
 *    is available from pic_last_error().
 *  - Memory: the caller owns all device memory.  pic_workspace_size() states
 *    how many bytes of device memory one simulation needs; the caller allocates
 *    them (for example as a torch uint8 tensor on the GPU) and passes the
 *    pointer to pic_init_manufactured(), which never allocates device memory
 *    of its own.  The workspace must stay valid until pic_destroy().  Pointer
 *    arguments documented as "device" must point into GPU memory of the
 *    context's device, "host" ones into CPU memory.
 *  - Streams: all GPU work of a context is enqueued on the HIP stream given at
 *    initialisation (NULL = the default stream).  pic_step() only enqueues;
 *    pic_errors(), pic_stats() and pic_get_state() synchronise that stream.
 *    Errors of asynchronous work (a CG that did not converge, a HIP fault) are
 *    reported by the next synchronising call.
 *  - Concurrency: one context per stream; calls on one context must not
 *    overlap.  Different contexts are independent.
 *  - Determinism: results do not depend on scheduling: the cell sort, pair
 *    selection and every floating-point reduction use a fixed order, so two
 *    runs with the same inputs produce identical bits.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pic_status {
  PIC_OK = 0,
  PIC_EINVAL = -1,      /* invalid argument or unsupported combination */
  PIC_EHIP = -2,        /* a HIP runtime call failed */
  PIC_ENOCONV = -3,     /* Poisson CG hit cg_max_iter before cg_tol */
  PIC_ENONFINITE = -4,  /* a non-finite value in the particle state or norms */
  PIC_ESTATE = -5,      /* call out of order (e.g. before initialisation) */
  PIC_ESPACE = -6,      /* workspace too small */
  PIC_WARN_NAVG = 1,    /* N_avg P_coll,max >= 0.5: eq. navg_ineq not satisfied */
  PIC_WARN_GMAX = 2     /* a candidate pair had g > g_max: (sigma g)_max is taken
                           over [0, g_max] (Sec. 5.2), so such a pair may accept
                           with sigma g / (sigma g)_max > 1 */
};

enum pic_precision {
  PIC_FP64 = 0,         /* every stage in FP64 */
  PIC_MIXED = 1         /* particle stages in FP32 (cell index + FP32 offset
                           positions); Poisson CG, inverse-CDF roots and error
                           norms in FP64 */
};

enum pic_family {
  PIC_MMS_PAPER = 0,    /* the manufactured functions of Sec. 5.2 */
  PIC_MMS_CFG = 1       /* density (N/V)(1 + rho_amp sin sin sin) on the box,
                           Gaussian velocities N(0, vbar^2), phi^M of Sec. 5.2;
                           time independent except phi^M */
};

enum pic_sigma {
  PIC_SIGMA_POLY = 0,   /* eq. sigma_ms: sigma(g) = sum_n sigma_n g^(2n-1) */
  PIC_SIGMA_VHS = 1     /* sigma_ref (g / g_ref)^(1 - 2 omega); omega in {0.5, 1} */
};

/* Polar scattering angle chi = F_pchi^{-1}(xi) (eq. chi).  PIC_CHI_MMS is the
 * manufactured anisotropy of Sec. 5.2 (eq. pchi_ms with C_0 = 1/2,
 * C_1 = 12/29, closed-form inverse eq. fpiv_ms); it satisfies eq. constraint_1,
 * so the manufactured collision source is the isotropic one.  PIC_CHI_VSS is
 * the variable soft sphere of eq. vss with exponent chi_alpha (inverse
 * cos(chi/2) = (1 - xi)^(1/(2 alpha)), the exact inverse of its CDF); for
 * alpha != 1 it violates eq. constraint_1, so the manufactured source is not
 * the collision operator's expectation there (a realistic model for the angle
 * metric, not a code-verification case). */
enum pic_chi {
  PIC_CHI_ISO = 0,      /* eq. chi_iso: cos chi = 1 - 2 xi */
  PIC_CHI_MMS = 1,      /* eq. pchi_ms / eq. fpiv_ms */
  PIC_CHI_VSS = 2       /* eq. vss */
};

/* The problem, in the paper's notation (Sec. 2, Sec. 3, Sec. 5.2). */
typedef struct {
  int family;               /* enum pic_family */
  double L[3];              /* box lengths L_{x_i}; nodes at x = i L / ncell */
  double nphys;             /* N, physical particles in the box (eq. fx) */
  double q, m, eps0;        /* charge, mass, permittivity */
  double T;                 /* time scale of the manufactured functions */
  double vbar;              /* paper: vbar; cfg family: Gaussian sigma_v */
  double phibar;            /* amplitude of phi^M */
  double rho_amp;           /* cfg family density amplitude (< 1) */
  int sigma_model;          /* enum pic_sigma */
  int n_sigma;              /* 1..3 polynomial terms (PIC_SIGMA_POLY) */
  double sigma_n[3];
  double sigma_ref, g_ref, omega; /* PIC_SIGMA_VHS */
  double g_max;             /* (sigma g)_max is the maximum over [0, g_max] */
  int chi_model;            /* enum pic_chi: polar scattering-angle model */
  int field_to_particles;   /* 0 => q/m = 0 in the push (Sec. 5.4) */
  int particles_to_field;   /* 0 => q = 0 in the Poisson source (Sec. 5.4) */
  int collisions;           /* 0 => no DSMC */
  int isolate;              /* 1 => exact-difference substitution of the
                               manufactured time derivatives (Sec. 5.4.1) */
  double chi_alpha;         /* VSS exponent alpha in [1, 2] (PIC_CHI_VSS) */
  int coding_error;         /* the deliberate coding errors of Sec. 5.4.1, for
                               verification studies only: 0 none; 1 Error 1,
                               v_cm = (v_p - v_q) / 2 in the collision; 2 Error 2,
                               an accepted pair swaps its velocities when
                               U_chi < 1/2 and is left unchanged otherwise */
} pic_problem;

/* The discretization (Table 1 columns). */
typedef struct {
  int ncell[3];             /* cells per dimension, >= 3; periodic nodes = cells */
  int64_t n_particles;      /* N_p >= 1 */
  double dt;                /* > 0 */
  int n_avg;                /* N_avg >= 1 (eq. avg_outcome) */
  double cg_tol;            /* stop when ||r||_2 <= cg_tol ||rhs||_2 */
  int cg_max_iter;          /* >= 1 */
  int poisson_op;           /* enum pic_poisson_op */
} pic_discretization;

/* Field discretization (Sec. 4.2), both written as L phi = b over the cell
 * volume: the periodic 7-point finite-difference Laplacian with a pointwise
 * right-hand side, or trilinear (Q1) finite elements: minus the 27-point
 * stiffness, the particle charge through the cloud-in-cell weights (exact for
 * point charges) and the manufactured terms through the consistent mass
 * matrix applied to their nodal values.  The Q1 form uses the global-memory
 * solver. */
enum pic_poisson_op {
  PIC_OP_FD7 = 0,
  PIC_OP_Q1 = 1
};

typedef struct pic_ctx pic_ctx;

/* Bytes of device workspace one simulation needs (host out-pointer).
 * Returns PIC_EINVAL for an invalid or unsupported problem. */
int pic_workspace_size(const pic_problem* prob, const pic_discretization* disc,
                       int precision, int64_t* bytes);

/*
 * Create a simulation and enqueue its initial state on `hip_stream`:
 * the six uniforms xi of each particle (Sec. 3.2) from Philox4x64-10 keyed by
 * (seed, replicate), x^0 = x^M(xi, 0) and v^0 = v^M(xi, 0) by inverse-CDF root
 * solves (eq. mms_sol), the stable cell sort, the charge deposit, the Poisson
 * solve (eq. poisson_mms) from phi = 0 and the nodal field E = -grad phi.
 * `workspace` (device, >= pic_workspace_size bytes) is owned by the caller.
 * On success *out receives a host-side context to be released with
 * pic_destroy().  Returns PIC_WARN_NAVG when N_avg P_coll,max >= 0.5
 * (eq. navg_ineq), which is a warning only.
 */
int pic_init_manufactured(pic_ctx** out, const pic_problem* prob,
                          const pic_discretization* disc, uint64_t seed,
                          uint32_t replicate, int precision, void* workspace,
                          int64_t workspace_bytes, void* hip_stream);

/*
 * Enqueue n_steps time steps of eq. velocity_verlet: collision call A at t^n
 * (Algorithm 1 run N_avg times and averaged, eq. avg_outcome, minus the
 * analytic source eq. vel_change_3), half kick, drift with the manufactured
 * term, stable cell sort, deposit, Poisson CG (warm-started), gradient,
 * collision call B at t^{n+1/2} on the new cells, half kick.
 * Asynchronous; returns PIC_ESTATE if the context is not initialised.
 */
int pic_step(pic_ctx* ctx, int n_steps);

/*
 * Run one collision call on the current state without applying it: for every
 * particle, in the current (cell-sorted) order, dv_avg = <dv_p> (eq.
 * avg_outcome) and dv_src = <dv_p^M> (eq. vel_change_3 / eq. vel_change_1c with
 * the particle's own velocity and its cell's count).  `call` is 0 (the first
 * half kick of a step) or 1 (the second); `t` is the time at which the
 * manufactured velocity distribution enters the source.  The random stream is
 * the one pic_step() would use at the current step index.
 * dv_avg, dv_src: device, 3 * n_particles doubles each, component-major
 * (x block, then y, then z).  pairlog: device, pairlog_cap records of 7
 * int64 (cell, call, outcome k, pair m, p, q, accepted), in no particular
 * order, or NULL; *pairlog_n (host, may be NULL) receives the number of
 * candidate pairs (which may exceed pairlog_cap; the excess is not written).
 * Synchronises the context stream.  Returns PIC_WARN_GMAX (outputs valid)
 * once any candidate pair since initialisation had g > g_max.
 */
int pic_collide(pic_ctx* ctx, int call, double t, double* dv_avg, double* dv_src,
                int64_t* pairlog, int64_t pairlog_cap, int64_t* pairlog_n);

/* Error norms at the current time t = step * dt (Sec. 4.3): l2 and linf of
 * x, y, z (minimum image), u, v, w over all particles and of phi over the
 * nodes.  Synchronises; returns PIC_ENOCONV / PIC_EHIP for an earlier
 * asynchronous failure, PIC_ENONFINITE for a non-finite norm or particle
 * state, and the warning PIC_WARN_GMAX (norms valid) once any candidate pair
 * since initialisation had g > g_max.  The partial sums live in the
 * context's workspace; the reduction order depends only on the sizes. */
typedef struct {
  double t;
  double l2[7];             /* x, y, z, u, v, w, phi */
  double linf[7];
} pic_error_norms;
int pic_errors(pic_ctx* ctx, pic_error_norms* out);

/* pic_errors for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and result, bit for bit, with the partial sums and results in
 * a static array of the library (131,200 bytes per GPU, held until the process
 * ends) instead of the context's workspace.  The array's address on the
 * context's GPU is looked up once, on the first call there.  Calls no
 * allocating routine.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (other
 * threads, other contexts on concurrent streams) race and must be serialised
 * by the caller.  Returns PIC_EINVAL if the partial sums would not fit (they
 * always do: at most 1024 workgroups per reduction); otherwise as pic_errors. */
int pic_errors_noalloc(pic_ctx* ctx, pic_error_norms* out);

/*
 * Refinement ensembles (the paper's refinement studies with independent
 * replicates, Sec. 4.3): `members` simulations of one problem and
 * discretization that differ only in the replicate, first_replicate + 0 ..
 * members - 1, run together: every stage of a step is one launch for all
 * members (members along the grid's z dimension), so small meshes are not
 * bound by launch latency.  Member m is bit for bit the simulation
 * pic_init_manufactured would create with replicate first_replicate + m.
 * The workspace (device, pic_ensemble_workspace_size bytes, 256-byte
 * aligned, caller-owned) holds each member's state in its own slice.  Steps
 * are enqueued with pic_step(); pic_stats() sums the collision counters over
 * the members and reports member 0's solver.  The calls that serve one
 * simulation (pic_errors, pic_errors_noalloc, pic_collide, pic_set_state, the
 * angle log and checkpoints) return PIC_EINVAL on an ensemble context.
 */
int pic_ensemble_workspace_size(const pic_problem* prob, const pic_discretization* disc,
                                int precision, int members, int64_t* bytes);
int pic_ensemble_init(pic_ctx** out, const pic_problem* prob, const pic_discretization* disc,
                      uint64_t seed, uint32_t first_replicate, int members, int precision,
                      void* workspace, int64_t workspace_bytes, void* hip_stream);
/* Sec. 4.3 norms of every member at the current time: out (host) holds
 * `members` entries.  Synchronises; status as pic_errors. */
int pic_ensemble_errors(pic_ctx* ctx, pic_error_norms* out);
/* pic_get_state for member `member` (0 .. members - 1). */
int pic_ensemble_get_state(pic_ctx* ctx, int member, int item, void* host_dst, int64_t bytes);

/* Captured steps.  With enable != 0, pic_step(n) for n >= 4 records the
 * inner part of two time steps (sort, field solve, the particle pass that
 * finishes one step and starts the next) as a HIP graph once per
 * double-buffer parity, on a private stream, and replays it on the context's
 * stream, two steps per launch; the kernels then read the step index from a
 * counter in the workspace.  The results are bit for bit those of ordinary
 * stepping.  The Poisson solver's workgroups are co-resident by the creation
 * time occupancy check, so inside a graph it is launched ordinarily.  Steps
 * with stage timing switched on run without graphs; the angle log and
 * checkpoint loads drop the recorded graphs.  Returns PIC_EINVAL when the
 * context does not use the fused step (PIC_UNFUSED, the collision-heavy FP64
 * mode). */
int pic_use_graphs(pic_ctx* ctx, int enable);

/* Scattering-angle recovery (eq. angle_recovery and the empirical-CDF errors
 * defined after it).  While a log is enabled, every accepted collision of
 * pic_step and pic_collide appends chi = acos(g'_z / g) and
 * eps = atan2(g'_y, g'_x) in [0, 2 pi) (from the post-collision relative
 * velocity g' and the pre-collision speed g) to a caller-owned device buffer
 * of pic_angle_buffer_bytes(capacity) bytes, 256-byte aligned, which also
 * holds the metric's sort scratch.  The record order depends on scheduling;
 * the set of records and the metric do not.  pic_angle_log resets the count;
 * a zero capacity switches recording off.  Enqueued on the context stream. */
int64_t pic_angle_buffer_bytes(int64_t capacity);
int pic_angle_log(pic_ctx* ctx, void* device_buffer, int64_t capacity);
/* out = {eps_2 chi, eps_inf chi, eps_2 eps, eps_inf eps}: root mean square and
 * maximum over the N records of e_r = F(alpha_r) - F^M(alpha_r), F the
 * empirical CDF with theta(0) = 1 and F^M the isotropic analytic CDF
 * ((1 - cos chi) / 2, eps / (2 pi)).  *n_records = N.  Synchronises;
 * PIC_ESPACE (and no metric) when more collisions occurred than the log holds,
 * PIC_EINVAL when no log is enabled. */
int pic_angle_errors(pic_ctx* ctx, double out[4], int64_t* n_records);

/* Checkpoint and resume: the whole evolving state (particles in their current
 * cell-sorted order, cells, tile tables, charge, potential, field, counters,
 * step) to and from host memory.  A context created with the same problem,
 * discretization, seed, replicate and precision and loaded from a checkpoint
 * continues bit for bit as the saved one would.  Save and load synchronise;
 * load returns PIC_EINVAL for a checkpoint of another problem. */
int pic_checkpoint_bytes(pic_ctx* ctx, int64_t* bytes);
int pic_checkpoint_save(pic_ctx* ctx, void* host_dst, int64_t bytes);
int pic_checkpoint_load(pic_ctx* ctx, const void* host_src, int64_t bytes);

/* Counters of the last completed work (synchronises). */
typedef struct {
  int64_t step;             /* completed time steps */
  int cg_iters;             /* iterations of the last Poisson solve */
  double cg_relres;         /* its final relative residual */
  int64_t n_accepted;       /* accepted collisions since initialisation */
  int64_t n_gmax;           /* candidate pairs with g > g_max */
  int cg_blocks;            /* workgroups of the Poisson solver */
  int cg_brick[3];          /* nodes per brick of the on-chip solver; 0 0 0 = global-memory solver */
  int cg_members_per_launch; /* ensembles: members whose solvers share one launch (all of
                                them when they fit on the GPU together, else 1) */
} pic_stats_t;
int pic_stats(pic_ctx* ctx, pic_stats_t* out);

/* Copy part of the state to host memory (synchronises).  Particle arrays are
 * in the current cell-sorted order. bytes must equal the size stated here. */
enum pic_state_item {
  PIC_STATE_X = 0,          /* 3 * n_particles doubles, component-major */
  PIC_STATE_V = 1,          /* 3 * n_particles doubles */
  PIC_STATE_ID = 2,         /* n_particles int64: particle identity */
  PIC_STATE_CELL_START = 3, /* (ncells + 1) int64 */
  PIC_STATE_RHO = 4,        /* ncells doubles (nodal charge density) */
  PIC_STATE_PHI = 5,        /* ncells doubles */
  PIC_STATE_E = 6           /* 3 * ncells doubles */
};
int pic_get_state(pic_ctx* ctx, int item, void* host_dst, int64_t bytes);

/* Replace the particle positions (PIC_STATE_X) or velocities (PIC_STATE_V):
 * host_src holds 3 * n_particles doubles, component-major, in the current
 * cell-sorted order (the order pic_get_state returns); bytes must equal that
 * size.  New positions are wrapped into the periodic box (a non-finite
 * coordinate becomes 0 and the next synchronising call reports
 * PIC_ENONFINITE), the particles are stable-sorted by their new cells from the
 * current order, and the charge is deposited and the Poisson equation
 * (eq. poisson_mms) solved at the current time, as at initialisation.
 * Velocities are taken as given (rounded to FP32 in the mixed form); a
 * non-finite one makes pic_errors return PIC_ENONFINITE.  The manufactured
 * solution and the particle identities are unchanged.  Synchronises;
 * PIC_EINVAL for other items or a size mismatch. */
int pic_set_state(pic_ctx* ctx, int item, const void* host_src, int64_t bytes);

/* Per-stage GPU time, measured with HIP events recorded on the context stream
 * around each stage's kernels while timing is enabled. */
enum pic_stage {
  PIC_STAGE_COLLIDE = 0,    /* Algorithm 1 x N_avg (both calls) */
  PIC_STAGE_KICK = 1,       /* gather + half kick (both halves) */
  PIC_STAGE_DRIFT = 2,      /* drift + new cell keys and counts */
  PIC_STAGE_SORT = 3,       /* scan, scatter, stable in-cell order, reorder */
  PIC_STAGE_DEPOSIT = 4,    /* cell moments, node charge, Poisson right-hand side */
  PIC_STAGE_CG = 5,         /* Poisson conjugate gradients */
  PIC_STAGE_GRADIENT = 6,   /* E = -grad phi */
  PIC_STAGE_PARTICLE = 7,   /* the fused particle kernel of the mixed form */
  PIC_STAGE_COUNT = 8
};
/* enable != 0 starts (and resets) the accumulation for every stage; 0 stops it. */
int pic_timing_enable(pic_ctx* ctx, int enable);
/* Starts (and resets) the accumulation for the stages whose bit (1u << stage)
 * is set in mask, so that a measurement can time one stage without the event
 * records of the others; mask 0 stops it.  Bits at or above PIC_STAGE_COUNT
 * are ignored.  Synchronises the context stream. */
int pic_timing_stages(pic_ctx* ctx, uint32_t mask);
/* ms (host, PIC_STAGE_COUNT doubles): summed milliseconds per stage;
 * launches (host, PIC_STAGE_COUNT int64): number of timed stage instances.
 * Synchronises the context stream. */
int pic_timing_read(pic_ctx* ctx, double* ms, int64_t* launches);

/* Release the host context (not the caller's workspace). */
void pic_destroy(pic_ctx* ctx);

/* Text of the last error of ctx (or of the last failed creation when ctx is
 * NULL).  Valid until the next call on the same context. */
const char* pic_last_error(const pic_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
