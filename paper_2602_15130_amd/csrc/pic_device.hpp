// Device-side building blocks of the PIC/DSMC manufactured-solution step:
// simulation constants, the counter-based random stream, and the manufactured
// solution of Sec. 3 / Sec. 5.2 (FP64, with FP32 variants for the mixed form).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr double kPi = 3.14159265358979323846;
constexpr float kPiF = 3.14159265358979323846f;

// Everything a kernel needs to know about the problem, derived once on the host.
// Unsigned division by a divisor d >= 1 fixed for the whole run, as one
// multiply-high and a shift (Granlund and Montgomery, PLDI 1994, the
// round-up multiplier): with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1, n / d = (mulhi(n, m) + n) >> s for
// every 32-bit n when the sum is formed in 64 bits.
struct DivMagic {
  uint32_t m, s;
};

__host__ __device__ inline DivMagic div_magic(uint32_t d) {
  uint32_t s = 0;
  while ((uint64_t(1) << s) < d) ++s;
  const uint64_t m = (((uint64_t(1) << s) - d) << 32) / d + 1;
  return {(uint32_t)m, s};
}

__host__ __device__ inline uint32_t div_by(DivMagic q, uint32_t n) {
  const uint64_t hi = ((uint64_t)n * q.m) >> 32;
  return (uint32_t)((hi + n) >> q.s);
}

struct SimConst {
  int family;          // 0 paper (Sec. 5.2), 1 configuration family
  int sigma_model;     // 0 polynomial (eq. sigma_ms), 1 variable hard sphere
  int n_sigma;
  int collisions, isolate, navg;
  int nc[3];
  int nn;              // nodes = cells
  DivMagic div_x, div_xy;  // division by nc[0] and by nc[0] nc[1]
  int64_t np;
  uint64_t seed;
  uint32_t rep;
  double L[3], h[3], inv_h[3], ih2[3];
  double qm;           // q/m, or 0 when the field does not act on the particles
  double p2f;          // 1 when the particles feed the Poisson source, else 0
  double q, eps0, T, vbar, phibar, rho_amp;
  double sigma_n[3];
  double sg_coef, sg_pow;  // VHS: sigma g = sg_coef g^sg_pow
  double sigma_ref, g_ref, omega, g_max;
  double sgmax;        // (sigma g)_max over [0, g_max]
  double sr[3];        // sigma_n vbar^(2n) / (sigma g)_max: the accept ratio in units of vbar
  double inv_vbar;     // 1 / vbar
  double pmax;         // Algorithm 1: (sigma g)_max w dt / dV
  double w, dV, dt;
  double rho_scale;    // q w / dV
  double src_half;     // w dt / (2 dV)
  double nphys;
  int poisson_op;      // field discretization: 0 7-point differences, 1 trilinear elements
  int chi_model;       // polar-angle model: 0 isotropic, 1 manufactured anisotropy, 2 VSS
  double chi_alpha;    // VSS exponent
  int coding_error;    // Sec. 5.4.1 Error 1 / Error 2 (verification studies), 0 none
  // completed steps, kept on the device for captured steps (shared by all
  // ensemble members; null when unused)
  const long long* stepc;
  double* anglog;      // scattering-angle records (chi, eps) of accepted collisions, or null
  int64_t angcap;      // records that fit
  // Ensembles: the members of one context share every size and differ only in
  // the replicate.  Member m = member0 + blockIdx.z uses replicate rep + m and
  // owns the workspace bytes starting m * mstride after member 0's.
  int member0;
  int64_t mstride;
};

// The ensemble member a workgroup works for, and a member-0 workspace pointer
// moved to that member's copy (null stays null).
__device__ inline int member_of(const SimConst& K) { return K.member0 + (int)blockIdx.z; }
template <class T>
__device__ inline T* mem(const SimConst& K, T* p) {
  return p ? (T*)((char*)p + (int64_t)member_of(K) * K.mstride) : p;
}
// The same for kernels that receive only the stride (members in blockIdx.z).
template <class T>
__device__ inline T* mem_z(int64_t mstride, T* p) {
  return p ? (T*)((char*)p + (int64_t)blockIdx.z * mstride) : p;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11).  Counter layout of the random stream:
//   c0 entity (particle id or cell), c1 step, c2 tag<<56 | call<<48 | outcome,
//   c3 block; key = (seed, replicate; an ensemble member adds its index to
//   the replicate).  The N_pairs uniforms of four
//   consecutive outcomes share one block: tag NPAIRS, outcome field k / 4,
//   word k mod 4.
// ---------------------------------------------------------------------------
enum : uint64_t { kTagInit = 1, kTagColl = 2, kTagRedraw = 3, kTagNpairs = 4 };

struct U64x4 {
  uint64_t w[4];
};

__host__ __device__ inline uint64_t mul_hi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline U64x4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1) {
  const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    uint64_t h0 = mul_hi64(m0, c0), l0 = m0 * c0;
    uint64_t h1 = mul_hi64(m1, c2), l1 = m1 * c2;
    uint64_t a = h1 ^ c1 ^ k0, b = h0 ^ c3 ^ k1;
    c0 = a; c1 = l1; c2 = b; c3 = l0;
    k0 += 0x9E3779B97F4A7C15ull;
    k1 += 0xBB67AE8584CAA73Bull;
  }
  return U64x4{{c0, c1, c2, c3}};
}

__device__ inline U64x4 stream_block(const SimConst& K, uint64_t entity, uint64_t step,
                                     uint64_t tag, uint64_t call, uint64_t k, uint64_t blk) {
  return philox(entity, step, (tag << 56) | (call << 48) | k, blk, K.seed,
                (uint64_t)K.rep + (uint64_t)member_of(K));
}

// [0,1) with 53 bits, (0,1) with 52 bits + 1/2, floor(U n) exactly.
__device__ inline double unif(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
__device__ inline double unif_open(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1.0p-52; }
__device__ inline float unif32(uint64_t w) { return (float)(uint32_t)(w >> 40) * 0x1.0p-24f; }
__device__ inline int index_below(uint64_t w, int n) {
  return (int)__umul64hi(w & ~0x7FFull, (uint64_t)n);
}

// ---------------------------------------------------------------------------
// Safeguarded Newton for a monotone CDF on [lo, hi].
// ---------------------------------------------------------------------------
template <class Cdf>
__device__ double invert_cdf(const Cdf& F, double target, double lo, double hi, double x) {
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double dens;
    double res = F(x, dens) - target;
    if (res == 0.0) break;
    if (res > 0.0) hi = x; else lo = x;
    double nx = x - res / dens;
    if (!(dens > 0.0) || !(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
    if (nx == lo || nx == hi) { x = nx; break; }
    double step = fabs(nx - x);
    x = nx;
    if (step <= 4.440892098500626e-16 * fabs(x)) break;
  }
  return x;
}

// ---------------------------------------------------------------------------
// Manufactured solution.
// ---------------------------------------------------------------------------
// Sec. 5.2 position densities per unit length and their CDFs from 0.
struct PaperPosCdf {
  int d;
  double L, e;  // e = exp(t / T)
  __device__ double operator()(double x, double& dens) const {
    double s = x / L;
    if (d == 0) {
      dens = (1.0 + 0.2 * e * sinpi(2.0 * s)) / L;
      return s + 0.2 * e * (1.0 - cospi(2.0 * s)) / (2.0 * kPi);
    }
    if (d == 1) {
      double c = 0.15 * e;
      dens = (1.0 + 0.2 * sinpi(2.0 * (s - c))) / L;
      return s + (cospi(2.0 * c) - cospi(2.0 * (s - c))) / (10.0 * kPi);
    }
    double c = e / 15.0;
    dens = (1.0 - (e / 6.0) * sinpi(2.0 * (s + c))) / L;
    return s - (e / (12.0 * kPi)) * (cospi(2.0 * c) - cospi(2.0 * (s + c)));
  }
};

// dF/dt at fixed x for the Sec. 5.2 position CDFs.
__device__ inline double paper_dFdt(int d, double x, double L, double T, double e) {
  double s = x / L;
  if (d == 0) return (0.2 * e / T) * (1.0 - cospi(2.0 * s)) / (2.0 * kPi);
  if (d == 1) {
    double c = 0.15 * e, cdot = c / T;
    return -(cdot / 5.0) * (sinpi(2.0 * c) + sinpi(2.0 * (s - c)));
  }
  double c = e / 15.0, cdot = c / T;
  double br = cospi(2.0 * c) - cospi(2.0 * (s + c));
  double dbr = 2.0 * kPi * cdot * (sinpi(2.0 * (s + c)) - sinpi(2.0 * c));
  return -(e / (12.0 * kPi * T)) * br - (e / (12.0 * kPi)) * dbr;
}

// Configuration family: CDF of z given (x, y), a = A sin(2 pi x/L) sin(2 pi y/L).
struct CfgZCdf {
  double L, a;
  __device__ double operator()(double z, double& dens) const {
    double s = z / L;
    dens = (1.0 + a * sinpi(2.0 * s)) / L;
    return s + a * (1.0 - cospi(2.0 * s)) / (2.0 * kPi);
  }
};

// Paper velocity CDF in units of vhat: G(a) = (1 + erf a)/2 - a e^{-a^2}/sqrt(pi).
struct PaperGCdf {
  __device__ double operator()(double a, double& dens) const {
    double ea = exp(-a * a);
    dens = 1.1283791670955126 * a * a * ea;  // 2/sqrt(pi)
    return 0.5 + 0.5 * erf(a) - 0.5641895835477563 * a * ea;
  }
};

struct NormalCdf {
  __device__ double operator()(double z, double& dens) const {
    dens = 0.3989422804014327 * exp(-0.5 * z * z);
    return 0.5 * erfc(-0.7071067811865476 * z);
  }
};

__device__ inline void init_uniforms(const SimConst& K, int64_t id, double xi[6]) {
  U64x4 a = stream_block(K, (uint64_t)id, 0, kTagInit, 0, 0, 0);
  U64x4 b = stream_block(K, (uint64_t)id, 0, kTagInit, 0, 0, 1);
  for (int d = 0; d < 3; ++d) {
    xi[d] = unif_open(a.w[d]);
    xi[3 + d] = unif_open(b.w[d]);
  }
}

__device__ inline void velocity_uniforms(const SimConst& K, int64_t id, double xv[3]) {
  U64x4 b = stream_block(K, (uint64_t)id, 0, kTagInit, 0, 0, 1);
  for (int d = 0; d < 3; ++d) xv[d] = unif_open(b.w[d]);
}

__device__ inline void position_uniforms(const SimConst& K, int64_t id, double xp[3]) {
  U64x4 a = stream_block(K, (uint64_t)id, 0, kTagInit, 0, 0, 0);
  for (int d = 0; d < 3; ++d) xp[d] = unif_open(a.w[d]);
}

__device__ inline void vhat_of_t(const SimConst& K, double t, double vh[3], double vd[3]) {
  if (K.family == 1) {
    vh[0] = vh[1] = vh[2] = K.vbar;
    vd[0] = vd[1] = vd[2] = 0.0;
    return;
  }
  double u = t / K.T;
  vh[0] = (1.0 + 0.2 * sinpi(0.5 * u)) * K.vbar;
  vh[1] = (1.0 + 0.2 * cospi(u)) * K.vbar;
  vh[2] = (1.0 + 0.2 * sinpi(1.5 * u)) * K.vbar;
  vd[0] = 0.2 * (0.5 * kPi / K.T) * cospi(0.5 * u) * K.vbar;
  vd[1] = -0.2 * (kPi / K.T) * sinpi(u) * K.vbar;
  vd[2] = 0.2 * (1.5 * kPi / K.T) * cospi(1.5 * u) * K.vbar;
}

// Standard normal quantile.  The root is taken on the lower tail, Phi(-z) =
// min(xi, 1 - xi) (1 - xi is exact for xi >= 1/2), which keeps the residual
// well conditioned in both tails; starting guess Abramowitz & Stegun 26.2.23
// (|error| < 4.5e-4), then Newton steps on 0.5 erfc(-y / sqrt 2) in FP64.
__device__ inline double normal_quantile(double xi) {
  const double pp = xi < 0.5 ? xi : 1.0 - xi;
  const double t = sqrt(-2.0 * log(pp));
  double y = -(t - (2.515517 + t * (0.802853 + t * 0.010328)) /
                       (1.0 + t * (1.432788 + t * (0.189269 + t * 0.001308))));
#pragma unroll 1
  for (int it = 0; it < 4; ++it) {
    double f = 0.5 * erfc(-0.7071067811865476 * y) - pp;
    double dens = 0.3989422804014327 * exp(-0.5 * y * y);
    double dy = f / dens;
    y -= dy;
    if (fabs(dy) <= 1e-16 * fabs(y)) break;
  }
  return xi < 0.5 ? y : -y;
}

// Paper family: a = G^{-1}(xi), time independent (v^M = vhat(t) a).  The
// density of eq. fv is even, so G^{-1}(xi) = -G^{-1}(1 - xi): solve on the
// lower half.
__device__ __noinline__ double paper_a(double xi) {
  const double pp = xi < 0.5 ? xi : 1.0 - xi;
  double a0 = cbrt(2.6586807763582730 * (pp - 0.5));  // 1.5 sqrt(pi)
  double a = invert_cdf(PaperGCdf{}, pp, -30.0, 0.0, a0);
  return xi < 0.5 ? a : -a;
}

// Velocity shape factor per component: v^M(t) = vhat(t) * shape.
__device__ inline void velocity_shape(const SimConst& K, const double xv[3], double a[3]) {
  for (int d = 0; d < 3; ++d) a[d] = (K.family == 1) ? normal_quantile(xv[d]) : paper_a(xv[d]);
}

__device__ inline void manufactured_velocity(const SimConst& K, const double a[3], double t,
                                             double v[3], double vdot[3]) {
  double vh[3], vd[3];
  vhat_of_t(K, t, vh, vd);
  for (int d = 0; d < 3; ++d) {
    v[d] = vh[d] * a[d];
    vdot[d] = vd[d] * a[d];
  }
}

__device__ inline void paper_position(const SimConst& K, const double xp[3], double t,
                                             const double* guess, double x[3]) {
  double e = exp(t / K.T);
  for (int d = 0; d < 3; ++d) {
    PaperPosCdf F{d, K.L[d], e};
    x[d] = invert_cdf(F, xp[d], 0.0, K.L[d], guess ? guess[d] : K.L[d] * xp[d]);
  }
}

__device__ inline void cfg_position(const SimConst& K, const double xp[3], double x[3]) {
  x[0] = K.L[0] * xp[0];
  x[1] = K.L[1] * xp[1];
  CfgZCdf F{K.L[2], K.rho_amp * sinpi(2.0 * x[0] / K.L[0]) * sinpi(2.0 * x[1] / K.L[1])};
  x[2] = invert_cdf(F, xp[2], 0.0, K.L[2], K.L[2] * xp[2]);
}

// eq. mms_sol for the positions; `guess` speeds up the paper-family roots.
__device__ inline void manufactured_position(const SimConst& K, const double xp[3], double t,
                                             const double* guess, double x[3]) {
  if (K.family == 1) cfg_position(K, xp, x);
  else paper_position(K, xp, t, guess, x);
}

// xdot^M = -(dF/dt)/f at x^M (Sec. 3.2).
__device__ inline void manufactured_xdot(const SimConst& K, const double xm[3], double t,
                                         double xd[3]) {
  if (K.family == 1) {
    xd[0] = xd[1] = xd[2] = 0.0;
    return;
  }
  double e = exp(t / K.T);
  for (int d = 0; d < 3; ++d) {
    PaperPosCdf F{d, K.L[d], e};
    double dens;
    (void)F(xm[d], dens);
    xd[d] = -paper_dFdt(d, xm[d], K.L[d], K.T, e) / dens;
  }
}

// Number density f_x (eq. fx), integrating to N over the box.
__device__ inline double number_density(const SimConst& K, const double x[3], double t) {
  if (K.family == 1) {
    double s = sinpi(2.0 * x[0] / K.L[0]) * sinpi(2.0 * x[1] / K.L[1]) * sinpi(2.0 * x[2] / K.L[2]);
    return K.nphys / (K.L[0] * K.L[1] * K.L[2]) * (1.0 + K.rho_amp * s);
  }
  double e = exp(t / K.T), r = K.nphys;
  for (int d = 0; d < 3; ++d) {
    PaperPosCdf F{d, K.L[d], e};
    double dens;
    (void)F(x[d], dens);
    r *= dens;
  }
  return r;
}

// phi^M = phibar e^{t/2T} prod sin(2 pi (x_d/L_d - c_d)), c = (1/7, 1/5, 1/3).
__device__ inline void phiM_factors(const SimConst& K, const double x[3], double s[3],
                                    double c[3]) {
  const double shift[3] = {1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0};
  for (int d = 0; d < 3; ++d) {
    double arg = 2.0 * (x[d] / K.L[d] - shift[d]);
    s[d] = sinpi(arg);
    c[d] = cospi(arg);
  }
}

__device__ inline double phiM(const SimConst& K, const double x[3], double t) {
  double s[3], c[3];
  phiM_factors(K, x, s, c);
  return K.phibar * exp(0.5 * t / K.T) * s[0] * s[1] * s[2];
}

__device__ inline double lap_phiM(const SimConst& K, const double x[3], double t) {
  double k2 = 0.0;
  for (int d = 0; d < 3; ++d) k2 += (2.0 * kPi / K.L[d]) * (2.0 * kPi / K.L[d]);
  return -k2 * phiM(K, x, t);
}

__device__ inline void EM(const SimConst& K, const double x[3], double t, double E[3]) {
  double s[3], c[3];
  phiM_factors(K, x, s, c);
  double a = K.phibar * exp(0.5 * t / K.T);
  E[0] = -a * (2.0 * kPi / K.L[0]) * c[0] * s[1] * s[2];
  E[1] = -a * (2.0 * kPi / K.L[1]) * s[0] * c[1] * s[2];
  E[2] = -a * (2.0 * kPi / K.L[2]) * s[0] * s[1] * c[2];
}

// Cross-section models known at compile time in the fused kernels.
enum { kSigHS = 0, kSigMaxwell = 1, kSigPoly = 2 };

template <int SIG>
__device__ inline double sigma_g_t(const SimConst& K, double g) {
  if (SIG == kSigHS) return K.sg_coef * g;          // omega = 1/2: sigma constant
  if (SIG == kSigMaxwell) return K.sg_coef;         // omega = 1: sigma g constant
  double g2 = g * g, r = K.sigma_n[0];
  if (K.n_sigma > 1) r += K.sigma_n[1] * g2;
  if (K.n_sigma > 2) r += K.sigma_n[2] * (g2 * g2);
  return r;
}

// sigma(g) g.
__device__ inline double sigma_g(const SimConst& K, double g) {
  if (K.sigma_model == 1) return K.sg_coef * pow(g, K.sg_pow);
  double g2 = g * g, r = K.sigma_n[0];
  if (K.n_sigma > 1) r += K.sigma_n[1] * g2;
  if (K.n_sigma > 2) r += K.sigma_n[2] * (g2 * g2);
  return r;
}

// Hard sphere, Gaussian partners: int g (v_q - v_p) f_v = -s^2 K(l) v_p/|v_p|.
// K(l) = [(l^4 + 2l^2 - 1) erf(l/sqrt2) + 2l(l^2+1) phi_N(l)] / l^2, summed as a
// power series below l = 0.5 where the closed form cancels.
__device__ inline double hs_kernel(double l) {
  if (l < 0.5) {
    // erf(l/sqrt2) = sqrt(2/pi) sum a_n l^(2n+1); 2 l phi_N(l) = sqrt(2/pi) sum b_n l^(2n+1)
    // with b_n = (-1/2)^n / n!, a_n = b_n / (2n+1); K = sqrt(2/pi) sum_j c_j l^(2j-1),
    // c_j = a_{j-2} + 2 a_{j-1} - a_j + b_{j-1} + b_j.
    double bm2 = 0.0, am2 = 0.0;         // n = j-2
    double bm1 = 1.0, am1 = 1.0;         // n = j-1 (j = 1)
    double sum = 0.0, l2 = l * l, lp = l;  // l^(2j-1)
    for (int j = 1; j < 30; ++j) {
      double bj = bm1 * (-0.5) / j, aj = bj / (2.0 * j + 1.0);
      sum += (am2 + 2.0 * am1 - aj + bm1 + bj) * lp;
      am2 = am1; bm2 = bm1; am1 = aj; bm1 = bj;
      lp *= l2;
    }
    (void)bm2;
    return 0.7978845608028654 * sum;
  }
  double l2 = l * l;
  double phin = 0.3989422804014327 * exp(-0.5 * l2);
  return ((l2 * l2 + 2.0 * l2 - 1.0) * erf(0.7071067811865476 * l) + 2.0 * l * (l2 + 1.0) * phin) / l2;
}

__device__ inline void poly_source_inl(const SimConst& K, const double u[3], double t,
                                       double out[3]);
__device__ __noinline__ void poly_source(const SimConst& K, const double u[3], double t,
                                         double out[3]);

// eq. vel_change_1c integral (no prefactor) at particle velocity u and time t.
__device__ inline void source_integral(const SimConst& K, const double u[3], double t,
                                       double out[3]) {
  if (K.sigma_model == 1) {
    if (K.omega == 1.0) {
      double c = K.sigma_ref * K.g_ref;
      for (int i = 0; i < 3; ++i) out[i] = -c * u[i];
      return;
    }
    double sp = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (sp == 0.0) {
      out[0] = out[1] = out[2] = 0.0;
      return;
    }
    double s = K.vbar;
    double kk = hs_kernel(sp / s);
    for (int i = 0; i < 3; ++i) out[i] = -K.sigma_ref * s * s * kk * u[i] / sp;
    return;
  }
  poly_source(K, u, t, out);
}

// Polynomial cross section (eq. sigma_ms): sum_n sigma_n f_n (eq. vel_change_3).
__device__ inline void poly_source_inl(const SimConst& K, const double u[3], double t,
                                       double out[3]) {
  double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double f[3][3];
  if (K.family == 0) {
    double vh[3], vd[3];
    vhat_of_t(K, t, vh, vd);
    double h2[3] = {vh[0] * vh[0], vh[1] * vh[1], vh[2] * vh[2]};
    double H = h2[0] + h2[1] + h2[2];
    double mix = h2[0] * u[0] * u[0] + h2[1] * u[1] * u[1] + h2[2] * u[2] * u[2];
    for (int i = 0; i < 3; ++i) {
      double others = h2[(i + 1) % 3] * h2[(i + 2) % 3];
      f[0][i] = -u[i];
      f[1][i] = -0.5 * (3.0 * H + 6.0 * h2[i] + 2.0 * u2) * u[i];
      f[2][i] = -0.25 * (15.0 * H * H + 36.0 * h2[i] * h2[i] + 24.0 * u2 * h2[i] + 4.0 * u2 * u2 +
                         24.0 * h2[i] * H + 12.0 * u2 * H + 24.0 * mix - 12.0 * others) * u[i];
    }
  } else {
    // symmetric product density with m2 = s^2, m4 = 3 s^4 per component
    double m2 = K.vbar * K.vbar, m4 = 3.0 * m2 * m2;
    for (int i = 0; i < 3; ++i) {
      int j = (i + 1) % 3, k = (i + 2) % 3;
      double ui2 = u[i] * u[i], uj2 = u[j] * u[j], uk2 = u[k] * u[k];
      double qj = m2 + uj2, qk = m2 + uk2;
      double s1 = qj + qk;
      double s2 = (m4 + 6.0 * uj2 * m2 + uj2 * uj2) + (m4 + 6.0 * uk2 * m2 + uk2 * uk2);
      f[0][i] = -u[i];
      f[1][i] = -u[i] * (3.0 * m2 + ui2 + s1);
      f[2][i] = -u[i] * (5.0 * m4 + 10.0 * ui2 * m2 + ui2 * ui2 + s2 + 2.0 * qj * qk +
                         2.0 * (3.0 * m2 + ui2) * s1);
    }
  }
  for (int i = 0; i < 3; ++i) {
    double r = 0.0;
    for (int n = 0; n < K.n_sigma; ++n) r += K.sigma_n[n] * f[n][i];
    out[i] = r;
  }
}

}  // namespace pic

namespace pic {
__device__ __noinline__ void poly_source(const SimConst& K, const double u[3], double t,
                                         double out[3]) {
  poly_source_inl(K, u, t, out);
}

// Source integral with the cross-section model fixed at compile time.
template <int SIG>
__device__ inline void source_integral_t(const SimConst& K, const double u[3], double t,
                                         double out[3]) {
  if (SIG == kSigMaxwell) {
    double c = K.sigma_ref * K.g_ref;
    for (int i = 0; i < 3; ++i) out[i] = -c * u[i];
  } else if (SIG == kSigHS) {
    double sp = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (sp == 0.0) {
      out[0] = out[1] = out[2] = 0.0;
      return;
    }
    double s = K.vbar;
    double kk = hs_kernel(sp / s);
    for (int i = 0; i < 3; ++i) out[i] = -K.sigma_ref * s * s * kk * u[i] / sp;
  } else {
    poly_source_inl(K, u, t, out);
  }
}
}  // namespace pic
