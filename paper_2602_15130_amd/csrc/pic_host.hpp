// Host-side derivation of the constants every kernel receives: the problem
// and discretization of include/pic.h turned into SimConst (and the FP32
// constants of one mixed-form pass, including the paper family's vhat(t)).  Host code only: no launches here, so
// host programs (the library and the test harness that runs the particle
// pass on the CPU) share one definition.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/pic.h"
#include "pic_mixed.hpp"

namespace pic {

inline double host_sigma_g(const SimConst& K, double g) {
  if (K.sigma_model == 1) return K.sg_coef * std::pow(g, K.sg_pow);
  double g2 = g * g, r = K.sigma_n[0];
  if (K.n_sigma > 1) r += K.sigma_n[1] * g2;
  if (K.n_sigma > 2) r += K.sigma_n[2] * (g2 * g2);
  return r;
}

inline SimConst derive(const pic_problem* p, const pic_discretization* d, uint64_t seed, uint32_t rep) {
  SimConst K;
  std::memset(&K, 0, sizeof(K));
  K.family = p->family;
  K.sigma_model = p->sigma_model;
  K.n_sigma = p->sigma_model == PIC_SIGMA_POLY ? p->n_sigma : 0;
  K.collisions = p->collisions;
  K.isolate = p->isolate;
  K.chi_model = p->chi_model;
  K.chi_alpha = p->chi_model == PIC_CHI_VSS ? p->chi_alpha : 1.0;
  K.coding_error = p->coding_error;
  K.navg = d->n_avg;
  K.np = d->n_particles;
  K.nn = d->ncell[0] * d->ncell[1] * d->ncell[2];
  K.div_x = div_magic((uint32_t)d->ncell[0]);
  K.div_xy = div_magic((uint32_t)(d->ncell[0] * d->ncell[1]));
  K.seed = seed;
  K.rep = rep;
  for (int k = 0; k < 3; ++k) {
    K.nc[k] = d->ncell[k];
    K.L[k] = p->L[k];
    K.h[k] = p->L[k] / d->ncell[k];
    K.inv_h[k] = (double)d->ncell[k] / p->L[k];
    K.ih2[k] = 1.0 / (K.h[k] * K.h[k]);
  }
  K.qm = p->field_to_particles ? p->q / p->m : 0.0;
  K.p2f = p->particles_to_field ? 1.0 : 0.0;
  K.q = p->q;
  K.eps0 = p->eps0;
  K.T = p->T;
  K.vbar = p->vbar;
  K.phibar = p->phibar;
  K.rho_amp = p->rho_amp;
  for (int k = 0; k < 3; ++k) K.sigma_n[k] = p->sigma_n[k];
  K.sigma_ref = p->sigma_ref;
  K.g_ref = p->g_ref;
  K.omega = p->omega;
  K.g_max = p->g_max;
  K.sg_coef = p->sigma_ref * std::pow(p->g_ref, 2.0 * p->omega - 1.0);
  K.sg_pow = 2.0 - 2.0 * p->omega;
  K.nphys = p->nphys;
  K.dt = d->dt;
  K.poisson_op = d->poisson_op;
  K.w = p->nphys / (double)d->n_particles;
  K.dV = (p->L[0] / d->ncell[0]) * (p->L[1] / d->ncell[1]) * (p->L[2] / d->ncell[2]);
  K.rho_scale = p->q * K.w / K.dV;
  K.src_half = K.w * K.dt / (2.0 * K.dV);
  // (sigma g)_max over [0, g_max] (Sec. 5.2)
  if (K.sigma_model == 1) {
    K.sgmax = host_sigma_g(K, p->g_max);  // nondecreasing in g for omega <= 1
  } else {
    double best = host_sigma_g(K, 0.0), e = host_sigma_g(K, p->g_max);
    if (e > best) best = e;
    if (K.n_sigma == 3 && K.sigma_n[2] != 0.0) {
      double G = -K.sigma_n[1] / (2.0 * K.sigma_n[2]);
      if (G > 0.0 && G < p->g_max * p->g_max) best = std::max(best, host_sigma_g(K, std::sqrt(G)));
    }
    K.sgmax = best;
  }
  K.pmax = K.sgmax * K.w * K.dt / K.dV;  // Algorithm 1
  K.inv_vbar = 1.0 / p->vbar;
  for (int n = 0; n < 3; ++n)
    K.sr[n] = K.sgmax > 0.0 ? K.sigma_n[n] * std::pow(p->vbar, 2.0 * n) / K.sgmax : 0.0;
  return K;
}

// vhat(t) and vhat'(t) of the paper's velocity distribution (Sec. 5.2), or
// vbar and 0 for the configuration family.  (Host and device: a captured step
// computes the constants of its pass on the device from the step counter.)
__host__ __device__ inline void host_vhat(const SimConst& K, double t, double vh[3], double vd[3]) {
  if (K.family == 1) {
    for (int d = 0; d < 3; ++d) {
      vh[d] = K.vbar;
      vd[d] = 0.0;
    }
    return;
  }
  const double u = t / K.T;
  vh[0] = (1.0 + 0.2 * sin(0.5 * kPi * u)) * K.vbar;
  vh[1] = (1.0 + 0.2 * cos(kPi * u)) * K.vbar;
  vh[2] = (1.0 + 0.2 * sin(1.5 * kPi * u)) * K.vbar;
  vd[0] = 0.2 * (0.5 * kPi / K.T) * cos(0.5 * kPi * u) * K.vbar;
  vd[1] = -0.2 * (kPi / K.T) * sin(kPi * u) * K.vbar;
  vd[2] = 0.2 * (1.5 * kPi / K.T) * cos(1.5 * kPi * u) * K.vbar;
}

// FP32 constants of one mixed-form pass with arguments a: call B and its kick
// at the end of step a.nb, call A and its kick and the drift of step a.na
// (collide-only: call A's source at time a.tB).
__host__ __device__ inline MixConst mix_const(const SimConst& K, const PartArgs& a) {
  const double dt = K.dt;
  const double tA = (double)a.na * dt, tB = ((double)a.nb + 1.0) * dt;  // the two kicks
  MixConst M{};
  M.dt = (float)dt;
  M.dtqm = (float)(dt * K.qm);
  for (int d = 0; d < 3; ++d) {
    M.inv_h[d] = (float)K.inv_h[d];
    M.inv_n[d] = (float)(1.0 / K.nc[d]);
    const double kd = 2.0 * kPi / K.L[d];
    M.emA[d] = (float)(K.phibar * exp(tA / (2.0 * K.T)) * kd);
    M.emB[d] = (float)(K.phibar * exp(tB / (2.0 * K.T)) * kd);
  }
  M.vbar = (float)K.vbar;
  M.src_w = (float)(K.w * K.dt / (2.0 * K.dV));
  M.sigma_ref = (float)K.sigma_ref;
  M.inv_vbar = (float)(1.0 / K.vbar);
  for (int n = 0; n < 3; ++n)
    M.pc[n] = (float)(K.sigma_n[n] * pow(K.vbar, 2.0 * n + 1.0));
  // kick B at t^{nb+1} (from t^{nb+1/2}), source at t^{nb+1/2}; kick A at t^{na}
  // (to t^{na+1/2}), source at t^{na}; drift at t^{na+1/2}
  const double thB = ((double)a.nb + 0.5) * dt, thA = ((double)a.na + 0.5) * dt;
  const double tsrcA = (a.mode & kCollideOnly) ? a.tB : tA;
  double vh[3], vd[3], vh2[3], vd2[3];
  host_vhat(K, thA, vh, vd);
  for (int d = 0; d < 3; ++d) M.vh_drift[d] = (float)vh[d];
  if (K.family == 0) {
    host_vhat(K, tB, vh, vd);
    host_vhat(K, thB, vh2, vd2);
    for (int d = 0; d < 3; ++d) M.hB[d] = (float)(K.isolate ? vh[d] - vh2[d] : 0.5 * dt * vd[d]);
    host_vhat(K, tA, vh, vd);
    host_vhat(K, thA, vh2, vd2);
    for (int d = 0; d < 3; ++d) M.hA[d] = (float)(K.isolate ? vh2[d] - vh[d] : 0.5 * dt * vd[d]);
  }
  host_vhat(K, thB, vh, vd);
  for (int d = 0; d < 3; ++d) M.h2B[d] = (float)((vh[d] / K.vbar) * (vh[d] / K.vbar));
  host_vhat(K, tsrcA, vh, vd);
  for (int d = 0; d < 3; ++d) M.h2A[d] = (float)((vh[d] / K.vbar) * (vh[d] / K.vbar));
  return M;
}

}  // namespace pic
