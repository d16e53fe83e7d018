// Mixed-precision form of the step: particle positions as a cell index plus an
// FP32 offset in cell units, FP32 velocities, FP32 gather / kick / drift /
// collisions, per-cell FP32 deposition sums with Neumaier compensation.  The
// inverse-CDF roots (for the paper's family, the manufactured positions of
// every drift), N_pairs, the Poisson CG and the error norms stay FP64.
#pragma once

#include "pic_particle.hpp"

namespace pic {

constexpr float kOneBelow = 0x1.fffffep-1f;  // largest float below 1

// Per-launch FP32 constants of the mixed pass.
struct MixConst {
  float dt, dtqm;          // dt and dt q/m
  float inv_h[3];          // 1 / h per dimension (offsets are in cell units)
  float inv_n[3];          // 1 / ncell per dimension
  float emA[3], emB[3];    // phibar e^{t/(2T)} 2 pi / L_d at the kick times of calls A and B
  float vbar;
  float src_w;             // w dt / (2 dV): source prefactor per (N - 1)
  float sigma_ref;
  // the velocity distribution v^M = vhat(t) a of the paper's family (Sec. 5.2);
  // configuration family: vhat = vbar, no kick term
  float vh_drift[3];       // vhat(t^{na+1/2}), the drift's manufactured velocity per unit shape
  float hB[3], hA[3];      // manufactured kick term per unit shape of kicks B and A:
                           // dt vdot^M / 2 = (dt / 2) vhat'(t) a, or in isolation
                           // mode vhat(t_to) - vhat(t_from) (Sec. 5.4.1)
  float h2B[3], h2A[3];    // (vhat / vbar)^2 at the source times of calls B and A
  float pc[3];             // sigma_n vbar^(2n+1): the paper-family source in units of vbar
  float inv_vbar;
};

// Initial state (eq. mms_sol): FP64 roots, then cell + FP32 offset.  An offset
// that would round up to 1 is kept just below it, so the cell is the one the
// FP64 position falls in.
__global__ void __launch_bounds__(kBlock) k_init_mixed(SimConst K, float* off, float* vf, float* ash,
                                                       int* id, int* key, int* slot, int* count) {
  off = mem(K, off);
  vf = mem(K, vf);
  ash = mem(K, ash);
  id = mem(K, id);
  key = mem(K, key);
  slot = mem(K, slot);
  count = mem(K, count);
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  bool valid = p < K.np;
  int kk = 0;
  if (valid) {
    double xi[6], xm[3], a[3];
    init_uniforms(K, p, xi);
    manufactured_position(K, xi, 0.0, nullptr, xm);
    velocity_shape(K, xi + 3, a);
    double vm[3], vd[3];
    manufactured_velocity(K, a, 0.0, vm, vd);
    int c[3];
    double o[3];
    locate(K, xm, c, o);
    kk = lin(K, c[0], c[1], c[2]);
    for (int d = 0; d < 3; ++d) {
      off[d * K.np + p] = fminf((float)o[d], kOneBelow);
      vf[d * K.np + p] = (float)vm[d];
      ash[d * K.np + p] = (float)a[d];
    }
    id[p] = (int)p;
    key[p] = kk;
  }
  int s = wave_aggregated_slot(count, kk, valid);
  if (valid) slot[p] = s;
}

// Positions given by the caller (FP64) as cell + FP32 offset, wrapped as in
// k_set_positions_f64; velocities given by the caller rounded to FP32.
__global__ void __launch_bounds__(kBlock) k_set_positions_mixed(SimConst K, const double* xin,
                                                                float* off, int* key, int* slot,
                                                                int* count, int* flags) {
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  bool valid = p < K.np;
  int kk = 0;
  if (valid) {
    bool bad = false;
    double xp[3];
    for (int d = 0; d < 3; ++d) xp[d] = wrap_box(xin[d * K.np + p], K.L[d], bad);
    if (bad) atomicOr(&flags[kFlagNonFinite], 1);
    int c[3];
    double o[3];
    locate(K, xp, c, o);
    kk = lin(K, c[0], c[1], c[2]);
    for (int d = 0; d < 3; ++d) off[d * K.np + p] = fminf((float)o[d], kOneBelow);
    key[p] = kk;
  }
  int s = wave_aggregated_slot(count, kk, valid);
  if (valid) slot[p] = s;
}

__global__ void __launch_bounds__(kBlock) k_set_velocities_mixed(SimConst K, const double* vin,
                                                                 float* vf) {
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (p >= K.np) return;
  for (int d = 0; d < 3; ++d) vf[d * K.np + p] = (float)vin[d * K.np + p];
}

// Neumaier-compensated accumulation: s + c carries the sum to about FP64 accuracy.
__device__ inline void neumaier_add(float& s, float& c, float x) {
  float t = s + x;
  if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// Cloud-in-cell cell moments with FP32 weights (the offsets are the weights),
// summed in cell-sorted order with compensation; hi and lo parts stored.
__global__ void __launch_bounds__(kBlock) k_deposit_moments_mixed(SimConst K, const float* off,
                                                                  const int* cstart, float* mom) {
  int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= K.nn) return;
  float s[8], e[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) s[k] = e[k] = 0.0f;
  for (int j = cstart[c]; j < cstart[c + 1]; ++j) {
    float ox = off[j], oy = off[K.np + j], oz = off[2 * K.np + j];
    float wx[2] = {1.0f - ox, ox}, wy[2] = {1.0f - oy, oy}, wz[2] = {1.0f - oz, oz};
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx)
          neumaier_add(s[cz * 4 + cy * 2 + cx], e[cz * 4 + cy * 2 + cx], wx[cx] * wy[cy] * wz[cz]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    mom[(int64_t)k * K.nn + c] = s[k];
    mom[(int64_t)(8 + k) * K.nn + c] = e[k];
  }
}

// The compensated cell moments by cell-aligned tiles (see k_deposit_tiles_f64):
// FP32 corner weights in parallel into LDS, then one lane per (cell, corner)
// accumulates them in sorted order with the same Neumaier steps as
// k_deposit_moments_mixed, so the two agree bit for bit.
__device__ inline void cic_weights_mixed(const float o[3], float w[8]) {
  float wx[2] = {1.0f - o[0], o[0]}, wy[2] = {1.0f - o[1], o[1]}, wz[2] = {1.0f - o[2], o[2]};
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) w[cz * 4 + cy * 2 + cx] = wx[cx] * wy[cy] * wz[cz];
}

__global__ void __launch_bounds__(kTileThreads) k_deposit_tiles_mixed(SimConst K, const float* off,
                                                                const int* cstart,
                                                                const int* tile_c0, float* mom) {
  off = mem(K, off);
  cstart = mem(K, cstart);
  tile_c0 = mem(K, tile_c0);
  mom = mem(K, mom);
  __shared__ float W[8 * kLdsSlots];
  __shared__ int sh_i[4];
  tile_range(K, tile_c0, cstart, blockIdx.x, sh_i);
  const int c0 = sh_i[0], ncells = sh_i[1] - sh_i[0], s0 = sh_i[2], ns = sh_i[3] - sh_i[2];
  const bool lds = ns <= kLdsSlots;
  const int NP = (int)K.np;
  if (lds) {
    for (int j = threadIdx.x; j < ns; j += kTileThreads) {
      const int p = s0 + j;
      float o[3] = {off[p], off[NP + p], off[2 * NP + p]}, w[8];
      cic_weights_mixed(o, w);
#pragma unroll
      for (int k = 0; k < 8; ++k) W[k * kLdsSlots + j] = w[k];
    }
    __syncthreads();
  }
  for (int l = threadIdx.x; l < 8 * ncells; l += kTileThreads) {
    const int k = l & 7, c = c0 + (l >> 3);
    const int a = cstart[c] - s0, e = cstart[c + 1] - s0;
    float sum = 0.0f, comp = 0.0f;
    if (lds) {
      for (int j = a; j < e; ++j) neumaier_add(sum, comp, W[k * kLdsSlots + j]);
    } else {
      for (int j = a; j < e; ++j) {
        const int p = s0 + j;
        float o[3] = {off[p], off[NP + p], off[2 * NP + p]}, w[8];
        cic_weights_mixed(o, w);
        neumaier_add(sum, comp, w[k]);
      }
    }
    mom[(int64_t)k * K.nn + c] = sum;
    mom[(int64_t)(8 + k) * K.nn + c] = comp;
  }
}

// Node charge from the compensated FP32 cell moments (summed in FP64) and the
// right-hand side of eq. poisson_mms; block partial sums of b.
__global__ void __launch_bounds__(kBlock) k_node_rhs_mixed(SimConst K, const float* mom, double t,
                                                           double* rho, double* b, double* part,
                                                           const long long* tstep) {
  if (tstep) t = ((double)*tstep + 1.0) * K.dt;  // a captured step: the end of step *tstep
  mom = mem(K, mom);
  rho = mem(K, rho);
  b = mem(K, b);
  part = mem(K, part);
  __shared__ double sh[kWaves];
  int n = blockIdx.x * kBlock + threadIdx.x;
  double bv = 0.0;
  if (n < K.nn) {
    int i, j, k;
    node_coords(K, n, i, j, k);
    double s = 0.0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          int kk = cz * 4 + cy * 2 + cx;
          int cell = lin(K, i - cx, j - cy, k - cz);
          s += (double)mom[(int64_t)kk * K.nn + cell] + (double)mom[(int64_t)(8 + kk) * K.nn + cell];
        }
    double r = K.rho_scale * s;
    rho[n] = r;
    bv = rhs_manufactured(K, i, j, k, t);
    if (K.p2f != 0.0) bv -= r / K.eps0;
    b[n] = bv;
  }
  double tot = block_sum(bv, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Hard-sphere kernel K(l) in FP32 (series below 0.5, closed form above).
__device__ inline float hs_kernel_f(float l) {
  if (l < 0.5f) {
    float bm2 = 0.0f, am2 = 0.0f, bm1 = 1.0f, am1 = 1.0f, sum = 0.0f, l2 = l * l, lp = l;
    for (int j = 1; j < 10; ++j) {
      float bj = bm1 * (-0.5f) / (float)j, aj = bj / (2.0f * j + 1.0f);
      sum += (am2 + 2.0f * am1 - aj + bm1 + bj) * lp;
      am2 = am1; bm2 = bm1; am1 = aj; bm1 = bj;
      lp *= l2;
    }
    (void)bm2;
    return 0.7978845608f * sum;
  }
  float l2 = l * l;
  float phin = 0.3989422804f * expf(-0.5f * l2);
  return ((l2 * l2 + 2.0f * l2 - 1.0f) * erff(0.7071067812f * l) + 2.0f * l * (l2 + 1.0f) * phin) / l2;
}

// eq. vel_change_3 with the paper's f_0, f_1, f_2 (Sec. 5.2 velocity
// distribution) in FP32, in units of vbar: with u~ = u / vbar and
// h2 = (vhat / vbar)^2 the integral is sum_n (sigma_n vbar^(2n+1)) f_n(u~, h2),
// every term a normal FP32 number in any unit system.
__device__ inline void paper_source_f(const SimConst& K, const MixConst& M, const float h2[3],
                                      const float u[3], float out[3]) {
  const float ut[3] = {u[0] * M.inv_vbar, u[1] * M.inv_vbar, u[2] * M.inv_vbar};
  const float u2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  const float H = h2[0] + h2[1] + h2[2];
  const float mix = h2[0] * ut[0] * ut[0] + h2[1] * ut[1] * ut[1] + h2[2] * ut[2] * ut[2];
  for (int i = 0; i < 3; ++i) {
    const float others = h2[(i + 1) % 3] * h2[(i + 2) % 3];
    const float f0 = -ut[i];
    const float f1 = -0.5f * (3.0f * H + 6.0f * h2[i] + 2.0f * u2) * ut[i];
    const float f2 = -0.25f * (15.0f * H * H + 36.0f * h2[i] * h2[i] + 24.0f * u2 * h2[i] +
                               4.0f * u2 * u2 + 24.0f * h2[i] * H + 12.0f * u2 * H +
                               24.0f * mix - 12.0f * others) * ut[i];
    float r = M.pc[0] * f0;
    if (K.n_sigma > 1) r += M.pc[1] * f1;
    if (K.n_sigma > 2) r += M.pc[2] * f2;
    out[i] = r;
  }
}

// eq. vel_change_1c integral in FP32; h2 = (vhat / vbar)^2 at the call's time
// (paper family).
template <int FAM, int SIG>
__device__ inline void source_integral_f(const SimConst& K, const MixConst& M, const float h2[3],
                                         const float u[3], float out[3]) {
  if (FAM == 0 && SIG == kSigPoly) {
    paper_source_f(K, M, h2, u, out);
  } else if (SIG == kSigMaxwell) {
    float c = (float)(K.sigma_ref * K.g_ref);
    for (int i = 0; i < 3; ++i) out[i] = -c * u[i];
  } else if (SIG == kSigHS) {
    float sp = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (sp == 0.0f) {
      out[0] = out[1] = out[2] = 0.0f;
      return;
    }
    float s = M.vbar;
    float kk = hs_kernel_f(sp / s);
    const float f = -M.sigma_ref * s * s * kk / sp;  // one division for the three components
    for (int i = 0; i < 3; ++i) out[i] = f * u[i];
  } else {
    // polynomial cross section with Gaussian moments m2 = s^2, m4 = 3 s^4
    float m2 = M.vbar * M.vbar, m4 = 3.0f * m2 * m2;
    float f[3][3];
    for (int i = 0; i < 3; ++i) {
      int j = (i + 1) % 3, k = (i + 2) % 3;
      float ui2 = u[i] * u[i], uj2 = u[j] * u[j], uk2 = u[k] * u[k];
      float qj = m2 + uj2, qk = m2 + uk2, s1 = qj + qk;
      float s2 = (m4 + 6.0f * uj2 * m2 + uj2 * uj2) + (m4 + 6.0f * uk2 * m2 + uk2 * uk2);
      f[0][i] = -u[i];
      f[1][i] = -u[i] * (3.0f * m2 + ui2 + s1);
      f[2][i] = -u[i] * (5.0f * m4 + 10.0f * ui2 * m2 + ui2 * ui2 + s2 + 2.0f * qj * qk +
                         2.0f * (3.0f * m2 + ui2) * s1);
    }
    for (int i = 0; i < 3; ++i) {
      float r = 0.0f;
      for (int n = 0; n < K.n_sigma; ++n) r += (float)K.sigma_n[n] * f[n][i];
      out[i] = r;
    }
  }
}

// CIC gather of the FP32 nodal field (AoS, 3 floats per node); the offsets are
// the interpolation weights.
__device__ inline void gather_mixed(const SimConst& K, const float* E32, int ci, int cj, int ck,
                                    const float o[3], float ep[3]) {
  ep[0] = ep[1] = ep[2] = 0.0f;
  float wx[2] = {1.0f - o[0], o[0]}, wy[2] = {1.0f - o[1], o[1]}, wz[2] = {1.0f - o[2], o[2]};
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const float* e = E32 + 3 * (int64_t)lin(K, ci + cx, cj + cy, ck + cz);
        float wgt = wx[cx] * wy[cy] * wz[cz];
        ep[0] += wgt * e[0];
        ep[1] += wgt * e[1];
        ep[2] += wgt * e[2];
      }
}

// E^M at the particle in FP32: position fraction (i + o) / n of the box.
__device__ inline void EM_mixed(const MixConst& M, int ci, int cj, int ck, const float o[3],
                                const float amp[3], float em[3]) {
  const float shift[3] = {1.0f / 7.0f, 1.0f / 5.0f, 1.0f / 3.0f};
  const int cc[3] = {ci, cj, ck};
  float s[3], c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float arg = 2.0f * (((float)cc[d] + o[d]) * M.inv_n[d] - shift[d]);
    sincospif(arg, &s[d], &c[d]);
  }
  em[0] = -amp[0] * c[0] * s[1] * s[2];
  em[1] = -amp[1] * s[0] * c[1] * s[2];
  em[2] = -amp[2] * s[0] * s[1] * c[2];
}

// The mixed-form fused pass, same phases as the FP64 one.  FAM: 0 the paper's
// manufactured family (time-dependent velocity distribution; the drift's
// manufactured term comes from k_paper_drift_mixed), 1 the configuration
// family.  Registers are capped for six waves per SIMD (measured best at 64^3:
// the pass is latency bound, and the extra resident waves outweigh the spills).
// DEVC: the instances of captured steps, which take the pass's constants
// from the device (written by k_step_consts) instead of the argument.  SORT:
// long event lists are sorted for the cell threads (sorted_list).
template <int FAM, int SIG, bool FULL, bool FAST, bool DEVC = false, bool SORT = true>
__global__ void __launch_bounds__(kTileThreads, FAST ? PIC_MIXED_LEAN_WAVES : PIC_MIXED_WAVES) k_particles_mixed(SimConst K, MixConst M, PartArgs a,
                                                            float* off, float* vf, const float* ash,
                                                            const float* E32) {
  a = member_view(K, a);
  off = mem(K, off);
  vf = mem(K, vf);
  ash = mem(K, ash);
  E32 = mem(K, E32);
  if constexpr (DEVC) {  // a captured step: its step index and constants from the device
    M = *a.mixc;
    a.nb = *K.stepc;
    a.na = a.nb + 1;
  }
  // Tile-resident copies of what the pass reads per particle more than once
  // (the velocity shape is read once, in the drift, straight from memory), and
  // the field acceleration kept from kick B for kick A; the copy-on-write
  // scratch of outcomes run by a cell thread is global.
  __shared__ float lv0[3 * kLdsSlots], lD[3 * kLdsSlots], loff[3 * kLdsSlots],
      lacc[3 * kLdsSlots];
  __shared__ int lkey[kLdsSlots];
  __shared__ int lcs[kCellCache + 1];  // cell starts of a tile of at most kCellCache cells
  // (the general instance, which takes the dense tiles, has the larger record
  // pool; the full one keeps the small pool and its occupancy)
  __shared__ CollideLds<float, 2, 128, (FAST || FULL) ? kPool : kPoolGeneral> cl;  // both calls drawn up front
  __shared__ int sh_i[4];
  const int tid = threadIdx.x;
  const int NP = (int)K.np;
  auto tile = [&](const int b) __attribute__((always_inline)) {
    if (tid == 0) {
      sh_i[0] = min(a.tile_c0[b], K.nn);
      sh_i[1] = min(a.tile_c0[b + 1], K.nn);
      sh_i[2] = a.tile_s0[b];
      sh_i[3] = a.tile_s0[b + 1];
      tile_lists_clear(cl);
    }
    __syncthreads();
    const int c0 = sh_i[0], ncells = max(sh_i[1] - sh_i[0], 0), s0 = sh_i[2], ns = sh_i[3] - sh_i[2];
    if (ns <= 0) return;
    if (FAST && ns > kLdsSlots) {  // (uniform) the general instance takes this tile
      defer_tile(a, b);
      return;
    }
    const bool lds = FAST || ns <= kLdsSlots;
    const int st = lds ? kLdsSlots : NP;
    float* v0 = lds ? lv0 : (float*)a.gv0 + s0;
    float* D = lds ? lD : (float*)a.gD + s0;
    const float* to = lds ? loff : off + s0;   // offsets at the start of the pass
    const int* tk = lds ? lkey : a.key + s0;   // cells at the start of the pass
    float* u = (float*)a.gu + s0;
    int* mark = a.gmark + s0;
    int* tl = a.gtl + s0;
    const float navg_f = (float)K.navg;
    const float inv_navg = 1.0f / navg_f;  // exact for a power-of-two N_avg

    // Field part of a half kick: dt q/m (E - E^M) at cell c, offset o.
    auto field_acc_at = [&](int c, const float o[3], const float amp[3], float acc[3]) {
      int ci, cj, ck;
      node_coords(K, c, ci, cj, ck);
      float ep[3], em[3];
      gather_mixed(K, E32, ci, cj, ck, o, ep);
      EM_mixed(M, ci, cj, ck, o, amp, em);
      for (int d = 0; d < 3; ++d) acc[d] = M.dtqm * (ep[d] - em[d]);
    };
    // A tile held in LDS computes the field part of its first kick while it
    // loads (the gather's loads then overlap the tile's other loads) and keeps
    // it in lacc; with both halves in one pass, kick B (end of step n) and kick A
    // (start of step n + 1) are at the same time t^{n+1} and position (no drift
    // between them, one field solve before the pass), so kick A reuses it:
    // bitwise what it would compute again.
    const bool pre = lds && !(a.mode & kCollideOnly);
    const bool reuse_A = pre && (!(a.mode & kDoB) || a.na == a.nb + 1);
    const float* amp0 = (a.mode & kDoB) ? M.emB : M.emA;
    const bool pass_coll = K.collisions && !(a.mode & kCollideOnly);
    if (pass_coll) tile_zero_D(ns, st, D);
    for (int j = tid; j < ns; j += kTileThreads) {
      const int p = s0 + j;
      for (int d = 0; d < 3; ++d) v0[d * st + j] = vf[(int64_t)d * NP + p];
      if (lds) {
        const int c = a.key[p];
        const float o[3] = {off[p], off[(int64_t)NP + p], off[2 * (int64_t)NP + p]};
        for (int d = 0; d < 3; ++d) loff[d * kLdsSlots + j] = o[d];
        lkey[j] = c;
        if (pre) {
          float acc[3];
          field_acc_at(c, o, amp0, acc);
          for (int d = 0; d < 3; ++d) lacc[d * kLdsSlots + j] = acc[d];
        }
      }
    }
    const bool few_cells = ncells <= kCellCache;
    if (few_cells)
      for (int i = tid; i <= ncells; i += kTileThreads) lcs[i] = a.cstart[c0 + i];
    if (pass_coll) tile_draw_pass(K, a, c0, ncells, cl);
    __syncthreads();
    if (FAST && pass_coll &&
        !tile_lane_only(cl, (a.mode & kDoB) ? 0 : 1, (a.mode & kDoA) ? 2 : 1)) {
      defer_tile(a, b);  // (uniform, and nothing written to memory yet)
      return;
    }
    auto cell_count = [&](int j) {
      const int c = tk[j];
      if (few_cells) return lcs[c - c0 + 1] - lcs[c - c0];
      return a.cstart[c + 1] - a.cstart[c];
    };

    // Field part of a half kick at slot j (tiles not held in LDS).
    auto field_acc = [&](int j, const float amp[3], float acc[3]) {
      const float o[3] = {to[j], to[st + j], to[2 * st + j]};
      field_acc_at(tk[j], o, amp, acc);
    };
    // Half kick of slot j: v += (acc + <dv> - <dv^M>) / 2, plus (paper family)
    // the manufactured term hman a with the particle's velocity shape a; h2 is
    // (vhat / vbar)^2 at the call's source time.
    auto kick_with = [&](int j, const float acc[3], bool coll_on, const float* h2,
                         const float* hman, const float* sa) {
      float vp[3] = {v0[j], v0[st + j], v0[2 * st + j]};
      float coll[3] = {0.0f, 0.0f, 0.0f};
      if (coll_on) {
        int n = cell_count(j);
        float I[3] = {0.0f, 0.0f, 0.0f};
        float coef = M.src_w * (float)(n - 1);
        if (n >= 2) source_integral_f<FAM, SIG>(K, M, h2, vp, I);
        for (int d = 0; d < 3; ++d) {
          coll[d] = D[d * st + j] * inv_navg - ((n >= 2) ? coef * I[d] : 0.0f);
          D[d * st + j] = 0.0f;  // cleared for the next call (a barrier follows every kick)
        }
      }
      for (int d = 0; d < 3; ++d) {
        float nv = vp[d] + 0.5f * (acc[d] + coll[d]);
        if constexpr (FAM == 0) nv = nv + hman[d] * sa[d];
        vp[d] = nv;
        v0[d * st + j] = vp[d];
      }
    };

    if (!FAST && (a.mode & kCollideOnly)) {  // (the lean instance never runs collide-only)
      tile_collide<SIG, float, FULL>(K, a, a.callA, a.na, c0, ncells, s0, ns, v0, u, D, mark, tl, 0, st,
                               NP, cl);
      for (int j = tid; j < ns; j += kTileThreads) {
        int n = cell_count(j);
        float vp[3] = {v0[j], v0[st + j], v0[2 * st + j]}, I[3] = {0, 0, 0};
        float coef = M.src_w * (float)(n - 1);
        if (n >= 2) source_integral_f<FAM, SIG>(K, M, M.h2A, vp, I);
        for (int d = 0; d < 3; ++d) {
          a.Dout[(int64_t)d * NP + s0 + j] = (double)(D[d * st + j] * inv_navg);
          a.Sout[(int64_t)d * NP + s0 + j] = (n >= 2) ? (double)(coef * I[d]) : 0.0;
        }
      }
      return;
    }

    if (a.mode & kDoB) {  // call B at t^{nb+1/2}, second half kick at t^{nb+1}
      if (K.collisions)
        tile_run<SIG, float, FULL, FAST, SORT>(K, a, 0, a.callB, a.nb, c0, ncells, s0, ns, v0, u, D, mark, tl, 0, st,
                                 NP, cl, few_cells ? lcs : nullptr);
      for (int j = tid; j < ns; j += kTileThreads) {
        float acc[3], sa[3] = {0.0f, 0.0f, 0.0f};
        if constexpr (FAM == 0) {
          const int p = s0 + j;
          for (int d = 0; d < 3; ++d) sa[d] = ash[(int64_t)d * NP + p];
        }
        if (pre) {
          for (int d = 0; d < 3; ++d) acc[d] = lacc[d * kLdsSlots + j];
        } else {
          field_acc(j, M.emB, acc);
        }
        kick_with(j, acc, K.collisions != 0, M.h2B, M.hB, sa);
      }
      if (tid == 0) cl.pool_n = 0;
      __syncthreads();
      if (!(a.mode & kDoA)) {
        for (int j = tid; j < ns; j += kTileThreads)
          for (int d = 0; d < 3; ++d) vf[(int64_t)d * NP + s0 + j] = v0[d * st + j];
        return;
      }
    }

    // call A at t^{na}, first half kick, drift to t^{na+1}
    if (K.collisions)
      tile_run<SIG, float, FULL, FAST, SORT>(K, a, 1, a.callA, a.na, c0, ncells, s0, ns, v0, u, D, mark, tl, K.navg,
                               st, NP, cl, few_cells ? lcs : nullptr);
    for (int base = 0; base < ns; base += kTileThreads) {
      int j = base + tid;
      bool valid = j < ns;
      int kk = 0;
      if (valid) {
        int p = s0 + j;
        // the velocity shape for the drift, loaded before the kick hides its latency
        const float sa[3] = {ash[p], ash[(int64_t)NP + p], ash[2 * (int64_t)NP + p]};
        float acc[3];
        if (reuse_A) {
          for (int d = 0; d < 3; ++d) acc[d] = lacc[d * kLdsSlots + j];
        } else {
          field_acc(j, M.emA, acc);
        }
        kick_with(j, acc, K.collisions != 0, M.h2A, M.hA, sa);
        int c = tk[j];
        int cc[3];
        node_coords(K, c, cc[0], cc[1], cc[2]);
        // Paper family: the manufactured term of the drift, in cells, from
        // k_paper_drift_mixed
        float dman[3] = {0.0f, 0.0f, 0.0f};
        if constexpr (FAM == 0)
          for (int d = 0; d < 3; ++d) dman[d] = a.mdrift32[(int64_t)d * NP + p];
        float on[3];
        for (int d = 0; d < 3; ++d) {
          // x += dt (v - v^M) in cell units, v^M = vhat(t^{n+1/2}) a, plus the
          // manufactured displacement (paper family)
          float vm = M.vh_drift[d] * sa[d];
          float o = to[d * st + j] + M.dt * (v0[d * st + j] - vm) * M.inv_h[d];
          if constexpr (FAM == 0) o = o + dman[d];
          float fl = floorf(o);
          o -= fl;
          int shift = (int)fl;
          if (o >= 1.0f) {  // a tiny negative offset rounds up to 1 after adding 1
            o -= 1.0f;
            shift += 1;
          }
          if (!(o >= 0.0f && o < 1.0f)) {  // non-finite
            atomicOr(&a.flags[kFlagNonFinite], 1);
            o = 0.0f;
            shift = 0;
          }
          const int nd = K.nc[d];
          if (shift >= nd || shift <= -nd) shift %= nd;  // more than a box length: rare
          int ni = cc[d] + shift;
          ni = ni < 0 ? ni + nd : (ni >= nd ? ni - nd : ni);
          cc[d] = ni;
          on[d] = o;
        }
        // (the global copies are written only now: in a large tile `to` and
        // `tk` read the global arrays themselves)
        for (int d = 0; d < 3; ++d) {
          off[(int64_t)d * NP + p] = on[d];
          vf[(int64_t)d * NP + p] = v0[d * st + j];
        }
        kk = (cc[2] * K.nc[1] + cc[1]) * K.nc[0] + cc[0];
        a.key[p] = kk;
      }
      int sl = wave_aggregated_slot(a.count, kk, valid);
      if (valid) a.slot[s0 + j] = sl;
    }
  };
  tile_sweep<FAST>(a, tile);
}

// Paper family: the manufactured term of every particle's drift in step na,
// in cells (FP32), from FP64 root solves of x^M (eq. mms_sol) started at the
// particle's position at the start of the pass: dt xdot^M at t^{na+1/2}, or
// x^M(t^{na+1}) - x^M(t^{na}) in isolation mode.  It depends only on the
// particle's identity, that position and the time, so it runs before the pass
// (which then keeps no root solver and its register budget); out is the idle
// half of the double-buffered offsets.
__global__ void __launch_bounds__(kBlock) k_paper_drift_mixed(SimConst K, PartArgs a, const float* off,
                                                              float* out) {
  a = member_view(K, a);
  off = mem(K, off);
  out = mem(K, out);
  if (a.step_dev) {  // a captured step: its step index from the device
    a.nb = *K.stepc;
    a.na = a.nb + 1;
  }
  const int64_t NP = K.np;
  const double t0 = (double)a.na * K.dt, th = ((double)a.na + 0.5) * K.dt,
               t1 = ((double)a.na + 1.0) * K.dt;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < NP;
       p += (int64_t)gridDim.x * blockDim.x) {
    int cc[3];
    node_coords(K, a.key[p], cc[0], cc[1], cc[2]);
    double xq[3], xg[3], disp[3];
    position_uniforms(K, a.id[p], xq);
    for (int d = 0; d < 3; ++d) xg[d] = ((double)cc[d] + (double)off[d * NP + p]) * K.h[d];
    if (K.isolate) {
      double xa[3], xb[3];
      manufactured_position(K, xq, t0, xg, xa);
      manufactured_position(K, xq, t1, xa, xb);
      for (int d = 0; d < 3; ++d) disp[d] = xb[d] - xa[d];
    } else {
      double xm[3], xd[3];
      manufactured_position(K, xq, th, xg, xm);
      manufactured_xdot(K, xm, th, xd);
      for (int d = 0; d < 3; ++d) disp[d] = K.dt * xd[d];
    }
    for (int d = 0; d < 3; ++d) out[d * NP + p] = (float)(disp[d] * K.inv_h[d]);
  }
}

// Positions and velocities exported as FP64 (component-major).
__global__ void __launch_bounds__(kBlock) k_export_mixed(SimConst K, const int* key, const float* off,
                                                         const float* vf, double* x, double* v) {
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (p >= K.np) return;
  int c = key[p];
  int cc[3];
  node_coords(K, c, cc[0], cc[1], cc[2]);
  for (int d = 0; d < 3; ++d) {
    if (x) x[d * K.np + p] = ((double)cc[d] + (double)off[d * K.np + p]) * K.h[d];
    if (v) v[d * K.np + p] = (double)vf[d * K.np + p];
  }
}

// Error norms of the mixed state: positions rebuilt in FP64, manufactured
// values from FP64 roots, FP64 reductions (same fixed grid and order as
// k_err_particles_f64).
__global__ void __launch_bounds__(kBlock) k_err_particles_mixed(SimConst K, double t, const int* key,
                                                                const float* off, const float* vf,
                                                                const int* id, double* part,
                                                                int* flags) {
  key = mem(K, key);
  off = mem(K, off);
  vf = mem(K, vf);
  id = mem(K, id);
  part = mem(K, part);
  flags = mem(K, flags);
  __shared__ double sh[kWaves];
  double s2[6] = {0, 0, 0, 0, 0, 0}, mx[6] = {0, 0, 0, 0, 0, 0};
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < K.np;
       i += (int64_t)gridDim.x * kBlock) {
    double xq[3], xv[3], xm[3], a[3], vm[3], vd[3], e[6];
    position_uniforms(K, id[i], xq);
    velocity_uniforms(K, id[i], xv);
    int c = key[i];
    int cc[3];
    node_coords(K, c, cc[0], cc[1], cc[2]);
    double xp[3];
    for (int d = 0; d < 3; ++d) xp[d] = ((double)cc[d] + (double)off[d * K.np + i]) * K.h[d];
    manufactured_position(K, xq, t, xp, xm);
    velocity_shape(K, xv, a);
    manufactured_velocity(K, a, t, vm, vd);
    for (int d = 0; d < 3; ++d) {
      double ex = xp[d] - xm[d];
      if (ex >= 0.5 * K.L[d]) ex -= K.L[d];
      if (ex < -0.5 * K.L[d]) ex += K.L[d];
      e[d] = ex;
      e[3 + d] = (double)vf[d * K.np + i] - vm[d];
    }
    for (int a2 = 0; a2 < 6; ++a2) {
      bad |= !isfinite(e[a2]);
      s2[a2] += e[a2] * e[a2];
      mx[a2] = fmax(mx[a2], fabs(e[a2]));
    }
  }
  if (bad) atomicOr(&flags[kFlagNonFinite], 1);
  for (int a2 = 0; a2 < 6; ++a2) {
    double s = block_sum(s2[a2], sh);
    double m = block_max(mx[a2], sh);
    if (threadIdx.x == 0) {
      part[blockIdx.x * 14 + a2] = s;
      part[blockIdx.x * 14 + 7 + a2] = m;
    }
  }
}

}  // namespace pic
