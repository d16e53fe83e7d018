// Collision calls where cells hold hundreds of particles and every outcome
// has tens of candidate pairs (the paper's refinement ladder: N_avg up to
// thousands, Table 1).  One workgroup per cell; each wave runs outcomes
// k = wave, wave + W, ... of Algorithm 1:
//   - the lanes draw the random blocks of the outcome's pairs in parallel
//     (pair m on lane m mod 64) and leave (p, q, U_acc, U_eps, U_chi) in LDS;
//   - lane 0 applies the pairs in order with the outcome's private velocities
//     kept in a per-wave map (slot -> list entry, tagged by the outcome) and
//     list (the touched slots and their current velocities), reading all
//     untouched velocities from the pre-collision state;
//   - the lanes add the outcome's velocity changes to the cell's accumulators.
// The accumulators are fixed point (int64, the change times 2^scale_bits):
// integer sums do not depend on the order in which the waves finish, so the
// result is reproducible, and the quantum 2^-scale_bits (chosen from N_avg and
// g_max so the sums cannot overflow) sits far below the FP64 state's rounding.
// <dv> = sum / N_avg (eq. avg_outcome).
#pragma once

#include "pic_kernels.hpp"

namespace pic {

constexpr int kHeavyWaves = 4;
// kHeavyMaxN particles per cell, kHeavyMaxPairs candidate pairs per outcome;
// cells that could exceed them (heavy_big_cell) are left to k_collide_f64.

struct HeavyWaveLds {
  unsigned mark[kHeavyMaxN];          // (outcome tag << 9) | list entry
  int lslot[2 * kHeavyMaxPairs];
  double lval[3][2 * kHeavyMaxPairs];
  int pp[64], pq[64];
  double pacc[64], peps[64], pchi[64];
};

constexpr size_t kHeavyLdsBytes = 3 * kHeavyMaxN * sizeof(long long) + kHeavyWaves * sizeof(HeavyWaveLds);

// Pre-collision velocities of the cell: v0[d * NP + s + j].
__global__ void __launch_bounds__(64 * kHeavyWaves) k_collide_heavy(SimConst K, int call, int64_t step,
                                                                    const double* v, const int* cstart,
                                                                    double* D, int scale_bits,
                                                                    long long* pairlog, int64_t cap,
                                                                    unsigned long long* counters,
                                                                    int* flags) {
  extern __shared__ char smem[];
  long long* acc = (long long*)smem;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  HeavyWaveLds& W = ((HeavyWaveLds*)(smem + 3 * kHeavyMaxN * sizeof(long long)))[wave];
  const int64_t NP = K.np;
  const int c = blockIdx.x;
  const int s = cstart[c], n = cstart[c + 1] - s;
  if (heavy_big_cell(K, n)) return;  // run by k_collide_f64 (big_only)
  if (n < 2) {
    for (int j = threadIdx.x; j < n; j += 64 * kHeavyWaves)
      for (int d = 0; d < 3; ++d) D[d * NP + s + j] = 0.0;
    return;
  }
  for (int j = threadIdx.x; j < 3 * n; j += 64 * kHeavyWaves) acc[j] = 0;
  for (int j = lane; j < n; j += 64) W.mark[j] = 0u;
  __syncthreads();

  const double scale = ldexp(1.0, scale_bits);
  const double dv_max = 8.0 * K.g_max;
  unsigned long long nacc = 0, ngmx = 0;
  unsigned tag = 0;
  for (int k = wave; k < K.navg; k += kHeavyWaves) {
    const U64x4 nb = stream_block(K, (uint64_t)c, (uint64_t)step, kTagNpairs, (uint64_t)call,
                                  (uint64_t)(k >> 2), 0);
    const double xp = (double)n * (double)(n - 1) * K.pmax / 2.0 + unif(nb.w[k & 3]);
    if (!(xp < (double)(kHeavyMaxPairs + 1))) {
      if (lane == 0) atomicOr(&flags[kFlagCapacity], 1);
      continue;
    }
    const int npairs = (int)floor(xp);
    if (npairs <= 0) continue;
    ++tag;
    int cnt = 0;  // list entries (meaningful on lane 0)
    for (int base = 0; base < npairs; base += 64) {
      const int m = base + lane;
      if (m < npairs) {
        U64x4 wa = stream_block(K, (uint64_t)c, (uint64_t)step, kTagColl, (uint64_t)call,
                                (uint64_t)k, (uint64_t)(1 + 2 * m));
        U64x4 wb = stream_block(K, (uint64_t)c, (uint64_t)step, kTagColl, (uint64_t)call,
                                (uint64_t)k, (uint64_t)(2 + 2 * m));
        const int p = index_below(wa.w[0], n);
        W.pp[lane] = p;
        W.pq[lane] = pick_partner(K, c, step, call, k, m, wa, wb, p, n);
        W.pacc[lane] = unif(wa.w[2]);
        W.peps[lane] = unif(wa.w[3]);
        W.pchi[lane] = unif(wb.w[0]);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (lane == 0) {
        const int mend = min(64, npairs - base);
        for (int j = 0; j < mend; ++j) {
          const int p = W.pp[j], q = W.pq[j];
          const unsigned mp = W.mark[p], mq = W.mark[q];
          int ip = (mp >> 9) == tag ? (int)(mp & 511u) : -1;
          int iq = (mq >> 9) == tag ? (int)(mq & 511u) : -1;
          double up[3], uq[3];
          for (int d = 0; d < 3; ++d) {
            up[d] = ip >= 0 ? W.lval[d][ip] : v[d * NP + s + p];
            uq[d] = iq >= 0 ? W.lval[d][iq] : v[d * NP + s + q];
          }
          const double dx = up[0] - uq[0], dy = up[1] - uq[1], dz = up[2] - uq[2];
          const double g = sqrt(dx * dx + dy * dy + dz * dz);
          if (g > K.g_max) ++ngmx;
          const bool ok = W.pacc[j] < sigma_g(K, g) / K.sgmax;
          if (ok) {
            ++nacc;
            double seps, ceps;  // eps = 2 pi U_eps, as sin(pi 2 U) and cos(pi 2 U)
            sincospi(2.0 * W.peps[j], &seps, &ceps);
            const double cchi = cos_chi<double>(K, W.pchi[j]);  // eq. chi
            const double schi = sqrt(fmax(0.0, (1.0 - cchi) * (1.0 + cchi)));
            const double nv[3] = {ceps * schi, seps * schi, cchi};  // eq. n
            if (ip < 0) {
              ip = cnt++;
              W.lslot[ip] = p;
              W.mark[p] = (tag << 9) | (unsigned)ip;
            }
            if (iq < 0) {
              iq = cnt++;
              W.lslot[iq] = q;
              W.mark[q] = (tag << 9) | (unsigned)iq;
            }
            double pn[3], qn[3];
            post_collision<double, true>(K, up, uq, g, nv, W.pchi[j], pn, qn);
            for (int d = 0; d < 3; ++d) {
              W.lval[d][ip] = pn[d];
              W.lval[d][iq] = qn[d];
            }
            record_angles<double>(pn, qn, g, K.anglog, K.angcap, counters);
          }
          if (pairlog) {
            unsigned long long slot = atomicAdd(&counters[kCntPairLog], 1ull);
            if ((int64_t)slot < cap) {
              long long* r = pairlog + 7 * slot;
              r[0] = c; r[1] = call; r[2] = k; r[3] = base + j; r[4] = p; r[5] = q; r[6] = ok;
            }
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    cnt = __shfl(cnt, 0);
    // the outcome's velocity changes into the cell's fixed-point sums
    for (int t = lane; t < cnt; t += 64) {
      const int j = W.lslot[t];
      for (int d = 0; d < 3; ++d) {
        double dv = W.lval[d][t] - v[d * NP + s + j];
        if (!(fabs(dv) <= dv_max)) {
          atomicOr(&flags[kFlagCapacity], 1);
          dv = dv > 0.0 ? dv_max : -dv_max;
        }
        atomicAdd((unsigned long long*)&acc[d * n + j], (unsigned long long)llrint(dv * scale));
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  if (lane == 0) {
    if (nacc) atomicAdd(&counters[kCntAccepted], nacc);
    if (ngmx) atomicAdd(&counters[kCntGmax], ngmx);
  }
  __syncthreads();
  const double inv = 1.0 / (scale * (double)K.navg);
  for (int j = threadIdx.x; j < 3 * n; j += 64 * kHeavyWaves) {
    const int d = j / n, jj = j - d * n;
    D[d * NP + s + jj] = (double)acc[j] * inv;
  }
}

// Bits of the fixed-point scale for N_avg outcomes: the sum of N_avg changes of
// magnitude at most 8 g_max stays below 2^62.
inline int heavy_scale_bits(double g_max, int navg) {
  const double bound = 8.0 * g_max * (double)navg;
  int e = 0;
  std::frexp(bound, &e);  // bound < 2^e
  return 62 - e;
}

}  // namespace pic
