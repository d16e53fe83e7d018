// Errors of the empirical CDFs of the recorded scattering angles against the
// analytic ones (the metric that follows eq. angle_recovery): the records are
// mapped through the analytic CDFs, F_chi of the polar-angle model and
// F_eps = eps / (2 pi), sorted (bitonic network over a power-of-two padded
// copy), and e_i = (rank of the last equal value) / N - F(alpha_(i)) is
// reduced to its root mean square and maximum with fixed-order sums.
#pragma once

#include "pic_kernels.hpp"

namespace pic {

// F_pchi(chi) of the polar-angle model: (1 - cos chi)/2 (eq. chi_iso);
// sin^2(chi/2) - (3 + 5 cos 2 chi) sin^2(chi) / 58 (manufactured anisotropy,
// Sec. 5.2); 1 - cos^(2 alpha)(chi/2) (eq. vss).
__device__ inline double chi_cdf(int model, double alpha, double chi) {
  if (model == 1) {
    const double s2 = sin(0.5 * chi), sc = sin(chi);
    return s2 * s2 - (3.0 + 5.0 * cos(2.0 * chi)) * sc * sc / 58.0;
  }
  if (model == 2) return 1.0 - pow(cos(0.5 * chi), 2.0 * alpha);
  return 0.5 * (1.0 - cos(chi));
}

// u[which][i] = F^M(alpha_i) for i < n, 2 (sorts last) up to the padded size P.
__global__ void __launch_bounds__(kBlock) k_angle_map(const double* rec, int64_t n, int64_t P,
                                                      int model, double alpha, double* u) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= P) return;
  if (i < n) {
    u[i] = chi_cdf(model, alpha, rec[2 * i]);
    u[P + i] = rec[2 * i + 1] / (2.0 * kPi);
  } else {
    u[i] = u[P + i] = 2.0;
  }
}

// One compare-exchange stage (k, j) of the bitonic sorting network on both
// arrays (P a power of two, one thread per element).
__global__ void __launch_bounds__(kBlock) k_bitonic_stage(double* u, int64_t P, int64_t k,
                                                          int64_t j) {
  const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (t >= 2 * P) return;
  const int64_t base = t >= P ? P : 0, i = t - base, l = i ^ j;
  if (l <= i) return;
  double* a = u + base;
  const bool up = (i & k) == 0;
  const double x = a[i], y = a[l];
  if ((x > y) == up) {
    a[i] = y;
    a[l] = x;
  }
}

// Block partial sums of e^2 and block maxima of |e| over the sorted values.
__global__ void __launch_bounds__(kBlock) k_angle_err(const double* u, int64_t n, int64_t P,
                                                      double* part) {
  __shared__ double sh[kWaves];
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  double e2[2] = {0.0, 0.0}, em[2] = {0.0, 0.0};
  if (i < n) {
    for (int w = 0; w < 2; ++w) {
      const double* a = u + w * P;
      // theta(0) = 1: equal values share the rank of the last of them
      int64_t lo = i, hi = n - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (a[mid] == a[i]) lo = mid; else hi = mid - 1;
      }
      const double e = (double)(lo + 1) / (double)n - a[i];
      e2[w] = e * e;
      em[w] = fabs(e);
    }
  }
  for (int w = 0; w < 2; ++w) {
    double s = block_sum(e2[w], sh);
    double m = block_max(em[w], sh);
    if (threadIdx.x == 0) {
      part[4 * blockIdx.x + 2 * w] = s;
      part[4 * blockIdx.x + 2 * w + 1] = m;
    }
  }
}

// out = {eps_2 chi, eps_inf chi, eps_2 eps, eps_inf eps} from the block partials.
__global__ void __launch_bounds__(kBlock) k_angle_final(const double* part, int nb, int64_t n,
                                                        double* out) {
  __shared__ double sh[kWaves];
  for (int w = 0; w < 2; ++w) {
    double s = 0.0, m = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
      s += part[4 * b + 2 * w];
      m = fmax(m, part[4 * b + 2 * w + 1]);
    }
    s = block_sum(s, sh);
    m = block_max(m, sh);
    if (threadIdx.x == 0) {
      out[2 * w] = n > 0 ? sqrt(s / (double)n) : 0.0;
      out[2 * w + 1] = m;
    }
  }
}

}  // namespace pic
