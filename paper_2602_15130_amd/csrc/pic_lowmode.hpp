// Exact solve of the lowest Fourier modes before the Poisson CG.
//
// The periodic 7-point operator A = -L_h is diagonalised by the discrete
// Fourier modes, so the products phi_a(i) phi_b(j) phi_c(k) of the 1-D modes
// 1, cos(2 pi k i / n), sin(2 pi k i / n) (k = 1..K_d) are exact eigenvectors
// with eigenvalue mu_a + mu_b + mu_c, mu = 4 sin^2(pi k / n) / h^2.  Before the
// CG, the initial residual r_0 = -b - A x_0 is projected on those modes and x_0
// corrected by coefficient / eigenvalue, which removes every low-mode
// component of the residual; the CG that follows (same recurrence, same
// stopping rule) then works on the remaining spectrum, whose smallest
// eigenvalue is several times larger, and needs proportionally fewer
// iterations.  The projection and the correction are separable: three 1-D
// transforms each way, every sum in a fixed order.
#pragma once

#include "pic_kernels.hpp"

namespace pic {

constexpr int kLowMaxK = 4;                  // modes per axis beyond the constant
constexpr int kLowMaxM = 2 * kLowMaxK + 1;   // 1-D basis functions per axis

struct LowArgs {
  int m[3];             // 1-D basis functions per axis, 2 K_d + 1
  int nmax;             // largest axis length (table stride)
  const double* tab;    // [3][kLowMaxM][nmax] basis values
  const double* mu;     // [3][kLowMaxM] 1-D eigenvalues
  double* t1;           // [m0][nz][ny] projections of the x lines
  double* t2;           // [m0][m1][nz]
  double* d1;           // [m2][m1][nx] partial back-transform
};

// 1-D basis function a at index i of an axis of n nodes: 1, then cos and sin
// of 2 pi k i / n for k = 1, 2, ...  (angle reduced exactly in integers).
__device__ inline double low_basis(int a, int i, int n) {
  if (a == 0) return 1.0;
  const int k = (a + 1) / 2;
  const double arg = (double)((2 * k * i) % (2 * n)) / (double)n;  // in units of pi
  return (a & 1) ? cospi(arg) : sinpi(arg);
}

__global__ void __launch_bounds__(kBlock) k_low_tables(SimConst K, LowArgs L, double* tab,
                                                       double* mu) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int per_axis = kLowMaxM * L.nmax;
  if (t < 3 * per_axis) {
    const int d = t / per_axis, a = (t / L.nmax) % kLowMaxM, i = t % L.nmax;
    tab[t] = (a < L.m[d] && i < K.nc[d]) ? low_basis(a, i, K.nc[d]) : 0.0;
  }
  if (t < 3 * kLowMaxM) {
    const int d = t / kLowMaxM, a = t % kLowMaxM;
    double v = 0.0;
    if (a > 0 && a < L.m[d]) {
      const double s = sinpi((double)((a + 1) / 2) / (double)K.nc[d]);
      v = 4.0 * s * s * K.ih2[d];
    }
    mu[t] = v;
  }
}

// Pass 1: r_0 = -b - A x_0 along each x line (one wave per line), projected on
// the x basis: t1[a][k][j] = sum_i r_0(i, j, k) phi_a(i).
__global__ void __launch_bounds__(64) k_low_project_x(SimConst K, LowArgs L, const double* b,
                                                      const double* x) {
  const int line = blockIdx.x, j = line % K.nc[1], k = line / K.nc[1];
  double acc[kLowMaxM];
#pragma unroll
  for (int a = 0; a < kLowMaxM; ++a) acc[a] = 0.0;
  for (int i = threadIdx.x; i < K.nc[0]; i += 64) {
    const int n = lin(K, i, j, k);
    const double r = -b[n] - neg_lap(K, i, j, k, [&](int m) { return x[m]; });
#pragma unroll
    for (int a = 0; a < kLowMaxM; ++a)
      if (a < L.m[0]) acc[a] += r * L.tab[a * L.nmax + i];
  }
#pragma unroll
  for (int a = 0; a < kLowMaxM; ++a) {
    if (a >= L.m[0]) break;
    const double s = wave_sum(acc[a]);
    if (threadIdx.x == 0) L.t1[((int64_t)a * K.nc[2] + k) * K.nc[1] + j] = s;
  }
}

// Pass 2: t2[a][b][k] = sum_j t1[a][k][j] phi_b(j).
__global__ void __launch_bounds__(kBlock) k_low_project_y(SimConst K, LowArgs L) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= L.m[0] * L.m[1] * K.nc[2]) return;
  const int k = t % K.nc[2], bb = (t / K.nc[2]) % L.m[1], a = t / (K.nc[2] * L.m[1]);
  const double* row = L.t1 + ((int64_t)a * K.nc[2] + k) * K.nc[1];
  const double* ph = L.tab + (kLowMaxM + bb) * L.nmax;
  double s = 0.0;
  for (int j = 0; j < K.nc[1]; ++j) s += row[j] * ph[j];
  L.t2[t] = s;  // index (a * m1 + bb) * nz + k
}

// Pass 3 (one block): coefficients c[a][b][c] = sum_k t2[a][b][k] phi_c(k),
// scaled by 1 / (eigenvalue * squared norm) (the constant mode is left
// alone), then the first back-transform d1[c][b][i] = sum_a c'[a][b][c] phi_a(i).
__global__ void __launch_bounds__(1024) k_low_solve(SimConst K, LowArgs L) {
  __shared__ double cf[kLowMaxM * kLowMaxM * kLowMaxM];
  const int m0 = L.m[0], m1 = L.m[1], m2 = L.m[2];
  for (int t = threadIdx.x; t < m0 * m1 * m2; t += blockDim.x) {
    const int cc = t % m2, bb = (t / m2) % m1, a = t / (m2 * m1);
    const double* row = L.t2 + ((int64_t)a * m1 + bb) * K.nc[2];
    const double* ph = L.tab + (2 * kLowMaxM + cc) * L.nmax;
    double s = 0.0;
    for (int k = 0; k < K.nc[2]; ++k) s += row[k] * ph[k];
    const double lam = L.mu[a] + L.mu[kLowMaxM + bb] + L.mu[2 * kLowMaxM + cc];
    const double nrm = (a ? 0.5 : 1.0) * (bb ? 0.5 : 1.0) * (cc ? 0.5 : 1.0) * (double)K.nn;
    cf[t] = lam > 0.0 ? s / (lam * nrm) : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < m2 * m1 * K.nc[0]; t += blockDim.x) {
    const int i = t % K.nc[0], bb = (t / K.nc[0]) % m1, cc = t / (K.nc[0] * m1);
    double s = 0.0;
    for (int a = 0; a < m0; ++a) s += cf[(a * m1 + bb) * m2 + cc] * L.tab[a * L.nmax + i];
    L.d1[t] = s;  // index (cc * m1 + bb) * nx + i
  }
}

// Pass 4: x(i, j, k) += sum_c phi_c(k) sum_b phi_b(j) d1[c][b][i].
__global__ void __launch_bounds__(kBlock) k_low_correct(SimConst K, LowArgs L, double* x) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= K.nn) return;
  int i, j, k;
  node_coords(K, n, i, j, k);
  double s = 0.0;
  for (int cc = 0; cc < L.m[2]; ++cc) {
    double sb = 0.0;
    for (int bb = 0; bb < L.m[1]; ++bb)
      sb += L.d1[((int64_t)cc * L.m[1] + bb) * K.nc[0] + i] * L.tab[(kLowMaxM + bb) * L.nmax + j];
    s += sb * L.tab[(2 * kLowMaxM + cc) * L.nmax + k];
  }
  x[n] += s;
}

}  // namespace pic
