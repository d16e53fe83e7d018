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

constexpr int kLowMaxK = 24;                 // modes per axis beyond the constant (at most)
constexpr int kLowDefaultK = 24;             // default modes per axis (fewest CG iterations)
constexpr int kLowMaxM = 2 * kLowMaxK + 1;   // 1-D basis functions per axis
constexpr int kLowChunk = 16;                // mesh rows staged in LDS at a time
constexpr int kLowBlocks = 256;              // target workgroups of the plane passes
constexpr int kLowThreads = 1024;            // threads per workgroup of the three passes

struct LowArgs {
  int m[3];             // 1-D basis functions per axis, 2 K_d + 1
  int nmax;             // largest axis length (table stride)
  int slabs, rows;      // each z plane is split into `slabs` slabs of `rows` y rows
  const double* tab;    // [3][kLowMaxM][nmax] basis values
  const double* mu;     // [3][kLowMaxM] 1-D eigenvalues
  double* t2;           // [slabs][m0][m1][nz] partial (x, y) projections per plane
  double* e;            // [nz][m1][nx] coefficients back-transformed along x and z
};

// The pre-solve's tables and partial sums of one ensemble member.
__device__ inline LowArgs member_view(const SimConst& K, LowArgs L) {
  L.tab = mem(K, L.tab);
  L.mu = mem(K, L.mu);
  L.t2 = mem(K, L.t2);
  L.e = mem(K, L.e);
  return L;
}

// LDS of the projection pass (doubles): the x basis, a chunk of residual rows
// (padded stride nx + 1), the slab's x projections and its y basis rows.
__host__ __device__ inline int low_project_lds(const LowArgs& L, int nx) {
  return L.m[0] * nx + kLowChunk * (nx + 1) + L.m[0] * L.rows + L.m[1] * (L.rows + 1);
}
// LDS of the solve pass: summed projections [m0][nz] (reused for the x
// back-transform [m2][nx]), the z basis [m2][nz + 1], the scaled coefficients
// [m0][m2] and the x basis [m0][nx].
__host__ __device__ inline int low_solve_lds(const LowArgs& L, int nx, int nz) {
  const int a = L.m[0] * nz > L.m[2] * nx ? L.m[0] * nz : L.m[2] * nx;
  return a + L.m[2] * (nz + 1) + L.m[0] * L.m[2] + L.m[0] * nx;
}
// LDS of the correction pass: the plane's transformed coefficients [m1][nx]
// and the slab's y basis rows [m1][rows].
__host__ __device__ inline int low_correct_lds(const LowArgs& L, int nx) {
  return L.m[1] * nx + L.m[1] * L.rows;
}

// Slabs per z plane so that the plane passes run about kLowBlocks workgroups;
// `rows` receives the y rows per slab (the last slab may hold fewer).
inline int low_slabs(int ny, int nz, int& rows) {
  int s = std::max(1, std::min(ny, (kLowBlocks + nz - 1) / nz));
  rows = (ny + s - 1) / s;
  return (ny + rows - 1) / rows;
}

// 1-D basis function a at index i of an axis of n nodes: 1, then cos and sin
// of 2 pi k i / n for k = 1, 2, ...  (angle reduced exactly in integers).
__device__ inline double low_basis(int a, int i, int n) {
  if (a == 0) return 1.0;
  const int k = (a + 1) / 2;
  const double arg = (double)((2 * k * i) % (2 * n)) / (double)n;  // in units of pi
  return (a & 1) ? cospi(arg) : sinpi(arg);
}

// sum_{t < n} u[t * su] v[t * sv], in order of t.
__device__ inline double low_dot(const double* u, int su, const double* v, int sv, int n) {
  double acc = 0.0;
#pragma unroll 8
  for (int t = 0; t < n; ++t) acc += u[t * su] * v[t * sv];
  return acc;
}

__global__ void __launch_bounds__(kBlock) k_low_tables(SimConst K, LowArgs L, double* tab,
                                                       double* mu) {
  tab = mem(K, tab);
  mu = mem(K, mu);
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

// Pass 1, workgroup (slab s, plane k): the residual r_0 = -b - A x_0 on the
// slab's rows, projected on the x basis (t1[a][j] = sum_i r_0 phi_a(i)) and
// then on the y basis over the slab's rows:
//   t2[s][a][b][k] = sum_{j in slab} t1[a][j] phi_b(j).
__global__ void __launch_bounds__(kLowThreads) k_low_project(SimConst K, LowArgs L, const double* b,
                                                        const double* x) {
  L = member_view(K, L);
  b = mem(K, b);
  x = mem(K, x);
  extern __shared__ double lds[];
  const int nx = K.nc[0], ny = K.nc[1], nz = K.nc[2];
  const int m0 = L.m[0], m1 = L.m[1];
  const int s = blockIdx.x % L.slabs, k = blockIdx.x / L.slabs;
  const int j0 = s * L.rows, nr = min(L.rows, ny - j0);
  const int py = L.rows + 1;
  double* phx = lds;                        // [m0][nx]
  double* rr = phx + m0 * nx;               // [kLowChunk][nx + 1]
  double* t1 = rr + kLowChunk * (nx + 1);   // [m0][rows]
  double* phy = t1 + m0 * L.rows;           // [m1][rows + 1]
#pragma unroll 4
  for (int t = threadIdx.x; t < m0 * nx; t += kLowThreads)
    phx[t] = L.tab[(t / nx) * L.nmax + t % nx];
#pragma unroll 4
  for (int t = threadIdx.x; t < m1 * nr; t += kLowThreads)
    phy[(t / nr) * py + t % nr] = L.tab[(kLowMaxM + t / nr) * L.nmax + j0 + t % nr];
  for (int c0 = 0; c0 < nr; c0 += kLowChunk) {
    const int cr = min(kLowChunk, nr - c0);
    __syncthreads();  // the previous chunk's rows are consumed
    for (int t = threadIdx.x; t < cr * nx; t += kLowThreads) {
      const int i = t % nx, jj = t / nx, j = j0 + c0 + jj;
      const int n = lin(K, i, j, k);
      rr[jj * (nx + 1) + i] = -b[n] - neg_lap(K, i, j, k, [&](int m) { return x[m]; });
    }
    __syncthreads();
    for (int o = threadIdx.x; o < m0 * cr; o += kLowThreads) {
      const int a = o / cr, jj = o % cr;
      t1[a * L.rows + c0 + jj] = low_dot(rr + jj * (nx + 1), 1, phx + a * nx, 1, nx);
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < m0 * m1; o += kLowThreads) {
    const int a = o / m1, bb = o % m1;
    L.t2[(((int64_t)s * m0 + a) * m1 + bb) * nz + k] = low_dot(t1 + a * L.rows, 1, phy + bb * py, 1, nr);
  }
}

// Pass 2, workgroup b: the z projection of the slab sums,
//   c[a][b][c] = sum_k (sum_s t2[s][a][b][k]) phi_c(k),
// scaled by 1 / (eigenvalue * squared norm) (the constant mode is left alone),
// then the back-transforms along x and z:
//   d1[c][i] = sum_a c'[a][b][c] phi_a(i),  e[k][b][i] = sum_c phi_c(k) d1[c][i].
// Workgroup (bb, q): y mode bb, x columns [i0, i0 + ni) of chunk q of
// gridDim.y: the chunks of one mode repeat its small coefficient step, and the
// back-transforms (most of the LDS operand traffic) spread over more CUs.
__global__ void __launch_bounds__(kLowThreads) k_low_solve(SimConst K, LowArgs L) {
  L = member_view(K, L);
  extern __shared__ double lds[];
  const int nx = K.nc[0], nz = K.nc[2];
  const int m0 = L.m[0], m1 = L.m[1], m2 = L.m[2];
  const int bb = blockIdx.x;
  const int i0 = (int)(((int64_t)nx * blockIdx.y) / gridDim.y);
  const int ni = (int)(((int64_t)nx * (blockIdx.y + 1)) / gridDim.y) - i0;
  const int pz = nz + 1;
  double* u = lds;                 // [m0][nz], then d1 [m2][nx]
  double* phz = u + max(m0 * nz, m2 * nx);  // [m2][nz + 1]
  double* cf = phz + m2 * pz;      // [m0][m2]
  double* phx = cf + m0 * m2;      // [m0][ni]: columns i0 .. i0 + ni - 1
#pragma unroll 4
  for (int t = threadIdx.x; t < m0 * nz; t += kLowThreads) {
    const int a = t / nz, k = t % nz;
    double acc = 0.0;
    for (int s = 0; s < L.slabs; ++s) acc += L.t2[(((int64_t)s * m0 + a) * m1 + bb) * nz + k];
    u[t] = acc;
  }
#pragma unroll 4
  for (int t = threadIdx.x; t < m2 * nz; t += kLowThreads)
    phz[(t / nz) * pz + t % nz] = L.tab[(2 * kLowMaxM + t / nz) * L.nmax + t % nz];
#pragma unroll 4
  for (int t = threadIdx.x; t < m0 * ni; t += kLowThreads)
    phx[t] = L.tab[(t / ni) * L.nmax + i0 + t % ni];
  __syncthreads();
  for (int t = threadIdx.x; t < m0 * m2; t += kLowThreads) {
    const int a = t / m2, cc = t % m2;
    const double acc = low_dot(u + a * nz, 1, phz + cc * pz, 1, nz);
    const double ma = L.mu[a], mb = L.mu[kLowMaxM + bb], mc = L.mu[2 * kLowMaxM + cc];
    double lam = ma + mb + mc;
    if (K.poisson_op == 1) {  // Q1: mu_d times the 1-D mass eigenvalues 1 - mu h^2 / 6 of the others
      const double sa = 1.0 - ma / (6.0 * K.ih2[0]), sb = 1.0 - mb / (6.0 * K.ih2[1]),
                   sc = 1.0 - mc / (6.0 * K.ih2[2]);
      lam = ma * sb * sc + sa * mb * sc + sa * sb * mc;
    }
    const double nrm = (a ? 0.5 : 1.0) * (bb ? 0.5 : 1.0) * (cc ? 0.5 : 1.0) * (double)K.nn;
    cf[t] = lam > 0.0 ? acc / (lam * nrm) : 0.0;
  }
  __syncthreads();
  double* d1 = u;  // the projections are consumed; [m2][ni]
  for (int t = threadIdx.x; t < m2 * ni; t += kLowThreads) {
    const int cc = t / ni, i = t % ni;
    d1[t] = low_dot(cf + cc, m2, phx + i, ni, m0);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nz * ni; t += kLowThreads) {
    const int k = t / ni, i = t % ni;
    L.e[((int64_t)k * m1 + bb) * nx + i0 + i] = low_dot(phz + k, pz, d1 + i, ni, m2);
  }
}

// Pass 3, workgroup (slab s, plane k): x(i, j, k) += sum_b phi_b(j) e[k][b][i]
// on the slab's rows.
__global__ void __launch_bounds__(kLowThreads) k_low_correct(SimConst K, LowArgs L, double* x) {
  L = member_view(K, L);
  x = mem(K, x);
  extern __shared__ double lds[];
  const int nx = K.nc[0], ny = K.nc[1];
  const int m1 = L.m[1];
  const int s = blockIdx.x % L.slabs, k = blockIdx.x / L.slabs;
  const int j0 = s * L.rows, nr = min(L.rows, ny - j0);
  double* e = lds;                // [m1][nx]
  double* phy = e + m1 * nx;      // [rows][m1]
  const double* ek = L.e + (int64_t)k * m1 * nx;
#pragma unroll 4
  for (int t = threadIdx.x; t < m1 * nx; t += kLowThreads) e[t] = ek[t];
#pragma unroll 4
  for (int t = threadIdx.x; t < m1 * nr; t += kLowThreads)
    phy[(t % nr) * m1 + t / nr] = L.tab[(kLowMaxM + t / nr) * L.nmax + j0 + t % nr];
  __syncthreads();
  for (int t = threadIdx.x; t < nr * nx; t += kLowThreads) {
    const int i = t % nx, jj = t / nx;
    x[lin(K, i, j0 + jj, k)] += low_dot(phy + jj * m1, 1, e + i, nx, m1);
  }
}

}  // namespace pic
