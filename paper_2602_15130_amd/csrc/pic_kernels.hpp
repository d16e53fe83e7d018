// HIP kernels of the FP64 form of the step, plus the pieces shared with the
// mixed form (sort, scan, Poisson CG, gradient, norms).
#pragma once

#include "pic_device.hpp"

namespace pic {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// Cell-aligned particle tiles of the sort and the fused particle pass.
#ifndef PIC_TILE_B
#define PIC_TILE_B 256
#endif
#ifndef PIC_TILE_THREADS
#define PIC_TILE_THREADS 256
#endif
constexpr int kTileB = PIC_TILE_B;               // particle slots that start cells in one tile
constexpr int kTileThreads = PIC_TILE_THREADS;   // threads of the tile kernels
#ifndef PIC_LDS_SLOTS
#define PIC_LDS_SLOTS (PIC_TILE_B + PIC_TILE_B / 4)
#endif
constexpr int kLdsSlots = PIC_LDS_SLOTS;          // LDS-resident slots per tile
// Minimum resident waves per SIMD requested for the fused particle kernels
// (their register budget is 512 / waves per lane).
#ifndef PIC_MIXED_WAVES
#define PIC_MIXED_WAVES 6
#endif
#ifndef PIC_F64_WAVES
#define PIC_F64_WAVES 4  // also the LDS limit: four 33 KB tiles per CU
#endif
// The same for the lean instances (smaller: no general collision path).
#ifndef PIC_MIXED_LEAN_WAVES
#define PIC_MIXED_LEAN_WAVES 6
#endif
#ifndef PIC_F64_LEAN_WAVES
#define PIC_F64_LEAN_WAVES 4
#endif

// Flags raised by kernels and read back at the next synchronising call.
enum { kFlagCgNoConv = 0, kFlagBarrier = 1, kFlagNonFinite = 2, kFlagCapacity = 3, kFlagCount = 4 };
// Work bounds that keep every kernel finite on degenerate input (a run-away
// state collapsing into one cell): candidate pairs per outcome, and the cell
// size for the in-cell stable rank.  Exceeding them raises kFlagCapacity.
constexpr int64_t kMaxPairsPerOutcome = int64_t(1) << 22;
constexpr int kMaxStableCell = 1 << 16;
// 64-bit counters: accepted collisions, candidate pairs with g > g_max, pair-log records.
enum { kCntAccepted = 0, kCntGmax = 1, kCntPairLog = 2, kCntAngles = 3, kCntCount = 4 };

// ---------------------------------------------------------------------------
// Block reductions with a fixed combination order (bitwise reproducible).
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Sum over a block of NT threads (sh holds NT / 64 values); every thread
// receives the same value.
template <int NT>
__device__ inline double block_sum_t(double v, double* sh) {
  v = wave_sum(v);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  __syncthreads();
  if (ln == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) r += sh[i];
  return r;
}
__device__ inline double block_sum(double v, double* sh) { return block_sum_t<kBlock>(v, sh); }
// block_sum_t of nv <= 3 values at once (one barrier pair for all of them;
// each value summed in the same order as block_sum_t).  sh: 3 * NT / 64 doubles.
template <int NT>
__device__ inline void block_sum3_t(double* v, int nv, double* sh) {
  constexpr int W = NT / 64;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  double w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = i < nv ? wave_sum(v[i]) : 0.0;
  __syncthreads();
  if (ln == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (i < nv) sh[i * W + wv] = w[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i >= nv) break;
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) r += sh[i * W + k];
    v[i] = r;
  }
}
__device__ inline double block_max(double v, double* sh) {
  v = wave_max(v);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  __syncthreads();
  if (ln == 0) sh[wv] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) r = fmax(r, sh[i]);
  return r;
}

// ---------------------------------------------------------------------------
// Fill kernels (used instead of hipMemsetAsync so that steps stay graph-safe).
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T* p, T v, int64_t n, int64_t mstride) {
  p = mem_z(mstride, p);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Mesh indexing: node / cell (i, j, k) -> (k ny + j) nx + i, periodic.
// ---------------------------------------------------------------------------
__device__ inline int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ inline int lin(const SimConst& K, int i, int j, int k) {
  return (wrapi(k, K.nc[2]) * K.nc[1] + wrapi(j, K.nc[1])) * K.nc[0] + wrapi(i, K.nc[0]);
}

// Cell and in-cell offset (cell units) of a position in [0, L).
__device__ inline void locate(const SimConst& K, const double x[3], int c[3], double o[3]) {
  for (int d = 0; d < 3; ++d) {
    double s = x[d] * K.inv_h[d];
    int i = (int)floor(s);
    i = i < 0 ? 0 : (i > K.nc[d] - 1 ? K.nc[d] - 1 : i);
    c[d] = i;
    o[d] = s - (double)i;
  }
}

// ---------------------------------------------------------------------------
// Stable counting sort by cell.
//   count:   slot[i] = position of particle i among its cell's arrivals, taken
//            with one atomic per (wave, key) group (ballot match);
//   scan:    cell_start = exclusive prefix sum of the counts;
//   scatter: tmp_idx[cell_start[key] + slot] = i;
//   order:   inside each cell, rank the source indices, which restores the
//            input order (stability) independently of atomic arrival order,
//            and gather the particle state into the destination arrays.
// ---------------------------------------------------------------------------
// Arrival slot of each valid lane in its cell: the wave's lanes are grouped by
// key with ballots and shuffles first (no memory traffic), then every group's
// first lane adds the group's size to the cell count -- all groups' atomics in
// one instruction, so the wave waits for one round trip, not one per cell --
// and each lane takes its group's base plus its rank among the group's lanes.
__device__ inline int wave_aggregated_slot(int* count, int key, bool valid) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(valid);
  int leader_of_mine = lane, rank = 0, total = 0;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int lkey = __shfl(key, leader);
    const bool mine = valid && key == lkey && ((pending >> lane) & 1ull);
    const unsigned long long grp = __ballot(mine);
    if (mine) {
      leader_of_mine = leader;
      rank = __popcll(grp & ((1ull << lane) - 1ull));
    }
    if (lane == leader) total = __popcll(grp);
    pending &= ~grp;
  }
  int base = 0;
  if (valid && lane == leader_of_mine) base = atomicAdd(&count[key], total);
  base = __shfl(base, leader_of_mine);
  return valid ? base + rank : 0;
}

__global__ void __launch_bounds__(kBlock) k_count(const int* key, int* slot, int* count, int n) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  bool valid = i < n;
  int k = valid ? key[i] : 0;
  int s = wave_aggregated_slot(count, k, valid);
  if (valid) slot[i] = s;
}

// Exclusive scan of n ints in three passes; 1024 items per block.
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

// Tile tables of the sort, filled before the third pass writes their bounds.
struct TileInit {
  int* c0;     // first cell per tile, filled with the cell count
  int* s0;     // first particle per tile, filled with the particle count
  int ntiles;  // entries 0..ntiles
  int ncell, np;
};

// Pass 1: per-block exclusive scans and block totals; also fills the tile tables.
__global__ void __launch_bounds__(kBlock) k_scan_local(const int* in, int* out, int* bsum, int n,
                                                       TileInit ti, int64_t mstride) {
  in = mem_z(mstride, in);
  out = mem_z(mstride, out);
  bsum = mem_z(mstride, bsum);
  ti.c0 = mem_z(mstride, ti.c0);
  ti.s0 = mem_z(mstride, ti.s0);
  for (int t = blockIdx.x * kBlock + threadIdx.x; t <= ti.ntiles; t += gridDim.x * kBlock) {
    ti.c0[t] = ti.ncell;
    ti.s0[t] = ti.np;
  }
  __shared__ int sh[kBlock];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems], tot = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    tot += v[j];
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {  // Hillis-Steele inclusive scan
    int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - tot;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = sh[kBlock - 1];
}

// One block scans the block totals; writes the grand total to out[n].
__global__ void __launch_bounds__(kBlock) k_scan_blocks(int* bsum, int nb, int* out, int n,
                                                        int64_t mstride) {
  bsum = mem_z(mstride, bsum);
  out = mem_z(mstride, out);
  __shared__ int sh[kBlock];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int start = 0; start < nb; start += kBlock) {
    int i = start + threadIdx.x;
    int v = i < nb ? bsum[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    int excl = carry + sh[threadIdx.x] - v;
    if (i < nb) bsum[i] = excl;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry += sh[kBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// Pass 3: adds the block prefixes, giving the cell starts; resets the counts
// to zero for the next counting pass; and writes the bounds of the cell-aligned
// tiles, tile_c0[t] = min{c : cstart[c] >= t kTileB} and tile_s0[t] =
// cstart[tile_c0[t]]: with lo = cstart[j] and hi = cstart[j + 1] = lo + count[j],
// cell c = j + 1 is that minimum for every t with lo < t kTileB <= hi.  Tile 0
// starts at cell 0; tiles past the end keep the fill of pass 1.
__global__ void __launch_bounds__(kBlock) k_scan_add(int* out, const int* bsum, int n, int* count,
                                                     TileInit ti, int64_t mstride) {
  out = mem_z(mstride, out);
  bsum = mem_z(mstride, bsum);
  count = mem_z(mstride, count);
  ti.c0 = mem_z(mstride, ti.c0);
  ti.s0 = mem_z(mstride, ti.s0);
  int base = blockIdx.x * kScanTile;
  int add = bsum[blockIdx.x];
  for (int j = threadIdx.x; j < kScanTile; j += kBlock) {
    const int jj = base + j;
    if (jj >= n) continue;
    const int lo = out[jj] + add, hi = lo + count[jj];
    out[jj] = lo;
    count[jj] = 0;
    for (int t = lo / kTileB + 1; t * kTileB <= hi && t <= ti.ntiles; ++t) {
      ti.c0[t] = jj + 1;
      ti.s0[t] = hi;
    }
    if (jj == 0) {
      ti.c0[0] = 0;
      ti.s0[0] = 0;
    }
  }
}

// Scatter slot of every particle: cell start + its slot in the cell;
// kScatterPer particles per thread, loads issued before the dependent ones.
constexpr int kScatterPer = 4;
__global__ void __launch_bounds__(kBlock) k_scatter(const int* key, const int* slot,
                                                    const int* cstart, int* tidx, int* tkey,
                                                    int n, int64_t mstride) {
  key = mem_z(mstride, key);
  slot = mem_z(mstride, slot);
  cstart = mem_z(mstride, cstart);
  tidx = mem_z(mstride, tidx);
  tkey = mem_z(mstride, tkey);
  const int base = blockIdx.x * (kBlock * kScatterPer) + threadIdx.x;
  int k[kScatterPer], sl[kScatterPer];
#pragma unroll
  for (int q = 0; q < kScatterPer; ++q) {
    const int i = base + q * kBlock;
    if (i < n) {
      k[q] = key[i];
      sl[q] = slot[i];
    }
  }
#pragma unroll
  for (int q = 0; q < kScatterPer; ++q) {
    const int i = base + q * kBlock;
    if (i < n) {
      const int dst = cstart[k[q]] + sl[q];
      tidx[dst] = i;
      tkey[dst] = k[q];
    }
  }
}

// Rank of `my` among the source indices of its cell segment.
__device__ inline int stable_rank(const int* tidx, int s, int e, int my) {
  int r = 0;
  for (int k = s; k < e; ++k) r += tidx[k] < my;
  return r;
}

// Destination of scatter slot j: its stable rank inside its cell, or (for a
// cell beyond kMaxStableCell, flagged as a capacity error) the slot itself.
__device__ inline int order_dst(const int* tidx, const int* tkey, const int* cstart, int j,
                                int* flags) {
  int c = tkey[j], s = cstart[c], e = cstart[c + 1];
  if (e - s > kMaxStableCell) {
    atomicOr(&flags[kFlagCapacity], 1);
    return j;
  }
  return s + stable_rank(tidx, s, e, tidx[j]);
}

// ---------------------------------------------------------------------------
// Initial state: xi -> x^M(0), v^M(0) in id order (eq. mms_sol), cell keys and
// counts for the sort.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_init_f64(SimConst K, double* x, double* v, double* ash,
                                                     int* id, int* key, int* slot, int* count) {
  x = mem(K, x);
  v = mem(K, v);
  ash = mem(K, ash);
  id = mem(K, id);
  key = mem(K, key);
  slot = mem(K, slot);
  count = mem(K, count);
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  bool valid = p < K.np;
  int kk = 0;
  if (valid) {
    double xi[6], xm[3], a[3], vm[3], vd[3];
    init_uniforms(K, p, xi);
    manufactured_position(K, xi, 0.0, nullptr, xm);
    velocity_shape(K, xi + 3, a);
    manufactured_velocity(K, a, 0.0, vm, vd);
    int c[3];
    double o[3];
    locate(K, xm, c, o);
    kk = lin(K, c[0], c[1], c[2]);
    for (int d = 0; d < 3; ++d) {
      x[d * K.np + p] = xm[d];
      v[d * K.np + p] = vm[d];
      ash[d * K.np + p] = a[d];  // time-independent velocity shape, v^M = vhat(t) a
    }
    id[p] = (int)p;
    key[p] = kk;
  }
  int s = wave_aggregated_slot(count, kk, valid);
  if (valid) slot[p] = s;
}

// Positions given by the caller (component-major FP64): wrapped into [0, L)
// (a non-finite coordinate becomes 0 and raises the non-finite flag), with the
// cell keys and arrival slots of the stable sort that follows.
__device__ inline double wrap_box(double x, double L, bool& bad) {
  double w = x - floor(x / L) * L;
  if (!(w >= 0.0 && w < L)) {  // rounded up to L, or non-finite
    bad |= !isfinite(x);
    w = 0.0;
  }
  return w;
}

__global__ void __launch_bounds__(kBlock) k_set_positions_f64(SimConst K, const double* xin,
                                                              double* x, int* key, int* slot,
                                                              int* count, int* flags) {
  int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  bool valid = p < K.np;
  int kk = 0;
  if (valid) {
    bool bad = false;
    double xp[3];
    for (int d = 0; d < 3; ++d) {
      xp[d] = wrap_box(xin[d * K.np + p], K.L[d], bad);
      x[d * K.np + p] = xp[d];
    }
    if (bad) atomicOr(&flags[kFlagNonFinite], 1);
    int c[3];
    double o[3];
    locate(K, xp, c, o);
    kk = lin(K, c[0], c[1], c[2]);
    key[p] = kk;
  }
  int s = wave_aggregated_slot(count, kk, valid);
  if (valid) slot[p] = s;
}

// ---------------------------------------------------------------------------
// Charge deposition (Sec. 2, cloud in cell), atomic free: each cell sums the
// eight corner weights of its own particles in cell-sorted order, then each
// node adds the eight cell moments that touch it in a fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_deposit_moments_f64(SimConst K, const double* x,
                                                                const int* cstart, double* mom) {
  int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= K.nn) return;
  double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = cstart[c]; j < cstart[c + 1]; ++j) {
    double xp[3] = {x[j], x[K.np + j], x[2 * K.np + j]};
    int ci[3];
    double o[3];
    locate(K, xp, ci, o);
    double wx[2] = {1.0 - o[0], o[0]}, wy[2] = {1.0 - o[1], o[1]}, wz[2] = {1.0 - o[2], o[2]};
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) m[cz * 4 + cy * 2 + cx] += wx[cx] * wy[cy] * wz[cz];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) mom[(int64_t)k * K.nn + c] = m[k];
}

// Node (= cell) index n = i + nc0 (j + nc1 k) split into its coordinates.
__device__ inline void node_coords(const SimConst& K, int n, int& i, int& j, int& k) {
  const int a = (int)div_by(K.div_x, (uint32_t)n);   // j + nc1 k
  const int b = (int)div_by(K.div_xy, (uint32_t)n);  // k
  i = n - a * K.nc[0];
  j = a - b * K.nc[1];
  k = b;
}

// Manufactured part of eq. poisson_mms at node (i, j, k): m = lap phi^M, plus
// q f_x / eps0 when the particles feed the field; pointwise for the 7-point
// operator, through the Q1 mass weights (1, 4, 1) / 6 per axis (the consistent
// mass matrix over the cell volume) for trilinear elements.
__device__ inline double rhs_manufactured(const SimConst& K, int i, int j, int k, double t) {
  auto m_at = [&](int ii, int jj, int kk) {
    const double xn[3] = {ii * K.h[0], jj * K.h[1], kk * K.h[2]};
    double v = lap_phiM(K, xn, t);
    if (K.p2f != 0.0) v += K.q * number_density(K, xn, t) / K.eps0;
    return v;
  };
  if (K.poisson_op != 1) return m_at(i, j, k);
  const double w1[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
  double v = 0.0;
  for (int c = -1; c <= 1; ++c)
    for (int bb = -1; bb <= 1; ++bb)
      for (int a = -1; a <= 1; ++a)
        v += w1[a + 1] * w1[bb + 1] * w1[c + 1] *
             m_at(wrapi(i + a, K.nc[0]), wrapi(j + bb, K.nc[1]), wrapi(k + c, K.nc[2]));
  return v;
}

// Node charge and the right-hand side of eq. poisson_mms; block partial sums
// of b for the mean removal.
template <class MomT>
__global__ void __launch_bounds__(kBlock) k_node_rhs(SimConst K, const MomT* mom, double t,
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
        for (int cx = 0; cx < 2; ++cx)
          s += (double)mom[(int64_t)(cz * 4 + cy * 2 + cx) * K.nn + lin(K, i - cx, j - cy, k - cz)];
    double r = K.rho_scale * s;
    rho[n] = r;
    bv = rhs_manufactured(K, i, j, k, t);
    if (K.p2f != 0.0) bv -= r / K.eps0;
    b[n] = bv;
  }
  double tot = block_sum(bv, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Removes the mean of b; also zeroes the Poisson solver's barrier words
// (nbar of them), which must read zero when the solver starts.
__global__ void __launch_bounds__(kBlock) k_sub_mean(SimConst K, double* b, const double* part,
                                                     int nparts, unsigned* bar, int nbar) {
  b = mem(K, b);
  part = mem(K, part);
  bar = mem(K, bar);
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < nbar; t += gridDim.x * kBlock) bar[t] = 0u;
  __shared__ double sh[kWaves];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) acc += part[i];
  double mean = block_sum(acc, sh) / (double)K.nn;
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n < K.nn) b[n] -= mean;
}

// ---------------------------------------------------------------------------
// Poisson CG: one cooperative persistent kernel.  A = -L_h (periodic 7-point),
// A phi = -b, in the single-reduction recurrence of Chronopoulos and Gear:
// the operator acts on the residual (w = A r), s = A p follows its own
// recurrence, and gamma = r.r and delta = w.r are reduced together, so an
// iteration has ONE grid-wide reduction.  The pointwise updates of iteration i
// (p, s, x, r) and the stencil w_{i+1} = A r_{i+1} share one sweep: the
// stencil rebuilds r_{i+1} at the six neighbours from r_i, w_i and s_{i-1},
// which were all published before the reduction, with the same expression the
// neighbour's owner evaluates (ping-pong buffers for r, w and s).  The
// reduction is also the grid barrier: every block publishes its partial sums
// and then a flag (one release store); block 0 waits for all flags, sums the
// partials in block order and publishes the result and a release word; every
// block waits on that word.  Waits poll with relaxed loads and take one
// acquire fence at the end; they are bounded and raise kFlagBarrier on
// timeout so every wave always leaves the kernel.
// ---------------------------------------------------------------------------
constexpr int kFlagStride = 32;  // 128 bytes between per-block flags
constexpr int kMaxRed = 3;       // values per reduction
static_assert(kMaxRed == 3, "block_sum3_t reduces up to three values");

struct CgArgs {
  const double* b;
  double* x;
  double* r[2];       // residual, ping-pong
  double* w[2];       // A r, ping-pong
  double* s[2];       // A p, ping-pong
  double* p;          // search direction
  double* part;       // [grid][kMaxRed]
  double* result;     // [kMaxRed]
  unsigned* arrive;   // [grid * kFlagStride], zero before launch
  unsigned* release;  // [1], zero before launch
  int* flags;
  int* iters_out;
  double* relres_out;
  double tol;
  int max_iter;
  double* pub;        // brick solver: published faces, [bricks][2][3][nh]
  int bdim[3];        // brick solver: nodes per brick along each axis
  int nbr[3];         // brick solver: bricks along each axis
};

__device__ inline bool spin_until(const unsigned* addr, unsigned want, int* flags) {
  unsigned spins = 0;
  while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > (1u << 24)) {
      atomicOr(&flags[kFlagBarrier], 1);
      return false;
    }
    if ((spins & 1023u) == 0 &&
        __hip_atomic_load(&flags[kFlagBarrier], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
  }
  return true;
}

// The solver's arrays of one ensemble member.
__device__ inline CgArgs member_view(const SimConst& K, CgArgs a) {
  a.b = mem(K, a.b);
  a.x = mem(K, a.x);
  for (int i = 0; i < 2; ++i) {
    a.r[i] = mem(K, a.r[i]);
    a.w[i] = mem(K, a.w[i]);
    a.s[i] = mem(K, a.s[i]);
  }
  a.p = mem(K, a.p);
  a.part = mem(K, a.part);
  a.result = mem(K, a.result);
  a.arrive = mem(K, a.arrive);
  a.release = mem(K, a.release);
  a.flags = mem(K, a.flags);
  a.iters_out = mem(K, a.iters_out);
  a.relres_out = mem(K, a.relres_out);
  a.pub = mem(K, a.pub);
  return a;
}

// Waits until this wave's outstanding vector-memory operations have completed
// (device code only: a host build of these headers has no such queue).
__device__ inline void wait_vector_memory() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#endif
}

// Grid-wide sum of nv block values; every thread of every block (NT threads
// each) gets the same nv results.  `gen` increases by one per call within a
// launch.
template <int NT>
__device__ inline bool grid_sum_t(const CgArgs& a, double* vals, int nv, unsigned gen, double* sh) {
  __shared__ int ok;
  __shared__ double res[kMaxRed];
  double tot[kMaxRed];
  if (gridDim.x == 1) {
    // One workgroup per solve: the block sum is the grid sum (the value the
    // flag protocol below would return, plus exact zeros); the workgroup
    // barrier inside it, after every wave's stores have completed, is the
    // ordering the solver's sweeps and face exchange need.
    wait_vector_memory();
    block_sum3_t<NT>(vals, nv, sh);
    // (as after the flag protocol: later plain loads must not hit lines of
    // this CU's cache that other waves' stores have made stale)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
  }
  // Every wave waits until its own global stores have reached L2 before the
  // block barrier; thread 0's agent-scope release below then writes back L2
  // and so publishes the whole block's stores with its flag.  (A workgroup
  // barrier alone does not wait for outstanding vector-memory stores.)
  wait_vector_memory();
  for (int i = 0; i < nv; ++i) tot[i] = vals[i];
  block_sum3_t<NT>(tot, nv, sh);
  if (threadIdx.x == 0) {
    for (int i = 0; i < nv; ++i) a.part[blockIdx.x * kMaxRed + i] = tot[i];
    __hip_atomic_store(&a.arrive[blockIdx.x * kFlagStride], gen, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
    ok = 1;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    int good = 1;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += NT)
      if (!spin_until(&a.arrive[b * kFlagStride], gen, a.flags)) good = 0;
    if (!good) ok = 0;
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double acc[kMaxRed] = {0.0, 0.0, 0.0};
    for (int i = 0; i < nv; ++i)
      for (int b = threadIdx.x; b < (int)gridDim.x; b += NT) acc[i] += a.part[b * kMaxRed + i];
    block_sum3_t<NT>(acc, nv, sh);
    if (threadIdx.x == 0)
      for (int i = 0; i < nv; ++i) a.result[i] = acc[i];
    if (threadIdx.x == 0)
      __hip_atomic_store(a.release, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0) {
    if (!spin_until(a.release, gen, a.flags)) ok = 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int i = 0; i < nv; ++i) res[i] = a.result[i];
  }
  __syncthreads();
  for (int i = 0; i < nv; ++i) vals[i] = res[i];
  return ok != 0;
}
__device__ inline bool grid_sum(const CgArgs& a, double* vals, int nv, unsigned gen, double* sh) {
  return grid_sum_t<kBlock>(a, vals, nv, gen, sh);
}

// (-L f)(n) for f given by a callable.  7-point: minus the summed second
// differences.  Trilinear elements (Sec. 4.2): the stiffness over the cell
// volume, 27 points: along each axis d the second difference in d times the
// 1-D mass weights (1, 4, 1) / 6 in the two other axes, summed over d.
template <class F>
__device__ inline double neg_lap(const SimConst& K, int i, int j, int k, const F& f) {
  if (K.poisson_op == 1) {
    const double w1[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    const double d2[3] = {1.0, -2.0, 1.0};
    double v = 0.0;
#pragma unroll
    for (int c = -1; c <= 1; ++c)
#pragma unroll
      for (int bb = -1; bb <= 1; ++bb)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
          const double wx = d2[a + 1] * K.ih2[0] * w1[bb + 1] * w1[c + 1];
          const double wy = w1[a + 1] * d2[bb + 1] * K.ih2[1] * w1[c + 1];
          const double wz = w1[a + 1] * w1[bb + 1] * d2[c + 1] * K.ih2[2];
          v += (wx + wy + wz) * f(lin(K, i + a, j + bb, k + c));
        }
    return -v;
  }
  double c = f(lin(K, i, j, k));
  double lx = f(lin(K, i + 1, j, k)) - 2.0 * c + f(lin(K, i - 1, j, k));
  double ly = f(lin(K, i, j + 1, k)) - 2.0 * c + f(lin(K, i, j - 1, k));
  double lz = f(lin(K, i, j, k + 1)) - 2.0 * c + f(lin(K, i, j, k - 1));
  return -(lx * K.ih2[0] + ly * K.ih2[1] + lz * K.ih2[2]);
}

__global__ void __launch_bounds__(kBlock) k_cg(SimConst K, CgArgs a) {
  a = member_view(K, a);
  __shared__ double sh[3 * kWaves];
  const int gsize = gridDim.x * kBlock;
  const int g0 = blockIdx.x * kBlock + threadIdx.x;
  unsigned gen = 0;
  // r_0 = -b - A x_0; gamma_0 = r_0.r_0 and ||b||^2
  double v2[kMaxRed] = {0.0, 0.0, 0.0};
  for (int n = g0; n < K.nn; n += gsize) {
    int i, j, k;
    node_coords(K, n, i, j, k);
    double ax = neg_lap(K, i, j, k, [&](int m) { return a.x[m]; });
    double rv = -a.b[n] - ax;
    a.r[0][n] = rv;
    v2[0] += rv * rv;
    v2[1] += a.b[n] * a.b[n];
  }
  if (!grid_sum(a, v2, 2, ++gen, sh)) return;
  double gamma = v2[0];
  const double bnorm = sqrt(v2[1]);
  int it = 0;
  if (bnorm == 0.0) {
    for (int n = g0; n < K.nn; n += gsize) a.x[n] = 0.0;
    gamma = 0.0;
  } else if (sqrt(gamma) > a.tol * bnorm) {
    // w_0 = A r_0, delta_0 = w_0.r_0
    double v1[kMaxRed] = {0.0, 0.0, 0.0};
    for (int n = g0; n < K.nn; n += gsize) {
      int i, j, k;
      node_coords(K, n, i, j, k);
      double wv = neg_lap(K, i, j, k, [&](int m) { return a.r[0][m]; });
      a.w[0][n] = wv;
      v1[0] += wv * a.r[0][n];
    }
    if (!grid_sum(a, v1, 1, ++gen, sh)) return;
    double alpha = gamma / v1[0], beta = 0.0;
    int cur = 0;
    while (true) {
      if (it >= a.max_iter) {
        if (g0 == 0) atomicOr(&a.flags[kFlagCgNoConv], 1);
        break;
      }
      const double* rc = a.r[cur];
      const double* wc = a.w[cur];
      const double* sc = a.s[cur];
      double* rn = a.r[cur ^ 1];
      double* wn = a.w[cur ^ 1];
      double* sn = a.s[cur ^ 1];
      const bool first = it == 0;  // p_{-1} = s_{-1} = 0: never read
      // r_{i+1} at any node, exactly as its owner computes it below
      auto rnext = [&](int m) {
        double sv = first ? wc[m] : wc[m] + beta * sc[m];
        return rc[m] - alpha * sv;
      };
      double gd[kMaxRed] = {0.0, 0.0, 0.0};
      for (int n = g0; n < K.nn; n += gsize) {
        int i, j, k;
        node_coords(K, n, i, j, k);
        double pv = first ? rc[n] : rc[n] + beta * a.p[n];
        double sv = first ? wc[n] : wc[n] + beta * sc[n];
        a.p[n] = pv;
        sn[n] = sv;
        a.x[n] += alpha * pv;
        double rv = rc[n] - alpha * sv;
        rn[n] = rv;
        double wv = neg_lap(K, i, j, k, rnext);
        wn[n] = wv;
        gd[0] += rv * rv;
        gd[1] += wv * rv;
      }
      if (!grid_sum(a, gd, 2, ++gen, sh)) return;
      cur ^= 1;
      ++it;
      beta = gd[0] / gamma;
      alpha = gd[0] / (gd[1] - beta * gd[0] / alpha);
      gamma = gd[0];
      if (sqrt(gamma) <= a.tol * bnorm) break;
    }
  }
  // zero-mean projection (Sec. 2)
  double s_x[kMaxRed] = {0.0, 0.0, 0.0};
  for (int n = g0; n < K.nn; n += gsize) s_x[0] += a.x[n];
  if (!grid_sum(a, s_x, 1, ++gen, sh)) return;
  double mean = s_x[0] / (double)K.nn;
  for (int n = g0; n < K.nn; n += gsize) a.x[n] -= mean;
  if (g0 == 0) {
    *a.iters_out = it;
    *a.relres_out = bnorm == 0.0 ? 0.0 : sqrt(gamma) / bnorm;
  }
}

// E = -grad phi, central differences; optional FP32 copy for the mixed form.
__global__ void __launch_bounds__(kBlock) k_gradient(SimConst K, const double* phi, double* E,
                                                     float* E32) {
  phi = mem(K, phi);
  E = mem(K, E);
  E32 = mem(K, E32);
  int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= K.nn) return;
  int i, j, k;
  node_coords(K, n, i, j, k);
  double ex = -(phi[lin(K, i + 1, j, k)] - phi[lin(K, i - 1, j, k)]) / (2.0 * K.h[0]);
  double ey = -(phi[lin(K, i, j + 1, k)] - phi[lin(K, i, j - 1, k)]) / (2.0 * K.h[1]);
  double ez = -(phi[lin(K, i, j, k + 1)] - phi[lin(K, i, j, k - 1)]) / (2.0 * K.h[2]);
  E[n] = ex;
  E[K.nn + n] = ey;
  E[2 * K.nn + n] = ez;
  if (E32) {
    E32[3 * n] = (float)ex;
    E32[3 * n + 1] = (float)ey;
    E32[3 * n + 2] = (float)ez;
  }
}

// ---------------------------------------------------------------------------
// Collisions, FP64: Algorithm 1 on each cell, N_avg independent outcomes from
// the same pre-collision velocities, averaged in increasing outcome order
// (eq. avg_outcome).  One thread per cell; the private velocity copy of an
// outcome lives in `u` at the cell's own particle slots.
// ---------------------------------------------------------------------------
// Scattering angles of an accepted collision recovered from the post-collision
// relative velocity g' = v_p' - v_q' with the pre-collision speed g
// (eq. angle_recovery): chi = acos(g'_z / g), eps = atan2(g'_y, g'_x) in
// [0, 2 pi).  Appended to `log` (chi, eps pairs) while it has room; the
// counter keeps counting past the capacity.
template <class R>
__device__ inline void record_angles(const R up[3], const R uq[3], R g, double* log, int64_t cap,
                                     unsigned long long* counters) {
  if (!log) return;
  double gx = (double)(up[0] - uq[0]), gy = (double)(up[1] - uq[1]), gz = (double)(up[2] - uq[2]);
  double cz = gz / (double)g;
  cz = fmin(1.0, fmax(-1.0, cz));
  double chi = acos(cz), eps = atan2(gy, gx);
  if (eps < 0.0) eps += 2.0 * kPi;
  unsigned long long s = atomicAdd(&counters[kCntAngles], 1ull);
  if ((int64_t)s < cap) {
    log[2 * s] = chi;
    log[2 * s + 1] = eps;
  }
}

__device__ inline uint64_t redraw_word(const SimConst& K, int cell, int64_t step, int call, int k,
                                       int64_t m, const U64x4& wb, int r) {
  if (r < 3) return wb.w[1 + r];
  int64_t j = (r - 3) / 4;
  U64x4 b = stream_block(K, (uint64_t)cell, (uint64_t)step, kTagRedraw, (uint64_t)call,
                         (uint64_t)k, ((uint64_t)m << 16) | (uint64_t)j);
  return b.w[(r - 3) % 4];
}

// Candidate partner q != p: Algorithm 1 redraws q while it equals p.
__device__ inline int pick_partner(const SimConst& K, int cell, int64_t step, int call, int k,
                                   int64_t m, const U64x4& wa, const U64x4& wb, int p, int n) {
  int q = index_below(wa.w[1], n);
  int r = 0;
  while (q == p) {
    if (r >= 3 + 4 * 65536) {
      q = (p + 1) % n;
      break;
    }
    q = index_below(redraw_word(K, cell, step, call, k, m, wb, r), n);
    ++r;
  }
  return q;
}

// cos chi = cos F_pchi^{-1}(xi) of the polar-angle model, in the working
// precision R:
//   isotropic, eq. chi_iso: 1 - 2 xi;
//   manufactured anisotropy (Sec. 5.2), eq. fpiv_ms: u = sin^2(chi/2) from the
//     closed-form a(xi), b(xi); cos chi = 1 - 2 u;
//   variable soft sphere, eq. vss: cos(chi/2) = (1 - xi)^(1/(2 alpha)), the
//     exact inverse of F = 1 - cos^(2 alpha)(chi/2); cos chi = 2 (1 - xi)^(1/alpha) - 1.
// ANY = false compiles the isotropic law alone (the fused kernels' lean
// instances, launched only for isotropic scattering).
template <class R, bool ANY = true>
__device__ inline R cos_chi(const SimConst& K, R xi) {
  if constexpr (!ANY) return (R)1.0 - (R)2.0 * xi;
  if (K.chi_model == 1) {
    const R inner = (R)298924665.0 +
                    (R)55680.0 * xi * ((R)376377.0 + (R)2320.0 * xi * ((R)-429.0 + (R)290.0 * xi));
    const R a = cbrt((R)81909.0 - (R)83520.0 * xi + sqrt(inner)) / ((R)40.0 * cbrt((R)9.0));
    const R b = (R)0.2 + a + ((R)161.0 - (R)290.0 * xi) / ((R)600.0 * a);
    const R sb = sqrt(b);
    const R u = (R)0.5 * ((R)1.0 - sb + sqrt((R)0.6 - b + (R)29.0 / ((R)40.0 * sb)));
    return (R)1.0 - (R)2.0 * u;
  }
  if (K.chi_model == 2) return (R)2.0 * pow((R)1.0 - xi, (R)1.0 / (R)K.chi_alpha) - (R)1.0;
  return (R)1.0 - (R)2.0 * xi;
}

// Post-collision velocities of an accepted pair: v_cm +- g n / 2 (Algorithm 1).
// The full instances also carry the deliberate coding errors of Sec. 5.4.1
// for verification studies: Error 1 takes v_cm = (v_p - v_q) / 2; Error 2
// swaps the two velocities when U_chi < 1/2 and leaves them unchanged
// otherwise.
template <class R, bool FULL>
__device__ inline void post_collision(const SimConst& K, const R up[3], const R uq[3], R g,
                                      const R nv[3], R uchi, R pn[3], R qn[3]) {
  if (FULL && K.coding_error == 2) {
    const bool swap = uchi < (R)0.5;
    for (int d = 0; d < 3; ++d) {
      pn[d] = swap ? uq[d] : up[d];
      qn[d] = swap ? up[d] : uq[d];
    }
    return;
  }
  for (int d = 0; d < 3; ++d) {
    const R vcm = (FULL && K.coding_error == 1) ? (R)0.5 * (up[d] - uq[d]) : (R)0.5 * (up[d] + uq[d]);
    pn[d] = vcm + (R)0.5 * g * nv[d];
    qn[d] = vcm - (R)0.5 * g * nv[d];
  }
}

// Capacity of the workgroup-per-cell collision kernel (k_collide_heavy):
// particles per cell and candidate pairs per outcome.  A cell that could
// exceed either (N_pairs = floor(n (n - 1) P_max / 2 + U) < n (n - 1) P_max / 2 + 1)
// is a "big" cell; in the collision-heavy mode it runs in k_collide_big instead.
constexpr int kHeavyMaxN = 2048;
constexpr int kHeavyMaxPairs = 192;
__device__ inline bool heavy_big_cell(const SimConst& K, int n) {
  return n > kHeavyMaxN ||
         (double)n * (double)(n - 1) * K.pmax / 2.0 + 1.0 >= (double)(kHeavyMaxPairs + 1);
}

__global__ void __launch_bounds__(kBlock) k_collide_f64(SimConst K, int call, int64_t step,
                                                        const double* v, const int* cstart,
                                                        double* D, double* u,
                                                        long long* pairlog, int64_t cap,
                                                        unsigned long long* counters, int* flags) {
  int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= K.nn) return;
  const int64_t NP = K.np;
  int s = cstart[c], n = cstart[c + 1] - s;
  for (int j = 0; j < n; ++j)
    for (int d = 0; d < 3; ++d) D[d * NP + s + j] = 0.0;
  if (n < 2) return;
  unsigned long long acc = 0, gmx = 0;
  bool touched = false;
  U64x4 w0{};
  for (int k = 0; k < K.navg; ++k) {
    if ((k & 3) == 0)
      w0 = stream_block(K, (uint64_t)c, (uint64_t)step, kTagNpairs, (uint64_t)call,
                        (uint64_t)(k >> 2), 0);
    double xpairs = (double)n * (double)(n - 1) * K.pmax / 2.0 + unif(w0.w[k & 3]);
    if (!(xpairs < (double)kMaxPairsPerOutcome)) {
      atomicOr(&flags[kFlagCapacity], 1);
      continue;
    }
    int64_t npairs = (int64_t)floor(xpairs);
    if (npairs <= 0) continue;
    for (int j = 0; j < n; ++j)
      for (int d = 0; d < 3; ++d) u[d * NP + s + j] = v[d * NP + s + j];
    for (int64_t m = 0; m < npairs; ++m) {
      U64x4 wa = stream_block(K, (uint64_t)c, (uint64_t)step, kTagColl, (uint64_t)call,
                              (uint64_t)k, (uint64_t)(1 + 2 * m));
      U64x4 wb = stream_block(K, (uint64_t)c, (uint64_t)step, kTagColl, (uint64_t)call,
                              (uint64_t)k, (uint64_t)(2 + 2 * m));
      int p = index_below(wa.w[0], n);
      int q = pick_partner(K, c, step, call, k, m, wa, wb, p, n);
      double* up[3] = {u + s + p, u + NP + s + p, u + 2 * NP + s + p};
      double* uq[3] = {u + s + q, u + NP + s + q, u + 2 * NP + s + q};
      double dx = *up[0] - *uq[0], dy = *up[1] - *uq[1], dz = *up[2] - *uq[2];
      double g = sqrt(dx * dx + dy * dy + dz * dz);
      if (g > K.g_max) ++gmx;
      bool ok = unif(wa.w[2]) < sigma_g(K, g) / K.sgmax;
      if (ok) {
        ++acc;
        double seps, ceps;  // eps = 2 pi U_eps, as sin(pi 2 U) and cos(pi 2 U)
        sincospi(2.0 * unif(wa.w[3]), &seps, &ceps);
        const double uchi = unif(wb.w[0]);
        double cchi = cos_chi<double>(K, uchi);  // eq. chi
        double schi = sqrt(fmax(0.0, (1.0 - cchi) * (1.0 + cchi)));
        double nv[3] = {ceps * schi, seps * schi, cchi};  // eq. n
        const double p0[3] = {*up[0], *up[1], *up[2]}, q0[3] = {*uq[0], *uq[1], *uq[2]};
        double pv[3], qv[3];
        post_collision<double, true>(K, p0, q0, g, nv, uchi, pv, qv);
        for (int d = 0; d < 3; ++d) {
          *up[d] = pv[d];
          *uq[d] = qv[d];
        }
        record_angles<double>(pv, qv, g, K.anglog, K.angcap, counters);
      }
      if (pairlog) {
        unsigned long long slot = atomicAdd(&counters[kCntPairLog], 1ull);
        if ((int64_t)slot < cap) {
          long long* r = pairlog + 7 * slot;
          r[0] = c; r[1] = call; r[2] = k; r[3] = m; r[4] = p; r[5] = q; r[6] = ok;
        }
      }
    }
    touched = true;
    for (int j = 0; j < n; ++j)
      for (int d = 0; d < 3; ++d) D[d * NP + s + j] += u[d * NP + s + j] - v[d * NP + s + j];
  }
  if (touched)
    for (int j = 0; j < n; ++j)
      for (int d = 0; d < 3; ++d) D[d * NP + s + j] /= (double)K.navg;
  if (acc) atomicAdd(&counters[kCntAccepted], acc);
  if (gmx) atomicAdd(&counters[kCntGmax], gmx);
}

// <dv^M> per particle (eq. vel_change_3 / vel_change_1c), for the collide API.
__global__ void __launch_bounds__(kBlock) k_source_f64(SimConst K, const double* v, const int* key,
                                                       const int* cstart, double t, double* S) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= K.np) return;
  int c = key[i];
  int n = cstart[c + 1] - cstart[c];
  double u[3] = {v[i], v[K.np + i], v[2 * K.np + i]}, I[3] = {0, 0, 0};
  double coef = (K.w * K.dt * (double)(n - 1)) / (2.0 * K.dV);
  if (n >= 2) source_integral(K, u, t, I);
  for (int d = 0; d < 3; ++d) S[d * K.np + i] = (n >= 2) ? coef * I[d] : 0.0;
}

// ---------------------------------------------------------------------------
// Half kick of eq. velocity_verlet at time t, FP64: CIC gather of E, the
// manufactured field, the collision terms <dv> - <dv^M> and the manufactured
// acceleration (or the exact difference in isolation mode).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_kick_f64(SimConst K, double t, double t_from,
                                                     double t_to, double t_src, const double* x,
                                                     double* v, const double* ash,
                                                     const int* id, const int* key,
                                                     const int* cstart, const double* E,
                                                     const double* D) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= K.np) return;
  const int64_t NP = K.np;
  double xp[3] = {x[i], x[NP + i], x[2 * NP + i]};
  double vp[3] = {v[i], v[NP + i], v[2 * NP + i]};
  int c[3];
  double o[3];
  locate(K, xp, c, o);
  double ep[3] = {0.0, 0.0, 0.0};
  double wx[2] = {1.0 - o[0], o[0]}, wy[2] = {1.0 - o[1], o[1]}, wz[2] = {1.0 - o[2], o[2]};
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        int nd = lin(K, c[0] + cx, c[1] + cy, c[2] + cz);
        double wgt = wx[cx] * wy[cy] * wz[cz];
        for (int d = 0; d < 3; ++d) ep[d] += wgt * E[(int64_t)d * K.nn + nd];
      }
  double em[3];
  EM(K, xp, t, em);
  double h[3] = {0.0, 0.0, 0.0};
  if (K.family == 0) {
    double a[3] = {ash[i], ash[NP + i], ash[2 * NP + i]}, va[3], vb[3], da[3], db[3];
    if (K.isolate) {
      manufactured_velocity(K, a, t_from, va, da);
      manufactured_velocity(K, a, t_to, vb, db);
      for (int d = 0; d < 3; ++d) h[d] = vb[d] - va[d];
    } else {
      manufactured_velocity(K, a, t, va, da);
      for (int d = 0; d < 3; ++d) h[d] = 0.5 * K.dt * da[d];
    }
  }
  double coll[3] = {0.0, 0.0, 0.0};
  if (K.collisions) {
    int cc = key[i];
    int n = cstart[cc + 1] - cstart[cc];
    double I[3] = {0, 0, 0};
    double coef = (K.w * K.dt * (double)(n - 1)) / (2.0 * K.dV);
    if (n >= 2) source_integral(K, vp, t_src, I);
    for (int d = 0; d < 3; ++d) coll[d] = D[d * NP + i] - ((n >= 2) ? coef * I[d] : 0.0);
  }
  for (int d = 0; d < 3; ++d) {
    double acc = K.dt * K.qm * (ep[d] - em[d]);
    v[d * NP + i] = vp[d] + 0.5 * (acc + coll[d]) + h[d];
  }
}

// Drift of eq. velocity_verlet with the manufactured term, periodic wrap, new
// cell key and its count for the next sort.
__global__ void __launch_bounds__(kBlock) k_drift_f64(SimConst K, double t0, double th, double t1,
                                                      double* x, const double* v,
                                                      const double* ash, const int* id, int* key,
                                                      int* slot, int* count, int* flags) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  bool valid = i < K.np;
  int kk = 0;
  if (valid) {
    const int64_t NP = K.np;
    double xp[3] = {x[i], x[NP + i], x[2 * NP + i]};
    int pid = id[i];
    double a[3] = {ash[i], ash[NP + i], ash[2 * NP + i]}, vm[3], vdm[3], h[3] = {0.0, 0.0, 0.0};
    manufactured_velocity(K, a, th, vm, vdm);
    if (K.family == 0) {
      double xq[3];
      position_uniforms(K, pid, xq);
      if (K.isolate) {
        double xa[3], xb[3];
        manufactured_position(K, xq, t0, nullptr, xa);
        manufactured_position(K, xq, t1, nullptr, xb);
        for (int d = 0; d < 3; ++d) h[d] = xb[d] - xa[d];
      } else {
        double xm[3], xd[3];
        manufactured_position(K, xq, th, nullptr, xm);
        manufactured_xdot(K, xm, th, xd);
        for (int d = 0; d < 3; ++d) h[d] = K.dt * xd[d];
      }
    }
    for (int d = 0; d < 3; ++d) {
      double xn = xp[d] + K.dt * (v[d * NP + i] - vm[d]) + h[d];
      if (xn < 0.0) xn += K.L[d];
      if (xn >= K.L[d]) xn -= K.L[d];
      if (!(xn >= 0.0 && xn < K.L[d])) {  // non-finite or more than a box length
        atomicOr(&flags[kFlagNonFinite], 1);
        xn = isfinite(xn) ? xn - floor(xn / K.L[d]) * K.L[d] : 0.0;
        if (!(xn >= 0.0 && xn < K.L[d])) xn = 0.0;
      }
      xp[d] = xn;
      x[d * NP + i] = xn;
    }
    int c[3];
    double o[3];
    locate(K, xp, c, o);
    kk = lin(K, c[0], c[1], c[2]);
    key[i] = kk;
  }
  int s = wave_aggregated_slot(count, kk, valid);
  if (valid) slot[i] = s;
}

// ---------------------------------------------------------------------------
// Error norms (Sec. 4.3): a fixed grid of at most kErrBlocks workgroups; each
// thread accumulates its strided particles (or nodes) in index order, each
// workgroup combines its threads in a fixed order into one partial, and a
// single workgroup combines the partials in block order.  The result depends
// only on the sizes, never on scheduling.  part layout: [blk][14].
// ---------------------------------------------------------------------------
constexpr int kErrBlocks = 1024;

__global__ void __launch_bounds__(kBlock) k_err_particles_f64(SimConst K, double t,
                                                              const double* x, const double* v,
                                                              const int* id, double* part,
                                                              int* flags) {
  x = mem(K, x);
  v = mem(K, v);
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
    double xp[3] = {x[i], x[K.np + i], x[2 * K.np + i]};
    manufactured_position(K, xq, t, xp, xm);
    velocity_shape(K, xv, a);
    manufactured_velocity(K, a, t, vm, vd);
    for (int d = 0; d < 3; ++d) {
      double ex = xp[d] - xm[d];
      if (ex >= 0.5 * K.L[d]) ex -= K.L[d];
      if (ex < -0.5 * K.L[d]) ex += K.L[d];
      e[d] = ex;
      e[3 + d] = v[d * K.np + i] - vm[d];
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

__global__ void __launch_bounds__(kBlock) k_err_nodes(SimConst K, double t, const double* phi,
                                                      double* part) {
  phi = mem(K, phi);
  part = mem(K, part);
  __shared__ double sh[kWaves];
  double s2 = 0.0, mx = 0.0;
  for (int n = blockIdx.x * kBlock + threadIdx.x; n < K.nn; n += gridDim.x * kBlock) {
    int i, j, k;
    node_coords(K, n, i, j, k);
    double xn[3] = {i * K.h[0], j * K.h[1], k * K.h[2]};
    const double e = phi[n] - phiM(K, xn, t);
    s2 += e * e;
    mx = fmax(mx, fabs(e));
  }
  double s = block_sum(s2, sh);
  double m = block_max(mx, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2] = s;
    part[blockIdx.x * 2 + 1] = m;
  }
}

__global__ void __launch_bounds__(kBlock) k_err_final(SimConst K, const double* ppart, int npb,
                                                      const double* npart, int nnb, double* out) {
  ppart = mem(K, ppart);
  npart = mem(K, npart);
  out = mem(K, out);
  __shared__ double sh[kWaves];
  for (int a2 = 0; a2 < 6; ++a2) {
    double s = 0.0, m = 0.0;
    for (int b = threadIdx.x; b < npb; b += kBlock) {
      s += ppart[b * 14 + a2];
      m = fmax(m, ppart[b * 14 + 7 + a2]);
    }
    s = block_sum(s, sh);
    m = block_max(m, sh);
    if (threadIdx.x == 0) {
      out[a2] = sqrt(s / (double)K.np);
      out[7 + a2] = m;
    }
  }
  double s = 0.0, m = 0.0;
  for (int b = threadIdx.x; b < nnb; b += kBlock) {
    s += npart[b * 2];
    m = fmax(m, npart[b * 2 + 1]);
  }
  s = block_sum(s, sh);
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    out[6] = sqrt(s / (double)K.nn);
    out[13] = m;
  }
}

}  // namespace pic
