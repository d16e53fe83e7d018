// Fused particle pass: for a cell-aligned tile of sorted particles, in one
// kernel, the collision call B of step nb and the second half kick, then the
// collision call A of step na, the first half kick and the drift of step na
// (eq. velocity_verlet with eq. avg_outcome and the manufactured sources).
// Either half can be switched off, and a collide-only mode writes <dv> and
// <dv^M> without touching the state.
//
// Tiles: tile t holds the cells whose first particle lies in [t B, (t+1) B)
// of the sorted order, i.e. cells [lower_bound(cstart, tB), lower_bound(cstart,
// (t+1)B)), so every cell is processed whole by one workgroup.  A tile holds
// fewer than B + (largest cell) particles; per-particle working arrays live in
// LDS when they fit and in global scratch otherwise.
//
// Collisions in a tile: (1) one lane per (cell, outcome) draws N_pairs
// (Algorithm 1) and records the few lanes that have candidate pairs; (2) one
// lane per such outcome with at most kSmallPairs pairs runs it on a private
// list of the velocities it changes and stores the changes; (3) one thread per
// cell adds, in increasing outcome order, the stored changes and runs the
// remaining outcomes itself on a copy-on-write private copy of its cell's
// velocities, so <dv> is summed exactly in the order of eq. avg_outcome.  If
// the event list of a tile overflows, step (3) redraws N_pairs for every
// outcome itself.
#pragma once

#include "pic_kernels.hpp"

namespace pic {

constexpr int kSmallPairs = 4;    // outcomes with at most this many pairs run one per lane
constexpr int kPool = 128;        // velocity-change records of those outcomes per tile (lean instances)
constexpr int kPoolGeneral = 512; // the same in the mixed general instances, which take the dense tiles
constexpr int kCellCache = 64;    // cells of a tile whose starts the mixed pass keeps in LDS

// LDS of one collision call over a tile: the events ((cell, outcome) lanes
// with candidate pairs), their pair counts, and the velocity changes of the
// outcomes run one per lane (record start | count << 16, or -1 when the
// outcome is left to its cell's thread).
// NL event lists of CAP (cell, outcome) lanes with pairs each: one list when
// every call draws just before it runs, two when both calls of a pass draw at
// the start of the tile (list 0 call B, list 1 call A).
template <class R, int NL, int CAP, int POOL = kPool>
struct CollideLds {
  static constexpr int kLists = NL, kCap = CAP, kPoolN = POOL;
  int evck[NL][CAP];  // tile-local cell of the event << 16 | its outcome
  int evn[NL][CAP];   // its N_pairs
  int evp[CAP];      // records of the list being run
  // the list being run sorted by (cell, outcome) when it is (sorted_list):
  // keys and event indices
  int skey[CAP], eord[CAP];
  int n_evt[NL], overflow[NL], pool_n;
  int need[NL], big[NL];  // pool records the list's outcomes need; an outcome over kSmallPairs
  int pslot[POOL];
  R pdv[3 * POOL];  // [3][POOL]
};

enum { kDoB = 1, kDoA = 2, kCollideOnly = 4 };

struct PartArgs {
  double* x;            // [3][np] positions, updated by the drift
  double* v;            // [3][np] velocities
  const double* ash;    // [3][np] velocity shape: v^M(t) = vhat(t) a (time independent)
  const int* id;
  int* key;             // cell of each particle (in), new cell after the drift (out)
  int* slot;            // arrival slot for the next sort
  int* count;           // per-cell counts for the next sort (zeroed by the caller)
  const int* cstart;
  const int* tile_c0;   // first cell of each tile, [ntiles + 1]
  const int* tile_s0;   // first particle of each tile, [ntiles + 1]
  const double* E;      // nodal field [3][nn]
  double* gv0;          // global fallback scratch [3][np]
  double* gu;           // global fallback scratch [3][np]
  double* gD;           // global fallback scratch [3][np]
  int* gmark;           // global fallback scratch [np]
  int* gtl;             // global fallback scratch [np]
  double* Dout;         // collide-only outputs [3][np]
  double* Sout;
  long long* pairlog;
  int64_t cap;
  unsigned long long* counters;
  int* flags;
  // tiles the lean instance leaves to the general one: [0] count, [1] workgroups
  // done with the list, [2 ..] tile indices; the general instance works through
  // the list when defer_list is set, else through all tiles
  int* defer;
  int ntiles, defer_list;
  // captured steps: nb = *K.stepc, na = nb + 1; the mixed pass reads its FP32
  // constants from mixc, written by k_step_consts before every pass
  int step_dev;
  const struct MixConst* mixc;
  // paper family: the manufactured displacement of each particle's drift,
  // [3][np], computed before the pass (k_paper_drift_*; FP64 in position
  // units, mixed in cells)
  const double* mdrift;
  const float* mdrift32;
  int mode;
  int64_t nb, na;       // step index of call B (second half) and of call A (first half)
  int callB, callA;     // random-stream call tags (collide-only mode uses callA)
  double tB;            // collide-only: time of the source
};

// The workspace arrays of one ensemble member.  The caller's own buffers (the
// collide-only outputs and the pair log) belong to single simulations and are
// left as they are.
__device__ inline PartArgs member_view(const SimConst& K, PartArgs a) {
  a.x = mem(K, a.x);
  a.v = mem(K, a.v);
  a.ash = mem(K, a.ash);
  a.id = mem(K, a.id);
  a.key = mem(K, a.key);
  a.slot = mem(K, a.slot);
  a.count = mem(K, a.count);
  a.cstart = mem(K, a.cstart);
  a.tile_c0 = mem(K, a.tile_c0);
  a.tile_s0 = mem(K, a.tile_s0);
  a.E = mem(K, a.E);
  a.gv0 = mem(K, a.gv0);
  a.gu = mem(K, a.gu);
  a.gD = mem(K, a.gD);
  a.gmark = mem(K, a.gmark);
  a.gtl = mem(K, a.gtl);
  a.counters = mem(K, a.counters);
  a.flags = mem(K, a.flags);
  a.defer = mem(K, a.defer);
  a.mdrift = mem(K, a.mdrift);
  a.mdrift32 = mem(K, a.mdrift32);
  return a;
}

// Hands tile b to the general instance (thread 0; the caller returns uniformly).
// The list is a count, dl[0], and the tiles from dl[1] on; the host clears the
// count before every lean launch.
__device__ inline void defer_tile(const PartArgs& a, int b) {
  if (threadIdx.x == 0) {
    const int i = atomicAdd(&a.defer[0], 1);
    if (i < a.ntiles) a.defer[1 + i] = b;
  }
}

// The tiles of one launch: the lean instance (FAST) and a plain general launch
// take tile blockIdx.x; the general instance after a lean one takes the
// deferred tiles, workgroup-strided.  (Its workgroups only read the list: a
// last-workgroup reset, one same-address atomic per workgroup, cost more than
// the whole general launch when nothing was deferred.)
template <bool FAST, class F>
__device__ __attribute__((always_inline)) inline void tile_sweep(const PartArgs& a, F&& tile) {
  const bool list = !FAST && a.defer_list;
  const int* dl = a.defer;
  const int n = list ? min(dl[0], a.ntiles) : (int)blockIdx.x + 1;
  for (int i = blockIdx.x; i < n; i += list ? (int)gridDim.x : 1) {
    tile(list ? dl[1 + i] : i);
    if (list) __syncthreads();
  }
}

__device__ inline int lower_bound_i(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Arithmetic of the collision step in the working precision R: FP64 in the
// FP64 form, FP32 in the mixed form (uniforms from the top 24 bits of the same
// words, so both forms draw from one stream).
template <class R> __device__ inline R unif_r(uint64_t w);
// sin(pi x) and cos(pi x) in the working precision (the azimuth eps = 2 pi U
// of a collision is evaluated as pi (2 U): 2 U is exact, and the argument
// reduction of a general sin / cos is not needed)
__device__ inline void sincospi_r(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ inline void sincospi_r(double x, double* s, double* c) { sincospi(x, s, c); }

template <> __device__ inline double unif_r<double>(uint64_t w) { return unif(w); }
template <> __device__ inline float unif_r<float>(uint64_t w) { return unif32(w); }

template <int SIG, class R>
__device__ inline R sigma_g_r(const SimConst& K, R g) {
  if (SIG == kSigHS) return (R)K.sg_coef * g;
  if (SIG == kSigMaxwell) return (R)K.sg_coef;
  R g2 = g * g, r = (R)K.sigma_n[0];
  if (K.n_sigma > 1) r += (R)K.sigma_n[1] * g2;
  if (K.n_sigma > 2) r += (R)K.sigma_n[2] * (g2 * g2);
  return r;
}

// sigma(g) g / (sigma g)_max, the accept probability of Algorithm 1.  In FP32 a
// polynomial cross section is evaluated in units of vbar (coefficients
// sigma_n vbar^(2n) / (sigma g)_max, relative speed g / vbar), which keeps
// every term a normal FP32 number whatever the unit system (in SI the
// paper's sigma_2 is ~5e-42, below FP32's normal range).
template <int SIG, class R>
__device__ inline R accept_ratio(const SimConst& K, R g) {
  if constexpr (SIG == kSigPoly && sizeof(R) == 4) {
    const R gt = g * (R)K.inv_vbar, g2 = gt * gt;
    R r = (R)K.sr[0];
    if (K.n_sigma > 1) r += (R)K.sr[1] * g2;
    if (K.n_sigma > 2) r += (R)K.sr[2] * (g2 * g2);
    return r;
  }
  return sigma_g_r<SIG, R>(K, g) / (R)K.sgmax;
}

// One outcome of Algorithm 1 on one cell of n particles (cell-local SoA arrays
// with stride st).  The outcome's private velocities are copy-on-write: slot j
// holds a private value in u when mark[j] == tag, else its value is v0[j]; the
// slots written are appended to the touched list tl.
template <int SIG, class R, bool FULL>
__device__ inline void ntc_outcome(const SimConst& K, int cell, int64_t step, int call, int k,
                                   int64_t npairs, int n, const R* v0, R* u, int* mark, int tag,
                                   int* tl, int& ntl, int st, int stu, long long* pairlog,
                                   int64_t cap, unsigned long long* counters,
                                   unsigned long long& acc, unsigned long long& gmx) {
  const R gmax = (R)K.g_max;
  for (int64_t m = 0; m < npairs; ++m) {
    U64x4 wa = stream_block(K, (uint64_t)cell, (uint64_t)step, kTagColl, (uint64_t)call,
                            (uint64_t)k, (uint64_t)(1 + 2 * m));
    U64x4 wb = stream_block(K, (uint64_t)cell, (uint64_t)step, kTagColl, (uint64_t)call,
                            (uint64_t)k, (uint64_t)(2 + 2 * m));
    int p = index_below(wa.w[0], n);
    int q = pick_partner(K, cell, step, call, k, m, wa, wb, p, n);
    const bool pp = mark[p] == tag, pq = mark[q] == tag;
    R up[3], uq[3];
    for (int d = 0; d < 3; ++d) {
      up[d] = pp ? u[d * stu + p] : v0[d * st + p];
      uq[d] = pq ? u[d * stu + q] : v0[d * st + q];
    }
    R dx = up[0] - uq[0], dy = up[1] - uq[1], dz = up[2] - uq[2];
    R g = sqrt(dx * dx + dy * dy + dz * dz);
    if (g > gmax) ++gmx;
    bool ok = unif_r<R>(wa.w[2]) < accept_ratio<SIG, R>(K, g);
    if (ok) {
      ++acc;
      R seps, ceps;  // eps = 2 pi U_eps, as sin(pi 2 U) and cos(pi 2 U)
      sincospi_r((R)2.0 * unif_r<R>(wa.w[3]), &seps, &ceps);
      const R uchi = unif_r<R>(wb.w[0]);
      R cchi = cos_chi<R, FULL>(K, uchi);  // eq. chi
      R schi = sqrt(fmax((R)0.0, ((R)1.0 - cchi) * ((R)1.0 + cchi)));
      R nv[3] = {ceps * schi, seps * schi, cchi};  // eq. n
      R pn[3], qn[3];
      post_collision<R, FULL>(K, up, uq, g, nv, uchi, pn, qn);
      for (int d = 0; d < 3; ++d) {
        u[d * stu + p] = pn[d];
        u[d * stu + q] = qn[d];
      }
      if constexpr (FULL) record_angles<R>(pn, qn, g, K.anglog, K.angcap, counters);
      if (mark[p] != tag) {
        mark[p] = tag;
        tl[ntl++] = p;
      }
      if (mark[q] != tag) {
        mark[q] = tag;
        tl[ntl++] = q;
      }
    }
    if (FULL && pairlog) {
      unsigned long long s = atomicAdd(&counters[kCntPairLog], 1ull);
      if ((int64_t)s < cap) {
        long long* r = pairlog + 7 * s;
        r[0] = cell; r[1] = call; r[2] = k; r[3] = m; r[4] = p; r[5] = q; r[6] = ok;
      }
    }
  }
}

// Algorithm 1: N_pairs = floor(N (N - 1) P_max / 2 + U), in FP64 in both forms,
// from the uniform word w.  Beyond kMaxPairsPerOutcome (a degenerate state) it
// raises kFlagCapacity.
__device__ inline int64_t npairs_from(const SimConst& K, int n, uint64_t w, int* flags) {
  double x = (double)n * (double)(n - 1) * K.pmax / 2.0 + unif(w);
  if (!(x < (double)kMaxPairsPerOutcome)) {
    atomicOr(&flags[kFlagCapacity], 1);
    return 0;
  }
  return (int64_t)floor(x);
}

__device__ inline U64x4 npairs_block(const SimConst& K, int cell, int64_t step, int call, int group) {
  return stream_block(K, (uint64_t)cell, (uint64_t)step, kTagNpairs, (uint64_t)call,
                      (uint64_t)group, 0);
}

__device__ inline int64_t npairs_of(const SimConst& K, int cell, int64_t step, int call, int k,
                                    int n, int* flags) {
  return npairs_from(K, n, npairs_block(K, cell, step, call, k >> 2).w[k & 3], flags);
}



// One outcome of Algorithm 1 with at most kSmallPairs candidate pairs, run by
// one lane: the velocities the outcome changes are kept in the lane's own
// records of the pool (slot in pslot, current value in pdv), everything else
// is read from v0; at the end the records are turned into velocity changes.
// Same arithmetic as ntc_outcome.  Returns the number of records.
template <int SIG, class R, bool FULL, int PS>
__device__ inline int ntc_outcome_small(const SimConst& K, int cell, int64_t step, int call, int k,
                                        int npairs, int n, const R* v0, int st, int* pslot, R* pdv,
                                        long long* pairlog, int64_t cap,
                                        unsigned long long* counters, unsigned long long& acc,
                                        unsigned long long& gmx) {
  const R gmax = (R)K.g_max;
  int cnt = 0;
  for (int m = 0; m < npairs; ++m) {
    U64x4 wa = stream_block(K, (uint64_t)cell, (uint64_t)step, kTagColl, (uint64_t)call,
                            (uint64_t)k, (uint64_t)(1 + 2 * m));
    U64x4 wb = stream_block(K, (uint64_t)cell, (uint64_t)step, kTagColl, (uint64_t)call,
                            (uint64_t)k, (uint64_t)(2 + 2 * m));
    int p = index_below(wa.w[0], n);
    int q = pick_partner(K, cell, step, call, k, m, wa, wb, p, n);
    int ip = -1, iq = -1;
    for (int t = 0; t < cnt; ++t) {
      if (pslot[t] == p) ip = t;
      if (pslot[t] == q) iq = t;
    }
    R up[3], uq[3];
    for (int d = 0; d < 3; ++d) {
      up[d] = ip >= 0 ? pdv[d * PS + ip] : v0[d * st + p];
      uq[d] = iq >= 0 ? pdv[d * PS + iq] : v0[d * st + q];
    }
    R dx = up[0] - uq[0], dy = up[1] - uq[1], dz = up[2] - uq[2];
    R g = sqrt(dx * dx + dy * dy + dz * dz);
    if (g > gmax) ++gmx;
    bool ok = unif_r<R>(wa.w[2]) < accept_ratio<SIG, R>(K, g);
    if (ok) {
      ++acc;
      R seps, ceps;  // eps = 2 pi U_eps, as sin(pi 2 U) and cos(pi 2 U)
      sincospi_r((R)2.0 * unif_r<R>(wa.w[3]), &seps, &ceps);
      const R uchi = unif_r<R>(wb.w[0]);
      R cchi = cos_chi<R, FULL>(K, uchi);  // eq. chi
      R schi = sqrt(fmax((R)0.0, ((R)1.0 - cchi) * ((R)1.0 + cchi)));
      R nv[3] = {ceps * schi, seps * schi, cchi};  // eq. n
      if (ip < 0) {
        ip = cnt++;
        pslot[ip] = p;
      }
      if (iq < 0) {
        iq = cnt++;
        pslot[iq] = q;
      }
      R pn[3], qn[3];
      post_collision<R, FULL>(K, up, uq, g, nv, uchi, pn, qn);
      for (int d = 0; d < 3; ++d) {
        pdv[d * PS + ip] = pn[d];
        pdv[d * PS + iq] = qn[d];
      }
      if constexpr (FULL) record_angles<R>(pn, qn, g, K.anglog, K.angcap, counters);
    }
    if (FULL && pairlog) {
      unsigned long long s = atomicAdd(&counters[kCntPairLog], 1ull);
      if ((int64_t)s < cap) {
        long long* r = pairlog + 7 * s;
        r[0] = cell; r[1] = call; r[2] = k; r[3] = m; r[4] = p; r[5] = q; r[6] = ok;
      }
    }
  }
  for (int t = 0; t < cnt; ++t)
    for (int d = 0; d < 3; ++d) pdv[d * PS + t] = pdv[d * PS + t] - v0[d * st + pslot[t]];
  return cnt;
}

// The outcomes of one cell that have candidate pairs, in increasing outcome
// order, summed into D (eq. avg_outcome; the division by N_avg is done where D
// is read).  Outcomes already run by a lane contribute their stored changes;
// the others run here.  Only the particles an outcome changed contribute to
// the sum; the others would add exact zeros.
// Whether a call's event list is sorted for the cell threads: always in the
// FP64 pass; in the mixed pass (SORT instances, launched where a tile's lists
// are expected to be long) from kSortEvents events on.  With few events the
// mixed pass is faster with the plain scan, and faster still in instances
// compiled without the sort at all.
constexpr int kSortEvents = 24;
template <class R, bool SORT>
__device__ inline bool sorted_list(int ne) { return sizeof(R) == 8 || (SORT && ne > kSortEvents); }

template <int SIG, class R, bool FULL, bool LANE_ONLY, bool SORT, class Lds>
__device__ __attribute__((always_inline)) inline void cell_outcomes(const SimConst& K, const PartArgs& a, int call, int64_t step,
                                     int c, int ci, int cs, int n, const R* v0, R* u, R* D,
                                     int* mark, int* tl, int tagbase, int st, int stu,
                                     const Lds& L, int li, int ne, int first, bool all,
                                     unsigned long long& acc, unsigned long long& gmx) {
  const int navg = K.navg;
  int last = -1, idx = first;
  bool marks_clear = false;  // this cell's marks are reset before its first own outcome
  for (int it = 0; it < navg; ++it) {
    int k, ev = -1;
    if (all) {
      k = it;
    } else if (sorted_list<R, SORT>(ne)) {  // next event in the sorted list
      if (idx >= ne || (L.skey[idx] >> 16) != ci) break;
      k = L.skey[idx] & 0xffff;
      ev = L.eord[idx];
      ++idx;
    } else {  // next event of this cell in increasing outcome order
      k = navg;
      for (int e = 0; e < ne; ++e) {
        const int eci = L.evck[li][e] >> 16, ek = L.evck[li][e] & 0xffff;
        if (eci == ci && ek > last && ek < k) {
          k = ek;
          ev = e;
        }
      }
      if (k == navg) break;
    }
    last = k;
    if (LANE_ONLY || (ev >= 0 && L.evp[ev] >= 0)) {  // run by a lane: add its stored changes
      const int r0 = L.evp[ev] & 0xffff, nr = L.evp[ev] >> 16;
      for (int t = 0; t < nr; ++t) {
        int j = cs + L.pslot[r0 + t];
        for (int d = 0; d < 3; ++d) D[d * st + j] += L.pdv[d * Lds::kPoolN + r0 + t];
      }
      continue;
    }
    int64_t np_ = ev >= 0 ? (int64_t)L.evn[li][ev] : npairs_of(K, c, step, call, k, n, a.flags);
    if (np_ <= 0) continue;
    if (!marks_clear) {
      for (int t = 0; t < n; ++t) mark[cs + t] = 0;
      marks_clear = true;
    }
    int ntl = 0;
    ntc_outcome<SIG, R, FULL>(K, c, step, call, k, np_, n, v0 + cs, u + cs, mark + cs, tagbase + k + 1,
                        tl + cs, ntl, st, stu, a.pairlog, a.cap, a.counters, acc, gmx);
    for (int t = 0; t < ntl; ++t) {
      int j = cs + tl[cs + t];
      for (int d = 0; d < 3; ++d) D[d * st + j] += u[d * stu + j] - v0[d * st + j];
    }
  }
}

// The big cells of the collision-heavy mode (heavy_big_cell), one thread per
// cell: the N_avg outcomes of Algorithm 1 in increasing order, each with
// copy-on-write private velocities (u, mark, touched list tl; the mark tag of
// outcome k is k + 1), its velocity changes added to D in outcome order and D
// divided by N_avg at the end, so D equals k_collide_f64's bit for bit.
// Other cells are left to k_collide_heavy.
template <int SIG>
__global__ void __launch_bounds__(kBlock) k_collide_big(SimConst K, int call, int64_t step,
                                                        const double* v, const int* cstart,
                                                        double* D, double* u, int* mark, int* tl,
                                                        long long* pairlog, int64_t cap,
                                                        unsigned long long* counters, int* flags) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= K.nn) return;
  const int64_t NP = K.np;
  const int s = cstart[c], n = cstart[c + 1] - s;
  if (!heavy_big_cell(K, n)) return;
  for (int j = 0; j < n; ++j) {
    mark[s + j] = 0;
    for (int d = 0; d < 3; ++d) D[d * NP + s + j] = 0.0;
  }
  unsigned long long acc = 0, gmx = 0;
  bool touched = false;
  for (int k = 0; k < K.navg; ++k) {
    const int64_t npairs = npairs_of(K, c, step, call, k, n, flags);
    if (npairs <= 0) continue;
    int ntl = 0;
    ntc_outcome<SIG, double, true>(K, c, step, call, k, npairs, n, v + s, u + s, mark + s, k + 1,
                             tl + s, ntl, (int)NP, (int)NP, pairlog, cap, counters, acc, gmx);
    for (int t = 0; t < ntl; ++t) {
      const int j = s + tl[s + t];
      for (int d = 0; d < 3; ++d) D[d * NP + j] += u[d * NP + j] - v[d * NP + j];
    }
    touched = true;
  }
  if (touched)
    for (int j = 0; j < n; ++j)
      for (int d = 0; d < 3; ++d) D[d * NP + s + j] /= (double)K.navg;
  if (acc) atomicAdd(&counters[kCntAccepted], acc);
  if (gmx) atomicAdd(&counters[kCntGmax], gmx);
}

// Collision calls over a tile, in two steps.  tile_draw finds the events
// ((cell, outcome) with candidate pairs) of up to two calls at once: lists
// [lo, hi) of calls[] / steps[] (list 0 call B, list 1 call A of a pass), one
// random block per four outcomes; N_pairs depends only on the cell counts, so
// both calls of a pass draw before either runs.  The caller clears n_evt and
// overflow of those lists before a barrier, and synchronises after.
template <class Lds>
__device__ inline void tile_draw(const SimConst& K, const PartArgs& a, int lo, int hi,
                                 const int calls[2], const int64_t steps[2], int c0, int ncells,
                                 Lds& L) {
  const int navg = K.navg;
  const int ngroups = (navg + 3) >> 2;
  const int64_t lanes = (int64_t)ncells * ngroups;
  for (int64_t l = threadIdx.x; l < (hi - lo) * lanes; l += kTileThreads) {
    const int li = lo + (l >= lanes ? 1 : 0);
    const int64_t r = l - (li - lo) * lanes;
    int ci = (int)(r / ngroups), g = (int)(r - (int64_t)ci * ngroups);
    int c = c0 + ci;
    int n = a.cstart[c + 1] - a.cstart[c];
    if (n < 2) continue;
    U64x4 w = npairs_block(K, c, steps[li], calls[li], g);
    for (int kk = 0; kk < 4; ++kk) {
      int k = 4 * g + kk;
      if (k >= navg) break;
      int64_t np_ = npairs_from(K, n, w.w[kk], a.flags);
      if (np_ > 0) {
        // (cells and outcomes beyond 16 bits go the overflow way)
        int e = ci < 0x8000 && k < 0x10000 ? atomicAdd(&L.n_evt[li], 1) : Lds::kCap;
        if (e < Lds::kCap) {
          L.evck[li][e] = ci << 16 | k;
          L.evn[li][e] = (int)np_;
          if (np_ > kSmallPairs) L.big[li] = 1;
          else atomicAdd(&L.need[li], 2 * (int)np_);
        } else {
          L.overflow[li] = 1;
        }
      }
    }
  }
}

// tile_run: the drawn call of list li: v0 (pre-collision velocities, tile
// slots, stride st) -> D = N_avg <dv> per slot.  u (stride stu), mark and tl
// are scratch of the tile's slots for the outcomes a cell thread runs itself;
// a cell's marks are cleared before its first such outcome in a call.  The
// caller has zeroed D[0, ns) and the record pool count before a barrier (each
// block-wide barrier costs the whole tile its slowest wave, so none is spent
// on that here).
template <int SIG, class R, bool FULL, bool LANE_ONLY, bool SORT, class Lds>
__device__ __attribute__((always_inline)) inline void tile_run(const SimConst& K, const PartArgs& a, int li, int call,
                                int64_t step, int c0, int ncells, int s0, int ns, const R* v0,
                                R* u, R* D, int* mark, int* tl, int tagbase, int st, int stu,
                                Lds& L, const int* lcs = nullptr) {
  const int tid = threadIdx.x;
  const int ne = min(L.n_evt[li], Lds::kCap);
  // start of tile-local cell ci: the tile's copy in LDS when the caller keeps one
  auto cell_start = [&](int ci) { return lcs ? lcs[ci] : a.cstart[c0 + ci]; };
  // LANE_ONLY: the caller has checked tile_lane_only, so every event runs on a lane
  const bool all = !LANE_ONLY && L.overflow[li] != 0;
  unsigned long long acc = 0, gmx = 0;
  // small outcomes, one per lane, into the record pool
  if (!all) {
    if (sorted_list<R, SORT>(ne)) {
      // The list sorted by (cell, outcome) keys, which are distinct: each
      // event's rank, on the waves after the first (idle while the first
      // wave's lanes run the outcomes), so that the cell threads below find
      // their events by binary search.
      if (tid >= 64)
        for (int e = tid - 64; e < ne; e += kTileThreads - 64) {
          const int key = L.evck[li][e];
          int rank = 0;
          for (int f = 0; f < ne; ++f) rank += L.evck[li][f] < key ? 1 : 0;
          L.skey[rank] = key;
          L.eord[rank] = e;
        }
    }
    for (int e = tid; e < ne; e += kTileThreads) {
      int np_ = L.evn[li][e];
      int start = -1;
      if (LANE_ONLY || np_ <= kSmallPairs) {
        start = atomicAdd(&L.pool_n, 2 * np_);
        if (!LANE_ONLY && start + 2 * np_ > Lds::kPoolN) start = -1;
      }
      if (!LANE_ONLY && start < 0) {
        L.evp[e] = -1;
        continue;
      }
      int ci = L.evck[li][e] >> 16, k = L.evck[li][e] & 0xffff;
      int c = c0 + ci;
      int cs = cell_start(ci) - s0, n = cell_start(ci + 1) - cell_start(ci);
      int cnt = ntc_outcome_small<SIG, R, FULL, Lds::kPoolN>(K, c, step, call, k, np_, n, v0 + cs, st,
                                          L.pslot + start, L.pdv + start, a.pairlog, a.cap,
                                          a.counters, acc, gmx);
      L.evp[e] = start | (cnt << 16);
    }
    __syncthreads();
  }
  // per cell, in increasing outcome order
  for (int ci = tid; ci < ncells; ci += kTileThreads) {
    int c = c0 + ci;
    int cs = cell_start(ci) - s0, n = cell_start(ci + 1) - cell_start(ci);
    if (n < 2) continue;
    int first = 0;  // (sorted list) the cell's first event in key order
    if (!all) {  // skip cells without events quickly
      if (sorted_list<R, SORT>(ne)) {
        first = lower_bound_i(L.skey, ne, ci << 16);
        if (first >= ne || (L.skey[first] >> 16) != ci) continue;
      } else {
        bool any = false;
        for (int e = 0; e < ne; ++e) any |= (L.evck[li][e] >> 16) == ci;
        if (!any) continue;
      }
    }
    cell_outcomes<SIG, R, FULL, LANE_ONLY, SORT>(K, a, call, step, c, ci, cs, n, v0, u, D, mark, tl, tagbase,
                                           st, stu, L, li, ne, first, all, acc, gmx);
  }
  if (acc) atomicAdd(&a.counters[kCntAccepted], acc);
  if (gmx) atomicAdd(&a.counters[kCntGmax], gmx);
  __syncthreads();
}

// Start-of-tile state of a pass's collisions: both event lists empty and no
// records (one thread, before the kernel's first barrier), D = 0 (before the
// barrier that ends the tile's loads).
template <class Lds>
__device__ inline void tile_lists_clear(Lds& L) {
  for (int i = 0; i < Lds::kLists; ++i) L.n_evt[i] = L.overflow[i] = L.need[i] = L.big[i] = 0;
  L.pool_n = 0;
}

template <class R>
__device__ inline void tile_zero_D(int ns, int st, R* D) {
  for (int j = threadIdx.x; j < ns; j += kTileThreads) D[j] = D[st + j] = D[2 * st + j] = (R)0.0;
}

// One collision call over the tile (draw, then run; list 0).  Inlined: as an
// out-of-line call its frame would give every wave of the pass a large
// private segment, which slows the whole launch even when no collide-only
// call runs.
template <int SIG, class R, bool FULL, class Lds>
__device__ __attribute__((always_inline)) inline void tile_collide(const SimConst& K, const PartArgs& a, int call,
                                    int64_t step, int c0, int ncells, int s0, int ns,
                                    const R* v0, R* u, R* D, int* mark, int* tl, int tagbase,
                                    int st, int stu, Lds& L) {
  if (threadIdx.x == 0) {
    L.n_evt[0] = 0;
    L.overflow[0] = 0;
    L.need[0] = 0;
    L.big[0] = 0;
    L.pool_n = 0;
  }
  for (int j = threadIdx.x; j < ns; j += kTileThreads) D[j] = D[st + j] = D[2 * st + j] = (R)0.0;
  __syncthreads();
  const int calls[2] = {call, call};
  const int64_t steps[2] = {step, step};
  tile_draw(K, a, 0, 1, calls, steps, c0, ncells, L);
  __syncthreads();
  tile_run<SIG, R, FULL, false, true>(K, a, 0, call, step, c0, ncells, s0, ns, v0, u, D, mark, tl, tagbase, st,
                         stu, L);
}

// The events of the pass's calls (B: list 0, A: list 1), drawn together at
// the start of a tile, beside the loads of the tile's state (the draw reads
// only the cell starts, so its random blocks overlap the loads' latency); the
// lists were cleared before the kernel's first barrier, and the barrier that
// ends the loads publishes them.
template <class Lds>
__device__ inline void tile_draw_pass(const SimConst& K, const PartArgs& a, int c0, int ncells,
                                      Lds& L) {
  static_assert(Lds::kLists == 2, "a pass draws into two lists");
  const int calls[2] = {a.callB, a.callA};
  const int64_t steps[2] = {a.nb, a.na};
  const int lo = (a.mode & kDoB) ? 0 : 1, hi = (a.mode & kDoA) ? 2 : 1;
  tile_draw(K, a, lo, hi, calls, steps, c0, ncells, L);
}

// Whether every outcome of the drawn lists [lo, hi) runs on a lane: no list
// overflowed, no outcome has more than kSmallPairs pairs, and each list's
// records fit the pool.  Read after the barrier that ends the draw.
template <class Lds>
__device__ inline bool tile_lane_only(const Lds& L, int lo, int hi) {
  bool ok = true;
  for (int li = lo; li < hi; ++li)
    ok = ok && !L.overflow[li] && !L.big[li] && L.need[li] <= Lds::kPoolN;
  return ok;
}

// Tile bounds of block b: first cell, cell count, first particle, particle count.
__device__ inline void tile_range(const SimConst& K, const int* tile_c0, const int* cstart, int b,
                                  int* sh_i) {
  if (threadIdx.x == 0) {
    int c0 = min(tile_c0[b], K.nn);
    int c1 = min(max(tile_c0[b + 1], c0), K.nn);
    sh_i[0] = c0;
    sh_i[1] = c1;
    sh_i[2] = cstart[c0];
    sh_i[3] = cstart[c1];
  }
  __syncthreads();
}

// Eight cloud-in-cell corner weights of an FP64 position, corner k = cz 4 + cy 2 + cx.
__device__ inline void cic_weights_f64(const SimConst& K, const double xp[3], double w[8]) {
  int ci[3];
  double o[3];
  locate(K, xp, ci, o);
  double wx[2] = {1.0 - o[0], o[0]}, wy[2] = {1.0 - o[1], o[1]}, wz[2] = {1.0 - o[2], o[2]};
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) w[cz * 4 + cy * 2 + cx] = wx[cx] * wy[cy] * wz[cz];
}

// Cell moments (the eight corner-weight sums of each cell) by cell-aligned
// tiles: the particles of a tile compute their weights in parallel into LDS,
// then one lane per (cell, corner) adds its cell's weights in sorted order,
// the order of the per-cell loop of k_deposit_moments_f64, so the two agree
// bit for bit.  Tiles larger than the LDS slots read the positions directly.
__global__ void __launch_bounds__(kTileThreads) k_deposit_tiles_f64(SimConst K, const double* x,
                                                              const int* cstart,
                                                              const int* tile_c0, double* mom) {
  x = mem(K, x);
  cstart = mem(K, cstart);
  tile_c0 = mem(K, tile_c0);
  mom = mem(K, mom);
  __shared__ double W[8 * kLdsSlots];
  __shared__ int sh_i[4];
  tile_range(K, tile_c0, cstart, blockIdx.x, sh_i);
  const int c0 = sh_i[0], ncells = sh_i[1] - sh_i[0], s0 = sh_i[2], ns = sh_i[3] - sh_i[2];
  const bool lds = ns <= kLdsSlots;
  const int NP = (int)K.np;
  if (lds) {
    for (int j = threadIdx.x; j < ns; j += kTileThreads) {
      const int p = s0 + j;
      double xp[3] = {x[p], x[NP + p], x[2 * NP + p]}, w[8];
      cic_weights_f64(K, xp, w);
#pragma unroll
      for (int k = 0; k < 8; ++k) W[k * kLdsSlots + j] = w[k];
    }
    __syncthreads();
  }
  for (int l = threadIdx.x; l < 8 * ncells; l += kTileThreads) {
    const int k = l & 7, c = c0 + (l >> 3);
    const int a = cstart[c] - s0, e = cstart[c + 1] - s0;
    double m = 0.0;
    if (lds) {
      for (int j = a; j < e; ++j) m += W[k * kLdsSlots + j];
    } else {
      for (int j = a; j < e; ++j) {
        const int p = s0 + j;
        double xp[3] = {x[p], x[NP + p], x[2 * NP + p]}, w[8];
        cic_weights_f64(K, xp, w);
        m += w[k];
      }
    }
    mom[(int64_t)k * K.nn + c] = m;
  }
}

__device__ inline void gather_f64(const SimConst& K, const double* E, const double xp[3], double ep[3],
                                  int c[3]) {
  double o[3];
  locate(K, xp, c, o);
  ep[0] = ep[1] = ep[2] = 0.0;
  double wx[2] = {1.0 - o[0], o[0]}, wy[2] = {1.0 - o[1], o[1]}, wz[2] = {1.0 - o[2], o[2]};
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        int nd = lin(K, c[0] + cx, c[1] + cy, c[2] + cz);
        double wgt = wx[cx] * wy[cy] * wz[cz];
        for (int d = 0; d < 3; ++d) ep[d] += wgt * E[(int64_t)d * K.nn + nd];
      }
}

// Half kick of one particle (eq. velocity_verlet): v += (acc + D - S)/2 + h.
// FAM: 0 paper family (time-dependent velocity shape), 1 configuration family.
template <int FAM, int SIG>
__device__ inline void half_kick_f64(const SimConst& K, const double acc[3], double t,
                                     double t_from, double t_to, double t_src,
                                     const double aa[3], int n, const double D[3], double v[3]) {
  double h[3] = {0.0, 0.0, 0.0};
  if (FAM == 0) {
    double va[3], vb[3], da[3], db[3];
    if (K.isolate) {
      manufactured_velocity(K, aa, t_from, va, da);
      manufactured_velocity(K, aa, t_to, vb, db);
      for (int d = 0; d < 3; ++d) h[d] = vb[d] - va[d];
    } else {
      manufactured_velocity(K, aa, t, va, da);
      for (int d = 0; d < 3; ++d) h[d] = 0.5 * K.dt * da[d];
    }
  }
  double coll[3] = {0.0, 0.0, 0.0};
  if (K.collisions) {
    double I[3] = {0.0, 0.0, 0.0};
    double coef = (K.w * K.dt * (double)(n - 1)) / (2.0 * K.dV);
    if (n >= 2) source_integral_t<SIG>(K, v, t_src, I);
    for (int d = 0; d < 3; ++d) coll[d] = D[d] - ((n >= 2) ? coef * I[d] : 0.0);
  }
  for (int d = 0; d < 3; ++d) v[d] = v[d] + 0.5 * (acc[d] + coll[d]) + h[d];
}

// Field part of a half kick at time t: dt q/m (E - E^M) at the particle.
__device__ inline void field_acc_f64(const SimConst& K, const double xp[3], const double ep[3],
                                     double t, double acc[3]) {
  double em[3];
  EM(K, xp, t, em);
  for (int d = 0; d < 3; ++d) acc[d] = K.dt * K.qm * (ep[d] - em[d]);
}

// Paper family, FP64 form: the manufactured term of every particle's drift in
// step na (position units), from FP64 root solves of x^M (eq. mms_sol) started
// at the uniform guess: dt xdot^M at t^{na+1/2}, or x^M(t^{na+1}) - x^M(t^{na})
// in isolation mode.  It depends only on the particle's identity and the time,
// so it runs before the pass (which then keeps no root solver); out is the
// idle half of the double-buffered positions.
__global__ void __launch_bounds__(kBlock) k_paper_drift_f64(SimConst K, PartArgs a, double* out) {
  a = member_view(K, a);
  out = mem(K, out);
  if (a.step_dev) {  // a captured step: its step index from the device
    a.nb = *K.stepc;
    a.na = a.nb + 1;
  }
  const int64_t NP = K.np;
  const double dt = K.dt;
  const double t0 = (double)a.na * dt, th = ((double)a.na + 0.5) * dt, t1 = ((double)a.na + 1.0) * dt;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < NP;
       p += (int64_t)gridDim.x * blockDim.x) {
    double xq[3], h[3];
    position_uniforms(K, a.id[p], xq);
    if (K.isolate) {
      double xa[3], xb[3];
      manufactured_position(K, xq, t0, nullptr, xa);
      manufactured_position(K, xq, t1, nullptr, xb);
      for (int d = 0; d < 3; ++d) h[d] = xb[d] - xa[d];
    } else {
      double xm[3], xd[3];
      manufactured_position(K, xq, th, nullptr, xm);
      manufactured_xdot(K, xm, th, xd);
      for (int d = 0; d < 3; ++d) h[d] = dt * xd[d];
    }
    for (int d = 0; d < 3; ++d) out[d * NP + p] = h[d];
  }
}

// Registers are capped for four resident waves per SIMD (128 VGPRs), accepting
// a few spills: the pass is latency bound and gains more from resident waves
// than it loses to spill traffic.  The paper family's instances take the same
// cap: their drift term's root solves run before the pass (k_paper_drift_f64).
template <int FAM, int SIG, bool FULL, bool FAST>
__global__ void __launch_bounds__(kTileThreads, FAST ? PIC_F64_LEAN_WAVES : PIC_F64_WAVES)
    k_particles_f64(SimConst K, PartArgs a) {
  a = member_view(K, a);
  if (a.step_dev) {  // a captured step: its step index from the device
    a.nb = *K.stepc;
    a.na = a.nb + 1;
  }
  // the copy-on-write scratch of outcomes run by a cell thread is global
  __shared__ double lv0[3 * kLdsSlots], lD[3 * kLdsSlots], lacc[3 * kLdsSlots];
  __shared__ int lkey[kLdsSlots];
  __shared__ int lcs[kCellCache + 1];  // cell starts of a tile of at most kCellCache cells
  // (one pool size for both instances: a larger one in the general instance
  // cut its occupancy more than it gained)
  __shared__ CollideLds<double, 2, 128> cl;  // both calls of the pass drawn up front
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
    double* v0 = lds ? lv0 : a.gv0 + s0;
    double* u = a.gu + s0;
    double* D = lds ? lD : a.gD + s0;
    int* mark = a.gmark + s0;
    int* tl = a.gtl + s0;
    const double dt = K.dt;
    const double inv_navg_den = (double)K.navg;

    const bool pass_coll = K.collisions && !(a.mode & kCollideOnly);
    // A tile held in LDS computes the field part of its first kick while it
    // loads and keeps it in lacc; with both halves in one pass kick B (end of
    // step n) and kick A (start of step n + 1) are at the same time and
    // position, so kick A reuses it (bitwise what it would compute again).
    const bool pre = lds && !(a.mode & kCollideOnly);
    const bool reuse_A = pre && (!(a.mode & kDoB) || a.na == a.nb + 1);
    const double t_pre = (a.mode & kDoB) ? ((double)a.nb + 1.0) * dt : (double)a.na * dt;
    if (pass_coll) tile_zero_D(ns, st, D);
    for (int j = tid; j < ns; j += kTileThreads) {
      const int p = s0 + j;
      for (int d = 0; d < 3; ++d) v0[d * st + j] = a.v[(int64_t)d * NP + p];
      if (lds) {
        lkey[j] = a.key[p];
        if (pre) {
          double xp[3] = {a.x[p], a.x[NP + p], a.x[2 * NP + p]}, ep[3], acc[3];
          int cc[3];
          gather_f64(K, a.E, xp, ep, cc);
          field_acc_f64(K, xp, ep, t_pre, acc);
          for (int d = 0; d < 3; ++d) lacc[d * kLdsSlots + j] = acc[d];
        }
      }
    }
    const bool few_cells = ncells <= kCellCache;
    if (few_cells)
      for (int i = tid; i <= ncells; i += kTileThreads) lcs[i] = a.cstart[c0 + i];
    if (pass_coll) tile_draw_pass(K, a, c0, ncells, cl);
    __syncthreads();
    // cell and particle count of slot j at the start of the pass
    auto cell_of = [&](int j) { return lds ? lkey[j] : a.key[s0 + j]; };
    auto count_of = [&](int c) {
      return few_cells ? lcs[c - c0 + 1] - lcs[c - c0] : a.cstart[c + 1] - a.cstart[c];
    };
    if (FAST && pass_coll &&
        !tile_lane_only(cl, (a.mode & kDoB) ? 0 : 1, (a.mode & kDoA) ? 2 : 1)) {
      defer_tile(a, b);  // (uniform, and nothing written to memory yet)
      return;
    }

    if (!FAST && (a.mode & kCollideOnly)) {  // (the lean instance never runs collide-only)
      tile_collide<SIG, double, FULL>(K, a, a.callA, a.na, c0, ncells, s0, ns, v0, u, D, mark, tl, 0, st,
                                NP, cl);
      for (int j = tid; j < ns; j += kTileThreads) {
        int c = a.key[s0 + j];
        int n = a.cstart[c + 1] - a.cstart[c];
        double vp[3] = {v0[j], v0[st + j], v0[2 * st + j]}, I[3] = {0, 0, 0};
        double coef = (K.w * K.dt * (double)(n - 1)) / (2.0 * K.dV);
        if (n >= 2) source_integral_t<SIG>(K, vp, a.tB, I);
        for (int d = 0; d < 3; ++d) {
          a.Dout[(int64_t)d * NP + s0 + j] = D[d * st + j] / inv_navg_den;
          a.Sout[(int64_t)d * NP + s0 + j] = (n >= 2) ? coef * I[d] : 0.0;
        }
      }
      return;
    }

    // With both halves in one pass, kick B (end of step n) and kick A (start of
    // step n + 1) are at the same time t^{n+1} and position, so the field part
    // of the acceleration is computed once and kept per slot in LDS (bitwise the
    // same).
    if (a.mode & kDoB) {
      // collision call B at t^{nb+1/2} on v^{nb+1/2}, then the second half kick at t^{nb+1}
      const double th = ((double)a.nb + 0.5) * dt, t1 = ((double)a.nb + 1.0) * dt;
      if (K.collisions)
        tile_run<SIG, double, FULL, FAST, true>(K, a, 0, a.callB, a.nb, c0, ncells, s0, ns, v0, u, D, mark, tl, 0, st,
                                  NP, cl, few_cells ? lcs : nullptr);
      for (int j = tid; j < ns; j += kTileThreads) {
        int p = s0 + j;
        double acc[3];
        if (pre) {
          for (int d = 0; d < 3; ++d) acc[d] = lacc[d * kLdsSlots + j];
        } else {
          double xp[3] = {a.x[p], a.x[NP + p], a.x[2 * NP + p]}, ep[3];
          int cc[3];
          gather_f64(K, a.E, xp, ep, cc);
          field_acc_f64(K, xp, ep, t1, acc);
        }
        const int n = count_of(cell_of(j));
        double vp[3] = {v0[j], v0[st + j], v0[2 * st + j]};
        double aa[3] = {a.ash[p], a.ash[NP + p], a.ash[2 * NP + p]};
        double Dj[3] = {0.0, 0.0, 0.0};
        if (K.collisions)
          for (int d = 0; d < 3; ++d) {
            Dj[d] = D[d * st + j] / inv_navg_den;
            D[d * st + j] = 0.0;  // cleared for call A (the barrier below orders it)
          }
        half_kick_f64<FAM, SIG>(K, acc, t1, th, t1, th, aa, n, Dj, vp);
        for (int d = 0; d < 3; ++d) v0[d * st + j] = vp[d];
      }
      if (tid == 0) cl.pool_n = 0;
      __syncthreads();
      if (!(a.mode & kDoA)) {
        for (int j = tid; j < ns; j += kTileThreads)
          for (int d = 0; d < 3; ++d) a.v[(int64_t)d * NP + s0 + j] = v0[d * st + j];
        return;
      }
    }

    // collision call A at t^{na} on v^{na}, first half kick, drift to t^{na+1}
    const double t0 = (double)a.na * dt, th = ((double)a.na + 0.5) * dt, t1 = ((double)a.na + 1.0) * dt;
    if (K.collisions)
      tile_run<SIG, double, FULL, FAST, true>(K, a, 1, a.callA, a.na, c0, ncells, s0, ns, v0, u, D, mark, tl, K.navg,
                                st, NP, cl, few_cells ? lcs : nullptr);
    for (int base = 0; base < ns; base += kTileThreads) {
      int j = base + tid;
      bool valid = j < ns;
      int kk = 0;
      if (valid) {
        int p = s0 + j;
        double xp[3] = {a.x[p], a.x[NP + p], a.x[2 * NP + p]}, acc[3];
        if (reuse_A) {
          for (int d = 0; d < 3; ++d) acc[d] = lacc[d * kLdsSlots + j];
        } else {
          double ep[3];
          int cc[3];
          gather_f64(K, a.E, xp, ep, cc);
          field_acc_f64(K, xp, ep, t0, acc);
        }
        const int n = count_of(cell_of(j));
        double vp[3] = {v0[j], v0[st + j], v0[2 * st + j]};
        double aa[3] = {a.ash[p], a.ash[NP + p], a.ash[2 * NP + p]};
        double Dj[3] = {0.0, 0.0, 0.0};
        if (K.collisions)
          for (int d = 0; d < 3; ++d) Dj[d] = D[d * st + j] / inv_navg_den;
        half_kick_f64<FAM, SIG>(K, acc, t0, t0, th, t0, aa, n, Dj, vp);
        // drift (eq. velocity_verlet) with the manufactured term
        double vm[3], vdm[3], h[3] = {0.0, 0.0, 0.0};
        if (FAM == 1) {
          for (int d = 0; d < 3; ++d) vm[d] = K.vbar * aa[d];
        } else {
          manufactured_velocity(K, aa, th, vm, vdm);
        }
        if (FAM == 0)  // the manufactured displacement, from k_paper_drift_f64
          for (int d = 0; d < 3; ++d) h[d] = a.mdrift[(int64_t)d * NP + p];
        for (int d = 0; d < 3; ++d) {
          double xn = xp[d] + dt * (vp[d] - vm[d]) + h[d];
          if (xn < 0.0) xn += K.L[d];
          if (xn >= K.L[d]) xn -= K.L[d];
          if (!(xn >= 0.0 && xn < K.L[d])) {  // non-finite or more than a box length
            atomicOr(&a.flags[kFlagNonFinite], 1);
            xn = isfinite(xn) ? xn - floor(xn / K.L[d]) * K.L[d] : 0.0;
            if (!(xn >= 0.0 && xn < K.L[d])) xn = 0.0;
          }
          xp[d] = xn;
          a.x[(int64_t)d * NP + p] = xn;
          a.v[(int64_t)d * NP + p] = vp[d];
        }
        int ci[3];
        double o[3];
        locate(K, xp, ci, o);
        kk = lin(K, ci[0], ci[1], ci[2]);
        a.key[p] = kk;
      }
      int sl = wave_aggregated_slot(a.count, kk, valid);
      if (valid) a.slot[s0 + j] = sl;
    }
  };
  tile_sweep<FAST>(a, tile);
}

}  // namespace pic
