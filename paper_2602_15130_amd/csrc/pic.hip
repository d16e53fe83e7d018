// Host side of the C ABI declared in include/pic.h: validation, derived
// constants, workspace layout and the launch sequence of a time step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "pic_kernels.hpp"
#include "pic_particle.hpp"
#include "pic_mixed.hpp"
#include "pic_cg_brick.hpp"
#include "pic_lowmode.hpp"
#include "pic_angles.hpp"
#include "pic_collide_heavy.hpp"
#include "pic_order.hpp"
#include "pic_host.hpp"

using namespace pic;

namespace {

thread_local std::string g_create_error;

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

enum Arr {
  A_X0, A_X1, A_V0, A_V1, A_SH0, A_SH1, A_ID0, A_ID1,  // FP64 particle state, two buffers
  A_OFF0, A_OFF1, A_VF0, A_VF1, A_ASF0, A_ASF1,      // mixed particle state, two buffers
  A_KEY, A_SLOT, A_TIDX, A_TKEY, A_D, A_U, A_V0G,
  A_COUNT, A_CSTART, A_BSUM, A_TILE, A_MOM, A_RHO, A_B, A_PHI, A_E, A_E32, A_CGV, A_LOW,
  A_PART_A, A_PART_B, A_EPART, A_NPART, A_NORMS, A_BAR, A_RESULT, A_FLAGS, A_CNT, A_CGIT, A_CGRR,
  A_DEFER, A_STEPC, A_MIXC,
  A_NARR
};

struct Layout {
  int64_t off[A_NARR];
  int64_t bytes[A_NARR];
  int64_t total;
};

Layout make_layout(const pic_discretization* d, int precision) {
  const int64_t np = d->n_particles;
  const int64_t nn = (int64_t)d->ncell[0] * d->ncell[1] * d->ncell[2];
  const int64_t nblk_p = (np + kBlock - 1) / kBlock, nblk_n = (nn + kBlock - 1) / kBlock;
  const int64_t nscan = (nn + kScanTile - 1) / kScanTile;
  const bool f64 = precision == PIC_FP64;
  const int64_t pf = f64 ? np : 0, pm = f64 ? 0 : np;
  Layout L;
  int64_t b[A_NARR] = {};
  b[A_X0] = b[A_X1] = b[A_V0] = b[A_V1] = b[A_SH0] = b[A_SH1] = 3 * pf * 8;
  b[A_ID0] = b[A_ID1] = np * 4;
  b[A_OFF0] = b[A_OFF1] = b[A_VF0] = b[A_VF1] = b[A_ASF0] = b[A_ASF1] = 3 * pm * 4;
  b[A_KEY] = b[A_SLOT] = b[A_TIDX] = b[A_TKEY] = np * 4;
  b[A_D] = 3 * np * (f64 ? 8 : 4);
  b[A_U] = 3 * np * 8;    // private collision copies; FP64 export of the mixed state
  b[A_V0G] = 3 * np * 8;
  b[A_COUNT] = nn * 4;
  b[A_CSTART] = (nn + 1) * 4;
  b[A_BSUM] = (nscan + 1) * 4;
  b[A_TILE] = 2 * ((np + kTileB - 1) / kTileB + 2) * 4;  // first cell and first particle per tile
  b[A_MOM] = 64 * nn;  // 8 FP64 cell moments, or 8 FP32 moments + 8 compensations
  b[A_RHO] = b[A_B] = b[A_PHI] = nn * 8;
  b[A_CGV] = 9 * nn * 8;  // CG vectors r, w, s (two each) and p, or the brick solver's faces
  {  // low-mode pre-solve: basis tables, eigenvalues, slab projections, x back-transform
    const int64_t nmax = std::max({d->ncell[0], d->ncell[1], d->ncell[2]});
    int rows = 0;
    const int64_t slabs = low_slabs((int)d->ncell[1], (int)d->ncell[2], rows);
    b[A_LOW] = (3 * kLowMaxM * nmax + 3 * kLowMaxM + slabs * kLowMaxM * kLowMaxM * d->ncell[2] +
                (int64_t)kLowMaxM * d->ncell[0] * d->ncell[2]) * 8;
  }
  b[A_E] = 3 * nn * 8;
  b[A_E32] = f64 ? 0 : 3 * nn * 4;
  b[A_PART_A] = b[A_PART_B] = std::max<int64_t>(nblk_n, 4096) * 8;
  b[A_EPART] = std::min<int64_t>(nblk_p, kErrBlocks) * 14 * 8;
  b[A_NPART] = std::min<int64_t>(nblk_n, kErrBlocks) * 2 * 8;
  b[A_NORMS] = 16 * 8;
  b[A_BAR] = (int64_t)(4096 + 1) * kFlagStride * 4;  // per-block arrival flags + release word
  b[A_RESULT] = kMaxRed * 8;
  b[A_FLAGS] = kFlagCount * 4;
  b[A_CNT] = kCntCount * 8;
  b[A_CGIT] = 4;
  b[A_CGRR] = 8;
  b[A_DEFER] = ((np + kTileB - 1) / kTileB + 1) * 4;  // tiles the lean pass leaves to the general one
  b[A_STEPC] = 8;                   // completed steps, for captured steps
  b[A_MIXC] = sizeof(MixConst);     // the mixed pass's constants of a captured step
  int64_t t = 0;
  for (int i = 0; i < A_NARR; ++i) {
    L.off[i] = t;
    L.bytes[i] = b[i];
    t += align_up(std::max<int64_t>(b[i], 1));
  }
  L.total = t;
  return L;
}

int validate(const pic_problem* p, const pic_discretization* d, int precision, std::string& err) {
  auto bad = [&](const char* m) {
    err = m;
    return PIC_EINVAL;
  };
  if (!p || !d) return bad("null problem or discretization");
  if (precision != PIC_FP64 && precision != PIC_MIXED) return bad("unknown precision");
  if (p->family != PIC_MMS_PAPER && p->family != PIC_MMS_CFG) return bad("unknown family");
  for (int k = 0; k < 3; ++k) {
    if (d->ncell[k] < 3 || d->ncell[k] > 1023) return bad("ncell must be in [3, 1023]");
    if (!(p->L[k] > 0.0)) return bad("L must be positive");
  }
  if ((int64_t)d->ncell[0] * d->ncell[1] * d->ncell[2] > (1 << 30)) return bad("too many cells");
  if (d->n_particles < 1 || d->n_particles > (int64_t)2147483647)
    return bad("n_particles must be in [1, 2^31 - 1]");
  if (!(d->dt > 0.0)) return bad("dt must be positive");
  if (d->n_avg < 1) return bad("n_avg must be >= 1");
  if (!(d->cg_tol > 0.0) || d->cg_max_iter < 1) return bad("bad CG controls");
  if (d->poisson_op != PIC_OP_FD7 && d->poisson_op != PIC_OP_Q1) return bad("poisson_op must be 0 or 1");
  if (!(p->nphys > 0.0) || !(p->eps0 > 0.0) || !(p->T > 0.0) || !(p->vbar > 0.0))
    return bad("nphys, eps0, T and vbar must be positive");
  if (p->field_to_particles && p->m == 0.0) return bad("m must be nonzero");
  if (p->family == PIC_MMS_CFG && !(std::fabs(p->rho_amp) < 1.0)) return bad("need |rho_amp| < 1");
  if (p->chi_model < PIC_CHI_ISO || p->chi_model > PIC_CHI_VSS) return bad("chi_model must be 0, 1 or 2");
  if (p->chi_model == PIC_CHI_VSS && !(p->chi_alpha >= 1.0 && p->chi_alpha <= 2.0))
    return bad("chi_alpha must lie in [1, 2]");
  if (p->coding_error < 0 || p->coding_error > 2) return bad("coding_error must be 0, 1 or 2");
  if (p->collisions) {
    if (!(p->g_max > 0.0)) return bad("g_max must be positive");
    if (p->sigma_model == PIC_SIGMA_POLY) {
      if (p->n_sigma < 1 || p->n_sigma > 3) return bad("n_sigma must be 1..3");
    } else if (p->sigma_model == PIC_SIGMA_VHS) {
      if (p->omega != 0.5 && p->omega != 1.0)
        return bad("VHS needs omega in {0.5, 1} (closed-form sources only)");
      if (p->omega == 0.5 && p->family != PIC_MMS_CFG)
        return bad("hard sphere needs the Gaussian (cfg) family");
      if (!(p->sigma_ref > 0.0) || !(p->g_ref > 0.0)) return bad("bad VHS constants");
    } else {
      return bad("unknown sigma model");
    }
  }
  return PIC_OK;
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }

// Instances of the brick solver: nodes per thread and threads per workgroup.
struct BrickKernel {
  int q, nt;
  const void* fn;
};
const BrickKernel kBrickKernels[] = {
    {1, 256, (const void*)k_cg_brick<1, 256>},   {2, 256, (const void*)k_cg_brick<2, 256>},
    {4, 256, (const void*)k_cg_brick<4, 256>},   {8, 256, (const void*)k_cg_brick<8, 256>},
    {16, 256, (const void*)k_cg_brick<16, 256>}, {16, 512, (const void*)k_cg_brick<16, 512>},
    {8, 1024, (const void*)k_cg_brick<8, 1024>},  {4, 1024, (const void*)k_cg_brick<4, 1024>},
};
constexpr int kNumBrickKernels = sizeof(kBrickKernels) / sizeof(kBrickKernels[0]);

// Brick decomposition for the on-chip solver: bricks of nt columns
// (bx x by = nt) of q nodes along z for one of the instances above that tile
// the mesh exactly, whose padded copy and halo table fit `lds_max` bytes,
// whose published faces fit the space they reuse, and whose count fits the
// co-resident grid of that instance (per_cu workgroups per CU) and the
// reduction scratch.  Among those, the count closest
// to `target` (ties: smallest face area, then the longest x extent for
// coalesced rows) wins.  Returns false when none exists.
struct BrickChoice {
  int kernel, bd[3], nbr[3];
};
bool choose_bricks(const int nc[3], const int per_cu[], int ncu, size_t lds_max, int target,
                   BrickChoice& out) {
  bool found = false;
  long best_cost = 0;
  for (int ki = 0; ki < kNumBrickKernels; ++ki) {
    const int nt = kBrickKernels[ki].nt, bz = kBrickKernels[ki].q, m = nt * bz;
    if (nc[2] % bz) continue;
    for (int bx = 1; bx <= nc[0]; ++bx) {
      if (nc[0] % bx || nt % bx) continue;
      const int by = nt / bx;
      if (by > nc[1] || nc[1] % by) continue;
      const int bdv[3] = {bx, by, bz};
      if (brick_lds_bytes(bdv) > lds_max) continue;
      // published faces (6 per surface node) must fit the 9 nn doubles they reuse
      const long area = 2L * (bx * by + by * bz + bx * bz);
      if (2 * area > 3L * m) continue;
      int64_t nb = (int64_t)(nc[0] / bx) * (nc[1] / by) * (nc[2] / bz);
      if (nb > (int64_t)ncu * per_cu[ki] || nb > 1024) continue;
      long cost = std::labs((long)nb - target) * 1000000L + area * 100L + (100 - std::min(bx, 99));
      if (!found || cost < best_cost) {
        found = true;
        best_cost = cost;
        out.kernel = ki;
        out.bd[0] = bx; out.bd[1] = by; out.bd[2] = bz;
        out.nbr[0] = nc[0] / bx; out.nbr[1] = nc[1] / by; out.nbr[2] = nc[2] / bz;
      }
    }
  }
  return found;
}

}  // namespace

struct pic_ctx {
  SimConst K{};
  int precision = PIC_FP64;
  int device = 0;               // the GPU the context's memory and stream belong to
  int members = 1;              // ensemble members (replicates rep .. rep + members - 1)
  int64_t mstride = 0;          // workspace bytes per member
  double cg_tol = 1e-12;
  int cg_max_iter = 1000;
  hipStream_t stream = nullptr;
  int cg_grid = 1;
  bool cg_members_together = true;  // all members' solvers co-resident in one launch
  bool plain_cg_launch = false;     // ordinary instead of cooperative solver launches
  int cg_q = 0;                 // nodes per thread of the brick solver; 0 = global solver
  int cg_nt = kBlock;           // threads per workgroup of the solver
  const void* cg_fn = nullptr;  // the solver kernel
  int cg_bd[3] = {0, 0, 0};     // brick dimensions
  int cg_nbr[3] = {0, 0, 0};    // bricks per axis
  size_t cg_lds = 0;            // padded brick, bytes of LDS
  int low_k = 0;                // Fourier modes per axis solved exactly before the CG
  size_t low_lds[3] = {0, 0, 0};  // dynamic LDS of the three pre-solve passes
  bool count_zero = false;        // cell counts known to be zero (left so by the scan)
  bool mom_ready = false;         // cell moments of the current positions deposited by the sort
  bool heavy = false;           // collision calls by k_collide_heavy (many pairs per outcome)
  int heavy_bits = 0;           // its fixed-point scale
  double* angbuf = nullptr;     // scattering-angle records and their sort scratch
  int64_t angcap = 0;
  LowArgs low{};
  bool ready = false;
  int64_t step = 0;
  int cur = 0;
  std::string err;
  char* ws = nullptr;
  Layout layout{};
  double* x[2]{};
  double* v[2]{};
  double* sh[2]{};
  int* id[2]{};
  float* off[2]{};
  float* vf[2]{};
  float* asf[2]{};
  int *key{}, *slot{}, *tidx{}, *tkey{}, *count{}, *cstart{}, *bsum{}, *tile_c0{}, *tile_s0{};
  double *D{}, *U{}, *V0G{};
  float* Df{};
  bool fused = true;
  bool lean_pass = true;        // lean pass instance first, general one for the tiles it defers
  bool sort_events = false;     // mixed pass instances that sort long event lists
  // Captured steps (pic_use_graphs): two steps per graph, one graph per
  // double-buffer parity, recorded on a private stream and replayed on the
  // context's stream; kernels then take the step from *stepc.
  bool graphs = false, capturing = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  long long* stepc = nullptr;
  MixConst* mixc = nullptr;
  int* defer = nullptr;         // the deferred tiles (count, done, list)
  void* mom{};
  double *rho{}, *b{}, *phi{}, *E{}, *cgv{}, *lowbuf{}, *partA{}, *partB{};
  float* E32{};
  double *epart{}, *npart{}, *norms{}, *cgrr{}, *result{};
  unsigned* bar{};
  int *flags{}, *cgit{};
  unsigned long long* cnt{};
  // stage timing with HIP events on the context stream
  bool timing = false;
  uint32_t timing_mask = 0;  // stages timed while timing is on (bit 1 << stage)
  struct Timed {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
  double stage_ms[PIC_STAGE_COUNT] = {};
  int64_t stage_n[PIC_STAGE_COUNT] = {};
  ~pic_ctx() {
    for (auto& t : timed) event_pool.push_back(t.a), event_pool.push_back(t.b);
    for (auto e : event_pool) (void)hipEventDestroy(e);
    for (auto& g : gexec)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

// Calls that serve one simulation (caller buffers, state replacement,
// checkpoints) refuse ensemble contexts.
int single_only(pic_ctx* c, const char* what) {
  if (c->members == 1) return PIC_OK;
  c->err = std::string(what) + " serves single simulations; use the pic_ensemble_ calls";
  return PIC_EINVAL;
}

// Moves a member-0 workspace pointer to member m's slice.
template <class T>
T* member_ptr(const pic_ctx* c, T* p, int m) {
  return p ? (T*)((char*)p + (int64_t)m * c->mstride) : p;
}

// Launch grid with the ensemble members along z.
dim3 G(const pic_ctx* c, unsigned x, unsigned y = 1) { return dim3(x, y, (unsigned)c->members); }

int hip_fail(pic_ctx* c, hipError_t e, const char* what) {
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return PIC_EHIP;
}

#define HIP_TRY(ctx, call)                                 \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

#define LAUNCH_CHECK(ctx, name)                                     \
  do {                                                              \
    hipError_t e_ = hipGetLastError();                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, "launch " name); \
  } while (0)

#define TRY(expr)          \
  do {                     \
    int st_ = (expr);      \
    if (st_ != PIC_OK) return st_; \
  } while (0)

hipEvent_t take_event(pic_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records HIP events around one stage while timing is enabled.
struct StageTimer {
  pic_ctx* c;
  int stage;
  hipEvent_t a = nullptr;
  StageTimer(pic_ctx* ctx, int st) : c(ctx), stage(st) {
    if (!c->timing || !((c->timing_mask >> st) & 1u)) return;
    a = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
  }
  ~StageTimer() { stop(); }
  void stop() {
    if (!c->timing || !a) return;
    hipEvent_t b = take_event(c);
    if (b) {
      (void)hipEventRecord(b, c->stream);
      c->timed.push_back({stage, a, b});
    } else {
      c->event_pool.push_back(a);
    }
    a = nullptr;
  }
};

// Fold recorded event pairs into the per-stage totals (stream must be idle).
void collect_timing(pic_ctx* c) {
  for (auto& t : c->timed) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->stage_ms[t.stage] += ms;
      c->stage_n[t.stage] += 1;
    }
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->timed.clear();
}

template <class T>
T* carve(pic_ctx* c, int idx) {
  return c->layout.bytes[idx] ? reinterpret_cast<T*>(c->ws + c->layout.off[idx]) : nullptr;
}

template <class T>
int fill(pic_ctx* c, T* p, T v, int64_t n) {
  int g = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
  k_fill<T><<<G(c, g), kBlock, 0, c->stream>>>(p, v, n, c->mstride);
  LAUNCH_CHECK(c, "fill");
  return PIC_OK;
}

// Cell counts at zero before a counting pass; the scan leaves them there.
int zero_counts(pic_ctx* c) {
  if (!c->count_zero) TRY(fill<int>(c, c->count, 0, c->K.nn));
  c->count_zero = false;  // the counting pass that follows raises them
  return PIC_OK;
}

// Exclusive scan of the cell counts into cell_start; the counts are left at
// zero and the tile tables of the sorted order are written on the way.
int scan_counts(pic_ctx* c) {
  int n = c->K.nn;
  int nb = (n + kScanTile - 1) / kScanTile;
  TileInit ti;
  ti.c0 = c->tile_c0;
  ti.s0 = c->tile_s0;
  ti.ntiles = (int)((c->K.np + kTileB - 1) / kTileB);
  ti.ncell = n;
  ti.np = (int)c->K.np;
  k_scan_local<<<G(c, nb), kBlock, 0, c->stream>>>(c->count, c->cstart, c->bsum, n, ti, c->mstride);
  k_scan_blocks<<<G(c, 1), kBlock, 0, c->stream>>>(c->bsum, nb, c->cstart, n, c->mstride);
  k_scan_add<<<G(c, nb), kBlock, 0, c->stream>>>(c->cstart, c->bsum, n, c->count, ti, c->mstride);
  LAUNCH_CHECK(c, "scan");
  c->count_zero = true;
  return PIC_OK;
}

// Sort the current buffer (keys, slots and counts already computed) into the other.
int sort_particles(pic_ctx* c) {
  StageTimer tm(c, PIC_STAGE_SORT);
  TRY(scan_counts(c));
  int np = (int)c->K.np;
  k_scatter<<<G(c, (unsigned)(((int64_t)np + kBlock * kScatterPer - 1) / (kBlock * kScatterPer))),
              kBlock, 0, c->stream>>>(c->key, c->slot, c->cstart, c->tidx, c->tkey, np, c->mstride);
  int s = c->cur, d = 1 - c->cur;
  const int ntiles = (int)((c->K.np + kTileB - 1) / kTileB);
  // the fused step deposits each tile as it is moved (cell moments for the
  // field solve that follows)
  const bool dep = c->fused;
  if (c->precision == PIC_FP64) {
    auto kfn = dep ? k_order_tiles<double, true> : k_order_tiles<double, false>;
    kfn<<<G(c, ntiles), kTileThreads, 0, c->stream>>>(c->K, c->tile_c0, c->tile_s0, c->tidx, c->tkey,
                                                 c->cstart, c->x[s], c->v[s], c->sh[s], c->id[s],
                                                 c->x[d], c->v[d], c->sh[d], c->id[d], c->key,
                                                 (double*)c->mom, np, c->flags);
  } else {
    auto kfn = dep ? k_order_tiles<float, true> : k_order_tiles<float, false>;
    kfn<<<G(c, ntiles), kTileThreads, 0, c->stream>>>(c->K, c->tile_c0, c->tile_s0, c->tidx, c->tkey,
                                                 c->cstart, c->off[s], c->vf[s], c->asf[s],
                                                 c->id[s], c->off[d], c->vf[d], c->asf[d],
                                                 c->id[d], c->key, (float*)c->mom, np, c->flags);
  }
  c->mom_ready = dep;
  LAUNCH_CHECK(c, "sort");
  c->cur = d;
  return PIC_OK;
}

// deposit -> RHS (eq. poisson_mms, mean removed) -> CG (warm start) -> E = -grad phi
int field_solve(pic_ctx* c, double t) {
  const SimConst& K = c->K;
  int nbn = grid_for(K.nn);
  {
    StageTimer tm(c, PIC_STAGE_DEPOSIT);
    const int ntiles = (int)((K.np + kTileB - 1) / kTileB);
    const bool have_mom = c->mom_ready;  // deposited by the sort's move
    c->mom_ready = false;
    if (c->precision == PIC_FP64) {
      if (!have_mom && c->fused)
        k_deposit_tiles_f64<<<G(c, ntiles), kTileThreads, 0, c->stream>>>(K, c->x[c->cur], c->cstart,
                                                              c->tile_c0, (double*)c->mom);
      else if (!have_mom)
        k_deposit_moments_f64<<<nbn, kBlock, 0, c->stream>>>(K, c->x[c->cur], c->cstart,
                                                             (double*)c->mom);
      k_node_rhs<double><<<G(c, nbn), kBlock, 0, c->stream>>>(K, (const double*)c->mom, t, c->rho, c->b,
                                                        c->partA, c->capturing ? c->stepc : nullptr);
    } else {
      if (!have_mom && c->fused)
        k_deposit_tiles_mixed<<<G(c, ntiles), kTileThreads, 0, c->stream>>>(K, c->off[c->cur], c->cstart,
                                                                c->tile_c0, (float*)c->mom);
      else if (!have_mom)
        k_deposit_moments_mixed<<<nbn, kBlock, 0, c->stream>>>(K, c->off[c->cur], c->cstart,
                                                               (float*)c->mom);
      k_node_rhs_mixed<<<G(c, nbn), kBlock, 0, c->stream>>>(K, (const float*)c->mom, t, c->rho, c->b,
                                                      c->partA, c->capturing ? c->stepc : nullptr);
    }
    // also zeroes the solver's arrival flags and release word
    k_sub_mean<<<G(c, nbn), kBlock, 0, c->stream>>>(K, c->b, c->partA, nbn, c->bar,
                                              (c->cg_grid + 1) * kFlagStride);
    LAUNCH_CHECK(c, "rhs");
  }
  // the Poisson solve (low-mode pre-solve and CG) is timed as one stage
  StageTimer tm_solve(c, PIC_STAGE_CG);
  if (c->low_k > 0) {  // exact solve of the low Fourier modes of the residual
    const LowArgs& L = c->low;
    const int planes = L.slabs * K.nc[2];
    k_low_project<<<G(c, planes), kLowThreads, c->low_lds[0], c->stream>>>(K, L, c->b, c->phi);
    // four x chunks per y mode (the LDS sized for all nx columns bounds a chunk's)
    const dim3 gsolve = G(c, (unsigned)L.m[1], (unsigned)std::min(4, K.nc[0]));
    k_low_solve<<<gsolve, kLowThreads, c->low_lds[1], c->stream>>>(K, L);
    k_low_correct<<<G(c, planes), kLowThreads, c->low_lds[2], c->stream>>>(K, L, c->phi);
    LAUNCH_CHECK(c, "low-mode solve");
  }
  CgArgs a;
  a.b = c->b;
  a.x = c->phi;
  for (int k = 0; k < 2; ++k) {
    a.r[k] = c->cgv + (int64_t)k * K.nn;
    a.w[k] = c->cgv + (int64_t)(2 + k) * K.nn;
    a.s[k] = c->cgv + (int64_t)(4 + k) * K.nn;
  }
  a.p = c->cgv + 6 * (int64_t)K.nn;
  a.pub = c->cgv;  // the brick solver's face buffers reuse the global solver's vectors (9 nn)
  a.part = c->partA;
  a.result = c->result;
  a.arrive = c->bar;
  a.release = c->bar + (int64_t)c->cg_grid * kFlagStride;
  a.flags = c->flags;
  a.iters_out = c->cgit;
  a.relres_out = c->cgrr;
  a.tol = c->cg_tol;
  a.max_iter = c->cg_max_iter;
  for (int d = 0; d < 3; ++d) {
    a.bdim[d] = c->cg_bd[d];
    a.nbr[d] = c->cg_nbr[d];
  }
  SimConst Kc = K;
  void* args[] = {&Kc, &a};
  // The solver's workgroups wait for each other, so they must be co-resident:
  // a cooperative launch guarantees it.  With plain_cg_launch the grid (sized
  // at creation to fit by the occupancy query) is launched ordinarily; should
  // its workgroups not all be resident, the bounded barrier wait raises the
  // barrier flag instead of hanging.
  auto launch = [&](dim3 grid) {
    return (c->plain_cg_launch || c->capturing)
               ? hipLaunchKernel(c->cg_fn, grid, dim3(c->cg_nt), args, c->cg_lds, c->stream)
               : hipLaunchCooperativeKernel(c->cg_fn, grid, dim3(c->cg_nt), args, c->cg_lds,
                                            c->stream);
  };
  if (c->cg_members_together) {
    // every member's solver in one co-resident grid (members along z; each
    // member's bricks synchronise only among themselves)
    HIP_TRY(c, launch(G(c, c->cg_grid)));
  } else {
    for (int m = 0; m < c->members; ++m) {
      Kc.member0 = m;
      HIP_TRY(c, launch(dim3(c->cg_grid)));
    }
  }
  tm_solve.stop();
  StageTimer tm(c, PIC_STAGE_GRADIENT);
  k_gradient<<<G(c, nbn), kBlock, 0, c->stream>>>(K, c->phi, c->E, c->E32);
  LAUNCH_CHECK(c, "gradient");
  return PIC_OK;
}

int collide(pic_ctx* c, int call, int64_t step, double* D, long long* pairlog, int64_t cap) {
  const SimConst& K = c->K;
  StageTimer tm(c, PIC_STAGE_COLLIDE);
  if (c->heavy) {
    // workgroup per cell; the few cells beyond its capacity run one thread each
    k_collide_heavy<<<K.nn, 64 * kHeavyWaves, kHeavyLdsBytes, c->stream>>>(
        K, call, step, c->v[c->cur], c->cstart, D, c->heavy_bits, pairlog, cap, c->cnt, c->flags);
    LAUNCH_CHECK(c, "collide (heavy)");
    // (the sort's index arrays are idle here: marks and touched lists)
    const int sig = K.sigma_model == 0 ? kSigPoly : (K.omega == 1.0 ? kSigMaxwell : kSigHS);
    const double* vc = c->v[c->cur];
    if (sig == kSigHS)
      k_collide_big<kSigHS><<<grid_for(K.nn), kBlock, 0, c->stream>>>(
          K, call, step, vc, c->cstart, D, c->U, c->tidx, c->tkey, pairlog, cap, c->cnt, c->flags);
    else if (sig == kSigMaxwell)
      k_collide_big<kSigMaxwell><<<grid_for(K.nn), kBlock, 0, c->stream>>>(
          K, call, step, vc, c->cstart, D, c->U, c->tidx, c->tkey, pairlog, cap, c->cnt, c->flags);
    else
      k_collide_big<kSigPoly><<<grid_for(K.nn), kBlock, 0, c->stream>>>(
          K, call, step, vc, c->cstart, D, c->U, c->tidx, c->tkey, pairlog, cap, c->cnt, c->flags);
  } else {
    k_collide_f64<<<grid_for(K.nn), kBlock, 0, c->stream>>>(K, call, step, c->v[c->cur], c->cstart,
                                                            D, c->U, pairlog, cap, c->cnt, c->flags);
  }
  LAUNCH_CHECK(c, "collide");
  return PIC_OK;
}

int kick(pic_ctx* c, double t, double t_from, double t_to, double t_src) {
  const SimConst& K = c->K;
  StageTimer tm(c, PIC_STAGE_KICK);
  int s = c->cur;
  k_kick_f64<<<grid_for(K.np), kBlock, 0, c->stream>>>(K, t, t_from, t_to, t_src, c->x[s], c->v[s],
                                                       c->sh[s], c->id[s], c->key, c->cstart, c->E,
                                                       c->D);
  LAUNCH_CHECK(c, "kick");
  return PIC_OK;
}

int drift(pic_ctx* c, double t0, double th, double t1) {
  const SimConst& K = c->K;
  StageTimer tm(c, PIC_STAGE_DRIFT);
  TRY(zero_counts(c));
  int s = c->cur;
  k_drift_f64<<<grid_for(K.np), kBlock, 0, c->stream>>>(K, t0, th, t1, c->x[s], c->v[s], c->sh[s],
                                                        c->id[s], c->key, c->slot, c->count,
                                                        c->flags);
  LAUNCH_CHECK(c, "drift");
  return PIC_OK;
}

PartArgs part_args(pic_ctx* c) {
  PartArgs a;
  std::memset(&a, 0, sizeof(a));
  int s = c->cur;
  a.x = c->x[s];
  a.v = c->v[s];
  a.ash = c->sh[s];
  a.id = c->id[s];
  a.key = c->key;
  a.slot = c->slot;
  a.count = c->count;
  a.cstart = c->cstart;
  a.tile_c0 = c->tile_c0;
  a.tile_s0 = c->tile_s0;
  a.E = c->E;
  a.gv0 = c->V0G;
  a.gu = c->U;
  a.gD = c->D;
  a.gmark = c->tidx;  // the sort's index arrays are idle during the particle pass
  a.gtl = c->tkey;
  a.counters = c->cnt;
  a.flags = c->flags;
  a.defer = c->defer;
  a.mixc = c->mixc;
  a.ntiles = (int)((c->K.np + kTileB - 1) / kTileB);
  a.defer_list = 0;
  a.callB = 1;
  a.callA = 0;
  return a;
}

// A captured step's mixed-pass FP32 constants (one thread): nb = *stepc
// (call B and the end of that step), na = nb + 1, written for the pass to read.
__global__ void k_step_consts(SimConst K, PartArgs a, MixConst* out) {
  if (a.step_dev) {
    a.nb = *K.stepc;
    a.na = a.nb + 1;
  }
  *out = mix_const(K, a);
}
// The end of a captured step.
__global__ void k_step_advance(long long* stepc) { *stepc += 1; }

// Instances of the fused passes: the full one (angle and pair logs, the
// anisotropic samplers), the general lean one and the lean one that leaves
// the tiles it cannot run on lanes alone to the general one.
using MixedFn = void (*)(SimConst, MixConst, PartArgs, float*, float*, const float*, const float*);
using F64Fn = void (*)(SimConst, PartArgs);
struct PassFns {
  MixedFn mixed[3];      // full, general, fast
  MixedFn mixed_dev[3];  // (none), general, fast of captured steps
  F64Fn f64[3];
};
template <int FAM, int SIG, bool S>
PassFns pass_fns() {
  return {{k_particles_mixed<FAM, SIG, true, false>, k_particles_mixed<FAM, SIG, false, false, false, S>,
           k_particles_mixed<FAM, SIG, false, true, false, S>},
          {nullptr, k_particles_mixed<FAM, SIG, false, false, true, S>,
           k_particles_mixed<FAM, SIG, false, true, true, S>},
          {k_particles_f64<FAM, SIG, true, false>, k_particles_f64<FAM, SIG, false, false>,
           k_particles_f64<FAM, SIG, false, true>}};
}
template <int FAM, int SIG>
PassFns pass_fns(bool sort) {
  return sort ? pass_fns<FAM, SIG, true>() : pass_fns<FAM, SIG, false>();
}
// sort: the mixed instances that sort long event lists (sort_events)
PassFns select_pass(const SimConst& K, bool sort) {
  const int sig = K.sigma_model == 0 ? kSigPoly : (K.omega == 1.0 ? kSigMaxwell : kSigHS);
  if (K.family == 1) {
    if (sig == kSigHS) return pass_fns<1, kSigHS>(sort);
    if (sig == kSigMaxwell) return pass_fns<1, kSigMaxwell>(sort);
    return pass_fns<1, kSigPoly>(sort);
  }
  if (sig == kSigMaxwell) return pass_fns<0, kSigMaxwell>(sort);
  return pass_fns<0, kSigPoly>(sort);
}

// Workgroups of the general instance that works through the deferred tiles.
constexpr int kDeferGrid = 2048;

// Fused pass: the lean instance over all tiles, then the general one over the
// tiles it deferred; or the general (or full) instance alone, for logged runs,
// collide-only calls and collision loads where most tiles would be deferred.
int launch_particles(pic_ctx* c, const PartArgs& a0) {
  const SimConst& K = c->K;
  PartArgs a = a0;
  if (K.family == 0 && (a.mode & kDoA) && !(a.mode & kCollideOnly)) {
    // the paper family's manufactured drift term, into the idle half of the
    // double-buffered state (the next sort writes it again)
    const int o = 1 - c->cur;
    if (c->precision == PIC_MIXED) {
      a.mdrift32 = c->off[o];
      k_paper_drift_mixed<<<G(c, grid_for(K.np)), kBlock, 0, c->stream>>>(K, a, c->off[c->cur],
                                                                         c->off[o]);
    } else {
      a.mdrift = c->x[o];
      k_paper_drift_f64<<<G(c, grid_for(K.np)), kBlock, 0, c->stream>>>(K, a, c->x[o]);
    }
    LAUNCH_CHECK(c, "paper drift term");
  }
  const int tiles = (int)((K.np + kTileB - 1) / kTileB);
  const PassFns fns = select_pass(K, c->sort_events);
  // the collision-angle and pair-log recording and the anisotropic polar-angle
  // samplers are compiled only into the full instances
  const bool full = K.anglog != nullptr || a.pairlog != nullptr || K.chi_model != PIC_CHI_ISO ||
                    K.coding_error != 0;
  const bool lean = c->lean_pass && !full && !(a.mode & kCollideOnly);
  const int which = full ? 0 : 1;
  PartArgs ag = a;
  ag.defer_list = lean ? 1 : 0;
  const dim3 grid_general = G(c, lean ? std::min(tiles, kDeferGrid) : tiles);
  if (c->precision == PIC_MIXED) {
    const MixConst M = mix_const(K, a);  // (a captured step computes them on the device)
    const MixedFn* fm = fns.mixed;
    if (a.step_dev) {
      if (full) {
        c->err = "captured steps do not run the full pass instance";
        return PIC_EINVAL;
      }
      k_step_consts<<<1, 1, 0, c->stream>>>(K, a, c->mixc);
      LAUNCH_CHECK(c, "pass constants");
      fm = fns.mixed_dev;
    }
    const int s = c->cur;
    if (lean) {
      TRY(fill(c, c->defer, 0, 1));  // an empty deferral list
      fm[2]<<<G(c, tiles), dim3(kTileThreads), 0, c->stream>>>(K, M, a, c->off[s], c->vf[s],
                                                              c->asf[s], c->E32);
      LAUNCH_CHECK(c, "particles (mixed, lean)");
    }
    fm[which]<<<grid_general, dim3(kTileThreads), 0, c->stream>>>(K, M, ag, c->off[s], c->vf[s],
                                                                c->asf[s], c->E32);
    LAUNCH_CHECK(c, "particles (mixed)");
    return PIC_OK;
  }
  if (lean) {
    TRY(fill(c, c->defer, 0, 1));  // an empty deferral list
    fns.f64[2]<<<G(c, tiles), kTileThreads, 0, c->stream>>>(K, a);
    LAUNCH_CHECK(c, "particles (lean)");
  }
  fns.f64[which]<<<grid_general, kTileThreads, 0, c->stream>>>(K, ag);
  LAUNCH_CHECK(c, "particles");
  return PIC_OK;
}

int particle_pass(pic_ctx* c, int mode, int64_t nb, int64_t na) {
  const SimConst& K = c->K;
  StageTimer tm(c, PIC_STAGE_PARTICLE);
  if (mode & kDoA) TRY(zero_counts(c));
  PartArgs a = part_args(c);
  a.mode = mode;
  a.nb = nb;
  a.na = na;
  if (c->capturing) a.step_dev = 1;  // the step index from the device
  TRY(launch_particles(c, a));
  return PIC_OK;
}

// n_steps of eq. velocity_verlet with the fused particle pass: the pass after
// each field solve finishes step s (call B, kick 2) and starts step s + 1
// (call A, kick 1, drift).
// One inner iteration of the fused stepping: sort, field solve at t^{s+1},
// and the pass that finishes step s and starts step s + 1.
int inner_step(pic_ctx* c) {
  const int64_t s = c->step;
  TRY(sort_particles(c));
  TRY(field_solve(c, ((double)s + 1.0) * c->K.dt));
  TRY(particle_pass(c, kDoB | kDoA, s, s + 1));
  if (c->capturing) {
    k_step_advance<<<1, 1, 0, c->stream>>>(c->stepc);
    LAUNCH_CHECK(c, "step advance");
  }
  c->step = s + 1;
  return PIC_OK;
}

// Records two inner iterations into the graph of the current buffer parity.
// Nothing runs while recording; the host bookkeeping (buffer parity, flags)
// advances as the two iterations would, and is back where it started after
// them, so the graph replays from any even offset of that parity.
int capture_two_steps(pic_ctx* c) {
  const int par = c->cur;
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const hipStream_t user = c->stream;
  const int64_t step0 = c->step;
  c->stream = c->cap_stream;
  c->capturing = true;
  int rc = PIC_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = PIC_EHIP;
  } else {
    for (int i = 0; i < 2 && rc == PIC_OK; ++i) rc = inner_step(c);
    if (hipStreamEndCapture(c->cap_stream, &g) != hipSuccess && rc == PIC_OK) rc = PIC_EHIP;
  }
  c->capturing = false;
  c->stream = user;
  c->step = step0;
  if (rc == PIC_OK && c->cur != par) rc = PIC_EHIP;  // (the parity returns after two steps)
  if (rc == PIC_OK && hipGraphInstantiate(&c->gexec[par], g, nullptr, nullptr, 0) != hipSuccess)
    rc = PIC_EHIP;
  if (g) (void)hipGraphDestroy(g);
  if (rc != PIC_OK) {
    (void)hipGetLastError();
    c->err = "step capture failed";
  }
  return rc;
}

int fused_steps(pic_ctx* c, int n_steps) {
  if (n_steps <= 0) return PIC_OK;
  TRY(particle_pass(c, kDoA, 0, c->step));
  int inner = n_steps - 1;
  // (runs that need the full pass instance, the angle log, anisotropic
  // scattering or a coding error, step without graphs)
  const bool full = c->K.anglog != nullptr || c->K.chi_model != PIC_CHI_ISO || c->K.coding_error != 0;
  if (c->graphs && !c->timing && !full && inner >= 2) {
    // the device counter starts at the host's; each replay advances both by two
    TRY(fill<long long>(c, c->stepc, (long long)c->step, 1));
    while (inner >= 2) {
      if (!c->gexec[c->cur]) TRY(capture_two_steps(c));
      HIP_TRY(c, hipGraphLaunch(c->gexec[c->cur], c->stream));
      c->step += 2;
      inner -= 2;
    }
  }
  for (; inner > 0; --inner) TRY(inner_step(c));
  const int64_t s = c->step;
  TRY(sort_particles(c));
  TRY(field_solve(c, ((double)s + 1.0) * c->K.dt));
  TRY(particle_pass(c, kDoB, s, 0));
  c->step = s + 1;
  return PIC_OK;
}

// Recorded steps bake in the context's constants and launch choices: drop
// them whenever those change.
void drop_graphs(pic_ctx* c) {
  for (auto& g : c->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

int one_step(pic_ctx* c) {
  const SimConst& K = c->K;
  const int64_t n = c->step;
  const double t0 = (double)n * K.dt, th = ((double)n + 0.5) * K.dt, t1 = ((double)n + 1.0) * K.dt;
  if (K.collisions) TRY(collide(c, 0, n, c->D, nullptr, 0));
  TRY(kick(c, t0, t0, th, t0));
  TRY(drift(c, t0, th, t1));
  TRY(sort_particles(c));
  TRY(field_solve(c, t1));
  if (K.collisions) TRY(collide(c, 1, n, c->D, nullptr, 0));
  TRY(kick(c, t1, th, t1, th));
  c->step = n + 1;
  return PIC_OK;
}

// Read back flags raised by earlier asynchronous work.
int check_flags(pic_ctx* c) {
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int f[kFlagCount] = {0, 0, 0, 0};
  for (int m = 0; m < c->members; ++m) {
    int fm[kFlagCount];
    HIP_TRY(c, hipMemcpy(fm, (const char*)c->flags + (int64_t)m * c->mstride, sizeof(fm),
                         hipMemcpyDeviceToHost));
    for (int i = 0; i < kFlagCount; ++i) f[i] |= fm[i];
  }
  if (f[kFlagBarrier]) {
    c->err = "grid barrier timed out in the Poisson solver";
    return PIC_EHIP;
  }
  if (f[kFlagCgNoConv]) {
    c->err = "Poisson CG reached cg_max_iter before cg_tol";
    return PIC_ENOCONV;
  }
  if (f[kFlagCapacity]) {
    c->err = "degenerate state: a cell exceeded the stable-sort or pair-count bound";
    return PIC_ENONFINITE;
  }
  if (f[kFlagNonFinite]) {
    c->err = "non-finite particle state";
    return PIC_ENONFINITE;
  }
  return PIC_OK;
}

// PIC_WARN_GMAX once a candidate pair with g > g_max has been seen since
// initialisation (stream idle).
int gmax_warning(pic_ctx* c) {
  unsigned long long n = 0;
  for (int m = 0; m < c->members; ++m) {
    unsigned long long nm = 0;
    HIP_TRY(c, hipMemcpy(&nm, (const char*)(c->cnt + kCntGmax) + (int64_t)m * c->mstride,
                         sizeof(nm), hipMemcpyDeviceToHost));
    n += nm;
  }
  if (n > 0) {
    c->err = std::to_string(n) + " candidate pairs had a relative speed above g_max";
    return PIC_WARN_GMAX;
  }
  return PIC_OK;
}

}  // namespace

// Static scratch of pic_errors_noalloc: the error-norm partial sums and
// results (at most kErrBlocks x 14 particle partials, kErrBlocks x 2 node
// partials and 14 results, 131 KB).  Each GPU holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: only the address hipGetSymbolAddress returns for a device is
// used, in kernel arguments and copies.
constexpr int64_t kNoAllocScratchDoubles = (int64_t)kErrBlocks * 16 + 16;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch's device address on the context's GPU, looked up once per
// device with that device current.
int noalloc_scratch(pic_ctx* c, double** out) {
  if (c->device < 0 || c->device >= kMaxDevices) {
    c->err = "device index beyond the static scratch table";
    return PIC_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[c->device]) {
    int prev = 0;
    HIP_TRY(c, hipGetDevice(&prev));
    if (prev != c->device) HIP_TRY(c, hipSetDevice(c->device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != c->device) HIP_TRY(c, hipSetDevice(prev));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[c->device] = (double*)ptr;
  }
  *out = g_scratch_ptr[c->device];
  return PIC_OK;
}

// Workgroups of the error-norm kernels: one per 256 items, at most kErrBlocks.
int err_grid(int64_t n) { return (int)std::min<int64_t>(kErrBlocks, grid_for(n)); }

// Sec. 4.3 norms with the partial sums in epart ([err_grid(np)][14]), npart
// ([err_grid(nn)][2]) and the 14 results in norms (device; each member's in its
// own workspace slice); out holds one entry per member.
int errors_into(pic_ctx* c, pic_error_norms* out, double* epart, double* npart, double* norms) {
  if (!out) {
    c->err = "null output";
    return PIC_EINVAL;
  }
  const SimConst& K = c->K;
  double t = (double)c->step * K.dt;
  const int nbp = err_grid(K.np), nbn = err_grid(K.nn);
  int s = c->cur;
  if (c->precision == PIC_FP64)
    k_err_particles_f64<<<G(c, nbp), kBlock, 0, c->stream>>>(K, t, c->x[s], c->v[s], c->id[s], epart,
                                                       c->flags);
  else
    k_err_particles_mixed<<<G(c, nbp), kBlock, 0, c->stream>>>(K, t, c->key, c->off[s], c->vf[s],
                                                         c->id[s], epart, c->flags);
  k_err_nodes<<<G(c, nbn), kBlock, 0, c->stream>>>(K, t, c->phi, npart);
  k_err_final<<<G(c, 1), kBlock, 0, c->stream>>>(K, epart, nbp, npart, nbn, norms);
  LAUNCH_CHECK(c, "errors");
  TRY(check_flags(c));
  for (int m = 0; m < c->members; ++m) {
    double h[14];
    HIP_TRY(c, hipMemcpy(h, (const char*)norms + (int64_t)m * c->mstride, sizeof(h),
                         hipMemcpyDeviceToHost));
    out[m].t = t;
    for (int a = 0; a < 7; ++a) {
      out[m].l2[a] = h[a];
      out[m].linf[a] = h[7 + a];
      if (!std::isfinite(h[a]) || !std::isfinite(h[7 + a])) {
        c->err = "non-finite error norm";
        return PIC_ENONFINITE;
      }
    }
  }
  return gmax_warning(c);
}

}  // namespace

extern "C" {

int pic_workspace_size(const pic_problem* prob, const pic_discretization* disc, int precision,
                       int64_t* bytes) {
  std::string err;
  int st = validate(prob, disc, precision, err);
  if (st != PIC_OK) {
    g_create_error = err;
    return st;
  }
  if (!bytes) {
    g_create_error = "null bytes";
    return PIC_EINVAL;
  }
  *bytes = make_layout(disc, precision).total;
  return PIC_OK;
}

}  // extern "C"

namespace {

// A context of `members` simulations that differ only in the replicate
// (replicate + 0 .. members - 1), each in its own slice of the workspace.
int create(pic_ctx** out, const pic_problem* prob, const pic_discretization* disc, uint64_t seed,
           uint32_t replicate, int members, int precision, void* workspace, int64_t workspace_bytes,
           void* hip_stream) {
  if (!out) {
    g_create_error = "null output pointer";
    return PIC_EINVAL;
  }
  *out = nullptr;
  if (members < 1 || members > 65535) {
    g_create_error = "members must be in [1, 65535]";
    return PIC_EINVAL;
  }
  int64_t per = 0;
  int st = pic_workspace_size(prob, disc, precision, &per);
  if (st != PIC_OK) return st;
  const int64_t need = align_up(per) * members;
  if (!workspace || workspace_bytes < need) {
    g_create_error = "workspace too small: need " + std::to_string(need) + " bytes";
    return PIC_ESPACE;
  }
  if (((uintptr_t)workspace) % kAlign) {
    g_create_error = "workspace must be 256-byte aligned";
    return PIC_EINVAL;
  }
  pic_ctx* c = new (std::nothrow) pic_ctx();
  if (!c) {
    g_create_error = "out of host memory";
    return PIC_EINVAL;
  }
  c->K = derive(prob, disc, seed, replicate);
  c->precision = precision;
  c->members = members;
  c->mstride = align_up(per);
  c->K.mstride = c->mstride;
  {
    const char* e = std::getenv("PIC_UNFUSED");
    c->fused = !(e && e[0] == '1') || precision == PIC_MIXED;
    // Many candidate pairs per outcome at the mean cell occupancy (the paper's
    // refinement ladder): the FP64 form runs its collision calls with
    // k_collide_heavy in the separate-kernel step.  PIC_HEAVY=0/1 overrides.
    const double nbar = (double)disc->n_particles / ((double)disc->ncell[0] * disc->ncell[1] * disc->ncell[2]);
    const double pairs = nbar * (nbar - 1.0) * c->K.pmax / 2.0;
    bool heavy = precision == PIC_FP64 && c->K.collisions && (double)c->K.navg * pairs >= 64.0;
    if (const char* h = std::getenv("PIC_HEAVY")) heavy = precision == PIC_FP64 && h[0] == '1';
    if (heavy && hipFuncSetAttribute((const void*)k_collide_heavy,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kHeavyLdsBytes) != hipSuccess) {
      (void)hipGetLastError();
      heavy = false;
    }
    if (members > 1) {  // ensembles run the fused passes, whose kernels take members
      heavy = false;
      c->fused = true;
    }
    c->heavy = heavy;
    c->heavy_bits = heavy_scale_bits(c->K.g_max, c->K.navg);
    if (heavy) c->fused = false;
    // The lean pass runs a tile's outcomes on lanes only, which needs at most
    // kSmallPairs pairs per outcome and kPool records per call; expected pool
    // use per call of a tile is 2 N_pairs-mean N_avg (cells per tile).  Above
    // the pool most tiles would be deferred, so the general instance runs
    // alone.  PIC_LEAN_PASS=0/1 overrides.
    const double need = 2.0 * pairs * (double)c->K.navg * ((double)kTileB / std::max(nbar, 1.0));
    c->lean_pass = !c->K.collisions || need <= kPool;
    if (const char* lp = std::getenv("PIC_LEAN_PASS")) c->lean_pass = lp[0] == '1';
    // Events per call of a tile, N_avg (cells per tile) P(N_pairs > 0): the
    // mixed pass sorts its lists for the cell threads where they are long
    // (the FP64 pass always does).  PIC_SORT_EVENTS=0/1 overrides.
    const double events = (double)c->K.navg * ((double)kTileB / std::max(nbar, 1.0)) *
                          (1.0 - std::exp(-pairs));
    c->sort_events = c->K.collisions && events > 16.0;
    if (const char* se = std::getenv("PIC_SORT_EVENTS")) c->sort_events = se[0] == '1';
  }
  c->cg_tol = disc->cg_tol;
  c->cg_max_iter = disc->cg_max_iter;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->layout = make_layout(disc, precision);
  c->x[0] = carve<double>(c, A_X0);
  c->x[1] = carve<double>(c, A_X1);
  c->v[0] = carve<double>(c, A_V0);
  c->v[1] = carve<double>(c, A_V1);
  c->sh[0] = carve<double>(c, A_SH0);
  c->sh[1] = carve<double>(c, A_SH1);
  c->off[0] = carve<float>(c, A_OFF0);
  c->off[1] = carve<float>(c, A_OFF1);
  c->vf[0] = carve<float>(c, A_VF0);
  c->vf[1] = carve<float>(c, A_VF1);
  c->asf[0] = carve<float>(c, A_ASF0);
  c->asf[1] = carve<float>(c, A_ASF1);
  c->id[0] = carve<int>(c, A_ID0);
  c->id[1] = carve<int>(c, A_ID1);
  c->key = carve<int>(c, A_KEY);
  c->slot = carve<int>(c, A_SLOT);
  c->tidx = carve<int>(c, A_TIDX);
  c->tkey = carve<int>(c, A_TKEY);
  c->D = carve<double>(c, A_D);
  c->U = carve<double>(c, A_U);
  c->V0G = carve<double>(c, A_V0G);
  c->count = carve<int>(c, A_COUNT);
  c->cstart = carve<int>(c, A_CSTART);
  c->bsum = carve<int>(c, A_BSUM);
  c->tile_c0 = carve<int>(c, A_TILE);
  c->tile_s0 = c->tile_c0 + (c->K.np + kTileB - 1) / kTileB + 2;
  c->mom = carve<void>(c, A_MOM);
  c->rho = carve<double>(c, A_RHO);
  c->b = carve<double>(c, A_B);
  c->phi = carve<double>(c, A_PHI);
  c->E = carve<double>(c, A_E);
  c->E32 = carve<float>(c, A_E32);
  c->cgv = carve<double>(c, A_CGV);
  c->lowbuf = carve<double>(c, A_LOW);
  c->partA = carve<double>(c, A_PART_A);
  c->partB = carve<double>(c, A_PART_B);
  c->epart = carve<double>(c, A_EPART);
  c->npart = carve<double>(c, A_NPART);
  c->norms = carve<double>(c, A_NORMS);
  c->bar = carve<unsigned>(c, A_BAR);
  c->result = carve<double>(c, A_RESULT);
  c->flags = carve<int>(c, A_FLAGS);
  c->cnt = carve<unsigned long long>(c, A_CNT);
  c->cgit = carve<int>(c, A_CGIT);
  c->cgrr = carve<double>(c, A_CGRR);
  c->defer = carve<int>(c, A_DEFER);
  c->stepc = carve<long long>(c, A_STEPC);  // member 0's: one counter for all members
  c->mixc = carve<MixConst>(c, A_MIXC);
  c->K.stepc = c->stepc;

  // Cooperative grid for the Poisson solver: one block per CU at most, never
  // more than the node count needs, and never more than can be co-resident.
  int dev = 0, ncu = 1, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cg, kBlock, 0);
  if (e != hipSuccess || per_cu < 1) {
    g_create_error = std::string("device query failed: ") + hipGetErrorString(e);
    delete c;
    return PIC_EHIP;
  }
  c->device = dev;
  c->cg_grid = (int)std::min<int64_t>({(int64_t)ncu, (int64_t)ncu * per_cu, (int64_t)grid_for(c->K.nn)});
  // PIC_CG_BLOCKS sets the solver grid wanted (fewer blocks make each grid-wide
  // reduction cheaper and each sweep longer); it never exceeds the co-resident
  // bound.  The brick solver is used when the mesh splits into bricks that
  // fit; PIC_CG_GLOBAL=1 keeps the global-memory solver.
  // Default brick count: about 2,048 nodes per workgroup, between a quarter of
  // the CUs and all of them (at 64^3, 128 bricks measured 5 % faster per solve
  // than 256 and 20 % faster than 64: the grid-wide reduction's latency
  // against the sweep's length).
  int target = (int)std::min<int64_t>(c->cg_grid, std::max<int64_t>(ncu / 4, (int64_t)c->K.nn / 2048));
  if (const char* ev = std::getenv("PIC_CG_BLOCKS")) {
    int want = std::atoi(ev);
    if (want >= 1) {
      target = want;
      c->cg_grid = std::min(c->cg_grid, want);
    }
  }
  c->cg_fn = (const void*)k_cg;
  c->cg_nt = kBlock;
  const char* force_global = std::getenv("PIC_CG_GLOBAL");
  // (the brick solver's on-chip stencil is the 7-point one)
  if (!(force_global && std::atoi(force_global) == 1) && c->K.poisson_op == PIC_OP_FD7) {
    // co-resident workgroups per CU of each instance at its largest LDS use
    int lds_max = 65536;
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    lds_max = std::max(lds_max, 65536);
    // PIC_CG_INSTANCE="q,nt" restricts the choice to one solver instance
    int only_q = 0, only_nt = 0;
    if (const char* ev = std::getenv("PIC_CG_INSTANCE")) {
      if (std::sscanf(ev, "%d,%d", &only_q, &only_nt) != 2) only_q = only_nt = 0;
    }
    int per[kNumBrickKernels];
    for (int ki = 0; ki < kNumBrickKernels; ++ki) {
      per[ki] = 0;
      if (only_q && (kBrickKernels[ki].q != only_q || kBrickKernels[ki].nt != only_nt)) continue;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[ki], kBrickKernels[ki].fn,
                                                       kBrickKernels[ki].nt, 0) != hipSuccess)
        per[ki] = 0;
    }
    BrickChoice bc{};
    if (choose_bricks(c->K.nc, per, ncu, (size_t)lds_max, std::min(target, ncu), bc)) {
      const BrickKernel& bk = kBrickKernels[bc.kernel];
      const size_t lds = brick_lds_bytes(bc.bd);
      const int grid = bc.nbr[0] * bc.nbr[1] * bc.nbr[2];
      bool ok = true;
      if (lds > 65536)
        ok = hipFuncSetAttribute(bk.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
             hipSuccess;
      // the chosen instance must be co-resident at this grid with its LDS
      int occ = 0;
      if (ok && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, bk.fn, bk.nt, lds) != hipSuccess ||
                 (int64_t)occ * ncu < grid))
        ok = false;
      if (ok) {
        c->cg_q = bk.q;
        c->cg_nt = bk.nt;
        c->cg_fn = bk.fn;
        for (int d = 0; d < 3; ++d) {
          c->cg_bd[d] = bc.bd[d];
          c->cg_nbr[d] = bc.nbr[d];
        }
        c->cg_grid = grid;
        c->cg_lds = lds;
      }
    }
    (void)hipGetLastError();
  }
  {
    int occ = 0;
    c->cg_members_together =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, c->cg_fn, c->cg_nt, c->cg_lds) == hipSuccess &&
        (int64_t)occ * ncu >= (int64_t)c->cg_grid * members;
    (void)hipGetLastError();
    // PIC_CG_MEMBER_LAUNCHES=1: one solver launch per member even when all fit
    if (const char* ev = std::getenv("PIC_CG_MEMBER_LAUNCHES"))
      if (ev[0] == '1') c->cg_members_together = false;
    // PIC_CG_PLAIN_LAUNCH=1: ordinary launches of the solver (rocprofv3 ends in
    // a crash of its own at process exit after any cooperative launch)
    if (const char* ev = std::getenv("PIC_CG_PLAIN_LAUNCH")) c->plain_cg_launch = ev[0] == '1';
  }
  // PIC_CG_LOWMODES: Fourier modes per axis solved exactly before the CG (default
  // kLowDefaultK, at most kLowMaxK; 0 switches the pre-solve off).
  {
    int kl = kLowDefaultK;
    if (const char* ev = std::getenv("PIC_CG_LOWMODES")) kl = std::max(0, std::min(kLowMaxK, std::atoi(ev)));
    const int nmax = std::max({c->K.nc[0], c->K.nc[1], c->K.nc[2]});
    int lds_cap = 65536;
    (void)hipDeviceGetAttribute(&lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const void* fns[3] = {(const void*)k_low_project, (const void*)k_low_solve,
                          (const void*)k_low_correct};
    LowArgs& L = c->low;
    L.nmax = nmax;
    L.slabs = low_slabs(c->K.nc[1], c->K.nc[2], L.rows);
    double* base = c->lowbuf;
    L.tab = base;
    L.mu = base + 3 * kLowMaxM * nmax;
    L.t2 = base + 3 * kLowMaxM * nmax + 3 * kLowMaxM;
    L.e = L.t2 + (int64_t)L.slabs * kLowMaxM * kLowMaxM * c->K.nc[2];
    // fewer modes where a pass would exceed the LDS of a workgroup
    c->low_k = 0;
    for (; kl > 0 && c->low_k == 0; --kl) {
      for (int d = 0; d < 3; ++d) L.m[d] = 2 * std::min(kl, (c->K.nc[d] - 1) / 2) + 1;
      if (L.m[0] * L.m[1] * L.m[2] <= 1) break;
      c->low_lds[0] = (size_t)low_project_lds(L, c->K.nc[0]) * 8;
      c->low_lds[1] = (size_t)low_solve_lds(L, c->K.nc[0], c->K.nc[2]) * 8;
      c->low_lds[2] = (size_t)low_correct_lds(L, c->K.nc[0]) * 8;
      bool fits = true;
      for (int q = 0; q < 3 && fits; ++q) fits = c->low_lds[q] <= (size_t)lds_cap;
      for (int q = 0; q < 3 && fits; ++q)
        fits = hipFuncSetAttribute(fns[q], hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)c->low_lds[q]) == hipSuccess;
      (void)hipGetLastError();
      if (fits) c->low_k = kl;
    }
  }

  auto init = [&]() -> int {
    const SimConst& K = c->K;
    TRY(fill<int>(c, c->flags, 0, kFlagCount));
    TRY(fill<int>(c, c->defer, 0, 1));
    TRY(fill<unsigned long long>(c, c->cnt, 0ull, kCntCount));
    c->count_zero = false;
    TRY(zero_counts(c));
    TRY(fill<double>(c, c->phi, 0.0, K.nn));
    if (c->low_k > 0) {
      k_low_tables<<<G(c, grid_for((int64_t)3 * kLowMaxM * c->low.nmax)), kBlock, 0, c->stream>>>(
          K, c->low, (double*)c->low.tab, (double*)c->low.mu);
      LAUNCH_CHECK(c, "low-mode tables");
    }
    // unsorted initial state in buffer 1, sorted into buffer 0
    c->cur = 1;
    if (c->precision == PIC_FP64)
      k_init_f64<<<G(c, grid_for(K.np)), kBlock, 0, c->stream>>>(K, c->x[1], c->v[1], c->sh[1], c->id[1],
                                                           c->key, c->slot, c->count);
    else
      k_init_mixed<<<G(c, grid_for(K.np)), kBlock, 0, c->stream>>>(K, c->off[1], c->vf[1], c->asf[1],
                                                             c->id[1], c->key, c->slot, c->count);
    LAUNCH_CHECK(c, "init");
    TRY(sort_particles(c));
    TRY(field_solve(c, 0.0));
    return PIC_OK;
  };
  st = init();
  if (st != PIC_OK) {
    g_create_error = c->err;
    delete c;
    return st;
  }
  c->ready = true;
  c->step = 0;
  *out = c;
  if ((double)c->K.navg * c->K.pmax >= 0.5 && c->K.collisions) return PIC_WARN_NAVG;
  return PIC_OK;
}

}  // namespace

extern "C" {

int pic_init_manufactured(pic_ctx** out, const pic_problem* prob, const pic_discretization* disc,
                          uint64_t seed, uint32_t replicate, int precision, void* workspace,
                          int64_t workspace_bytes, void* hip_stream) {
  return create(out, prob, disc, seed, replicate, 1, precision, workspace, workspace_bytes,
                hip_stream);
}

int pic_ensemble_workspace_size(const pic_problem* prob, const pic_discretization* disc,
                                int precision, int members, int64_t* bytes) {
  if (members < 1 || members > 65535 || !bytes) {
    g_create_error = "members must be in [1, 65535] and bytes non-null";
    return PIC_EINVAL;
  }
  int64_t per = 0;
  const int st = pic_workspace_size(prob, disc, precision, &per);
  if (st != PIC_OK) return st;
  *bytes = align_up(per) * members;
  return PIC_OK;
}

int pic_ensemble_init(pic_ctx** out, const pic_problem* prob, const pic_discretization* disc,
                      uint64_t seed, uint32_t first_replicate, int members, int precision,
                      void* workspace, int64_t workspace_bytes, void* hip_stream) {
  return create(out, prob, disc, seed, first_replicate, members, precision, workspace,
                workspace_bytes, hip_stream);
}

int pic_step(pic_ctx* c, int n_steps) {
  if (!c || !c->ready) return PIC_ESTATE;
  if (n_steps < 0) {
    c->err = "n_steps must be >= 0";
    return PIC_EINVAL;
  }
  if (c->fused) return fused_steps(c, n_steps);
  for (int s = 0; s < n_steps; ++s) TRY(one_step(c));
  return PIC_OK;
}

int pic_collide(pic_ctx* c, int call, double t, double* dv_avg, double* dv_src, int64_t* pairlog,
                int64_t pairlog_cap, int64_t* pairlog_n) {
  if (!c || !c->ready) return PIC_ESTATE;
  TRY(single_only(c, "pic_collide"));
  if ((call != 0 && call != 1) || !dv_avg || !dv_src || pairlog_cap < 0 ||
      (pairlog_cap > 0 && !pairlog)) {
    c->err = "bad pic_collide arguments";
    return PIC_EINVAL;
  }
  const SimConst& K = c->K;
  TRY(fill<unsigned long long>(c, c->cnt + kCntPairLog, 0ull, 1));
  if (c->fused) {
    PartArgs a = part_args(c);
    a.mode = kCollideOnly;
    a.na = c->step;
    a.callA = call;
    a.tB = t;
    a.Dout = dv_avg;
    a.Sout = dv_src;
    a.pairlog = pairlog_cap > 0 ? (long long*)pairlog : nullptr;
    a.cap = pairlog_cap;
    TRY(launch_particles(c, a));
  } else {
    TRY(collide(c, call, c->step, dv_avg, pairlog_cap > 0 ? (long long*)pairlog : nullptr,
                pairlog_cap));
    k_source_f64<<<grid_for(K.np), kBlock, 0, c->stream>>>(K, c->v[c->cur], c->key, c->cstart, t,
                                                          dv_src);
    LAUNCH_CHECK(c, "source");
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (pairlog_n) {
    unsigned long long nlog = 0;
    HIP_TRY(c, hipMemcpy(&nlog, c->cnt + kCntPairLog, sizeof(nlog), hipMemcpyDeviceToHost));
    *pairlog_n = (int64_t)nlog;
  }
  TRY(check_flags(c));
  return gmax_warning(c);
}

int pic_errors(pic_ctx* c, pic_error_norms* out) {
  if (!c || !c->ready) return PIC_ESTATE;
  TRY(single_only(c, "pic_errors"));
  return errors_into(c, out, c->epart, c->npart, c->norms);
}

int pic_ensemble_errors(pic_ctx* c, pic_error_norms* out) {
  if (!c || !c->ready) return PIC_ESTATE;
  return errors_into(c, out, c->epart, c->npart, c->norms);
}

int pic_errors_noalloc(pic_ctx* c, pic_error_norms* out) {
  if (!c || !c->ready) return PIC_ESTATE;
  TRY(single_only(c, "pic_errors_noalloc"));
  const int npb = err_grid(c->K.np), nnb = err_grid(c->K.nn);
  const int64_t need = (int64_t)npb * 14 + (int64_t)nnb * 2 + 16;
  if (need > kNoAllocScratchDoubles) {
    c->err = "pic_errors_noalloc: the partial sums need " + std::to_string(need) +
             " doubles, more than the " + std::to_string(kNoAllocScratchDoubles) +
             " of the static scratch";
    return PIC_EINVAL;
  }
  double* s = nullptr;
  TRY(noalloc_scratch(c, &s));
  return errors_into(c, out, s, s + (int64_t)npb * 14, s + (int64_t)npb * 14 + (int64_t)nnb * 2);
}

namespace {
int64_t angle_pad(int64_t cap) {
  int64_t P = 1;
  while (P < cap) P <<= 1;
  return P;
}
}  // namespace

namespace {
// Checkpoint: a header, then the arrays that carry the state from one pic_step
// call to the next: the particle arrays of the current buffer (in their cell-
// sorted order), the cells and cell starts, the tile tables, the charge, the
// potential (the next solve's warm start), the nodal field and the counters.
struct CkptHeader {
  uint32_t magic, version;
  int32_t precision, cur;
  int64_t np, nn, step;
  uint64_t seed;
  uint32_t rep;
  int32_t navg;
  double dt;
};
constexpr uint32_t kCkptMagic = 0x31434950u;  // "PIC1"

int ckpt_arrays(const pic_ctx* c, int* a) {
  int n = 0;
  const int k = c->cur;
  if (c->precision == PIC_FP64) {
    a[n++] = k ? A_X1 : A_X0;
    a[n++] = k ? A_V1 : A_V0;
    a[n++] = k ? A_SH1 : A_SH0;
  } else {
    a[n++] = k ? A_OFF1 : A_OFF0;
    a[n++] = k ? A_VF1 : A_VF0;
    a[n++] = k ? A_ASF1 : A_ASF0;
    a[n++] = A_E32;
  }
  a[n++] = k ? A_ID1 : A_ID0;
  a[n++] = A_KEY;
  a[n++] = A_CSTART;
  a[n++] = A_TILE;
  a[n++] = A_RHO;
  a[n++] = A_PHI;
  a[n++] = A_E;
  a[n++] = A_CNT;
  return n;
}

int64_t ckpt_bytes(const pic_ctx* c) {
  int a[16];
  const int n = ckpt_arrays(c, a);
  int64_t t = sizeof(CkptHeader);
  for (int i = 0; i < n; ++i) t += c->layout.bytes[a[i]];
  return t;
}
}  // namespace

int pic_checkpoint_bytes(pic_ctx* c, int64_t* bytes) {
  if (!c || !c->ready) return PIC_ESTATE;
  if (!bytes) return PIC_EINVAL;
  *bytes = ckpt_bytes(c);
  return PIC_OK;
}

int pic_checkpoint_save(pic_ctx* c, void* host_dst, int64_t bytes) {
  if (!c || !c->ready) return PIC_ESTATE;
  TRY(single_only(c, "pic_checkpoint_save"));
  if (!host_dst || bytes != ckpt_bytes(c)) {
    c->err = "checkpoint save: buffer size must equal pic_checkpoint_bytes";
    return PIC_EINVAL;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  TRY(check_flags(c));
  CkptHeader h{kCkptMagic, 1u, c->precision, c->cur, c->K.np, (int64_t)c->K.nn, c->step,
               c->K.seed, c->K.rep, c->K.navg, c->K.dt};
  char* dst = (char*)host_dst;
  std::memcpy(dst, &h, sizeof(h));
  dst += sizeof(h);
  int a[16];
  const int n = ckpt_arrays(c, a);
  for (int i = 0; i < n; ++i) {
    HIP_TRY(c, hipMemcpy(dst, c->ws + c->layout.off[a[i]], c->layout.bytes[a[i]],
                         hipMemcpyDeviceToHost));
    dst += c->layout.bytes[a[i]];
  }
  return PIC_OK;
}

int pic_checkpoint_load(pic_ctx* c, const void* host_src, int64_t bytes) {
  if (c) drop_graphs(c);
  if (!c || !c->ready) return PIC_ESTATE;
  TRY(single_only(c, "pic_checkpoint_load"));
  if (!host_src || bytes < (int64_t)sizeof(CkptHeader)) {
    c->err = "checkpoint load: no header";
    return PIC_EINVAL;
  }
  CkptHeader h;
  std::memcpy(&h, host_src, sizeof(h));
  if (h.magic != kCkptMagic || h.version != 1u || h.precision != c->precision ||
      h.np != c->K.np || h.nn != (int64_t)c->K.nn || h.seed != c->K.seed || h.rep != c->K.rep ||
      h.navg != c->K.navg || h.dt != c->K.dt || (h.cur != 0 && h.cur != 1)) {
    c->err = "checkpoint load: the checkpoint belongs to another problem, seed or precision";
    return PIC_EINVAL;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->cur = h.cur;
  if (bytes != ckpt_bytes(c)) {
    c->err = "checkpoint load: size mismatch";
    return PIC_EINVAL;
  }
  const char* src = (const char*)host_src + sizeof(h);
  int a[16];
  const int n = ckpt_arrays(c, a);
  for (int i = 0; i < n; ++i) {
    HIP_TRY(c, hipMemcpy(c->ws + c->layout.off[a[i]], src, c->layout.bytes[a[i]],
                         hipMemcpyHostToDevice));
    src += c->layout.bytes[a[i]];
  }
  c->step = h.step;
  c->count_zero = false;
  c->mom_ready = false;
  return PIC_OK;
}

int64_t pic_angle_buffer_bytes(int64_t capacity) {
  if (capacity < 1) return 0;
  const int64_t P = angle_pad(capacity);
  return (2 * capacity + 2 * P + 4 * ((P + kBlock - 1) / kBlock) + 4) * (int64_t)sizeof(double);
}

int pic_angle_log(pic_ctx* c, void* buffer, int64_t capacity) {
  if (c) drop_graphs(c);  // the log selects another pass instance
  if (!c || !c->ready) return PIC_ESTATE;
  TRY(single_only(c, "pic_angle_log"));
  if (capacity < 0 || (capacity > 0 && !buffer)) {
    c->err = "angle log: a buffer is needed for a positive capacity";
    return PIC_EINVAL;
  }
  if (capacity > 0 && ((uintptr_t)buffer) % 256) {
    c->err = "angle log: buffer must be 256-byte aligned";
    return PIC_EINVAL;
  }
  c->angbuf = capacity > 0 ? (double*)buffer : nullptr;
  c->angcap = capacity;
  c->K.anglog = c->angbuf;
  c->K.angcap = capacity;
  TRY(fill<unsigned long long>(c, c->cnt + kCntAngles, 0ull, 1));
  return PIC_OK;
}

int pic_angle_errors(pic_ctx* c, double out[4], int64_t* n_records) {
  if (!c || !c->ready) return PIC_ESTATE;
  if (!out || !c->angbuf) {
    c->err = "angle errors: no angle log is enabled";
    return PIC_EINVAL;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  unsigned long long total = 0;
  HIP_TRY(c, hipMemcpy(&total, c->cnt + kCntAngles, sizeof(total), hipMemcpyDeviceToHost));
  if (n_records) *n_records = (int64_t)total;
  if ((int64_t)total > c->angcap) {
    c->err = "angle errors: more collisions than the angle log holds";
    return PIC_ESPACE;
  }
  const int64_t n = (int64_t)total, P = angle_pad(std::max<int64_t>(n, 1));
  if (n == 0) {
    for (int i = 0; i < 4; ++i) out[i] = 0.0;
    return check_flags(c);
  }
  double* u = c->angbuf + 2 * c->angcap;
  double* part = u + 2 * angle_pad(c->angcap);
  const int nb = (int)((P + kBlock - 1) / kBlock);
  double* res = part + 4 * ((angle_pad(c->angcap) + kBlock - 1) / kBlock);
  k_angle_map<<<nb, kBlock, 0, c->stream>>>(c->angbuf, n, P, c->K.chi_model, c->K.chi_alpha, u);
  for (int64_t k = 2; k <= P; k <<= 1)
    for (int64_t j = k >> 1; j > 0; j >>= 1)
      k_bitonic_stage<<<(int)((2 * P + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(u, P, k, j);
  k_angle_err<<<nb, kBlock, 0, c->stream>>>(u, n, P, part);
  k_angle_final<<<1, kBlock, 0, c->stream>>>(part, nb, n, res);
  LAUNCH_CHECK(c, "angle errors");
  HIP_TRY(c, hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return check_flags(c);
}

int pic_stats(pic_ctx* c, pic_stats_t* out) {
  if (!c || !c->ready) return PIC_ESTATE;
  if (!out) return PIC_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int it = 0;
  double rr = 0.0;
  unsigned long long cnt[kCntCount];
  HIP_TRY(c, hipMemcpy(&it, c->cgit, sizeof(it), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(&rr, c->cgrr, sizeof(rr), hipMemcpyDeviceToHost));
  for (int i = 0; i < kCntCount; ++i) cnt[i] = 0;
  for (int m = 0; m < c->members; ++m) {
    unsigned long long cm[kCntCount];
    HIP_TRY(c, hipMemcpy(cm, member_ptr(c, c->cnt, m), sizeof(cm), hipMemcpyDeviceToHost));
    for (int i = 0; i < kCntCount; ++i) cnt[i] += cm[i];
  }
  out->step = c->step;
  out->cg_iters = it;
  out->cg_relres = rr;
  out->n_accepted = (int64_t)cnt[kCntAccepted];
  out->n_gmax = (int64_t)cnt[kCntGmax];
  out->cg_blocks = c->cg_grid;
  for (int d = 0; d < 3; ++d) out->cg_brick[d] = c->cg_q ? c->cg_bd[d] : 0;
  out->cg_members_per_launch = c->cg_members_together ? c->members : 1;
  return check_flags(c);
}

}  // extern "C"

namespace {

int get_state_member(pic_ctx* c, int m, int item, void* host_dst, int64_t bytes) {
  if (!c || !c->ready) return PIC_ESTATE;
  if (m < 0 || m >= c->members) {
    c->err = "member index out of range";
    return PIC_EINVAL;
  }
  const SimConst& K = c->K;
  int64_t np = K.np, nn = K.nn;
  int64_t need;
  switch (item) {
    case PIC_STATE_X:
    case PIC_STATE_V: need = 3 * np * 8; break;
    case PIC_STATE_ID: need = np * 8; break;
    case PIC_STATE_CELL_START: need = (nn + 1) * 8; break;
    case PIC_STATE_RHO:
    case PIC_STATE_PHI: need = nn * 8; break;
    case PIC_STATE_E: need = 3 * nn * 8; break;
    default: c->err = "unknown state item"; return PIC_EINVAL;
  }
  if (!host_dst || bytes != need) {
    c->err = "destination size mismatch: need " + std::to_string(need);
    return PIC_EINVAL;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int s = c->cur;
  if (c->precision == PIC_MIXED && (item == PIC_STATE_X || item == PIC_STATE_V)) {
    double* U = member_ptr(c, c->U, m);
    k_export_mixed<<<grid_for(np), kBlock, 0, c->stream>>>(K, member_ptr(c, c->key, m),
                                                           member_ptr(c, c->off[s], m),
                                                           member_ptr(c, c->vf[s], m),
                                                           item == PIC_STATE_X ? U : nullptr,
                                                           item == PIC_STATE_V ? U : nullptr);
    LAUNCH_CHECK(c, "export");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(host_dst, U, need, hipMemcpyDeviceToHost));
    return check_flags(c);
  }
  switch (item) {
    case PIC_STATE_X: HIP_TRY(c, hipMemcpy(host_dst, member_ptr(c, c->x[s], m), need, hipMemcpyDeviceToHost)); break;
    case PIC_STATE_V: HIP_TRY(c, hipMemcpy(host_dst, member_ptr(c, c->v[s], m), need, hipMemcpyDeviceToHost)); break;
    case PIC_STATE_ID:
    case PIC_STATE_CELL_START: {
      const int* src = member_ptr(c, item == PIC_STATE_ID ? c->id[s] : c->cstart, m);
      int64_t n = need / 8;
      std::vector<int> tmp((size_t)n);
      HIP_TRY(c, hipMemcpy(tmp.data(), src, n * 4, hipMemcpyDeviceToHost));
      int64_t* d = (int64_t*)host_dst;
      for (int64_t i = 0; i < n; ++i) d[i] = tmp[(size_t)i];
      break;
    }
    case PIC_STATE_RHO: HIP_TRY(c, hipMemcpy(host_dst, member_ptr(c, c->rho, m), need, hipMemcpyDeviceToHost)); break;
    case PIC_STATE_PHI: HIP_TRY(c, hipMemcpy(host_dst, member_ptr(c, c->phi, m), need, hipMemcpyDeviceToHost)); break;
    case PIC_STATE_E: HIP_TRY(c, hipMemcpy(host_dst, member_ptr(c, c->E, m), need, hipMemcpyDeviceToHost)); break;
  }
  return check_flags(c);
}

}  // namespace

extern "C" {

int pic_get_state(pic_ctx* c, int item, void* host_dst, int64_t bytes) {
  return get_state_member(c, 0, item, host_dst, bytes);
}

int pic_ensemble_get_state(pic_ctx* c, int member, int item, void* host_dst, int64_t bytes) {
  return get_state_member(c, member, item, host_dst, bytes);
}

int pic_set_state(pic_ctx* c, int item, const void* host_src, int64_t bytes) {
  if (!c || !c->ready) return PIC_ESTATE;
  TRY(single_only(c, "pic_set_state"));
  if (item != PIC_STATE_X && item != PIC_STATE_V) {
    c->err = "pic_set_state: only PIC_STATE_X and PIC_STATE_V can be set";
    return PIC_EINVAL;
  }
  const SimConst& K = c->K;
  const int64_t need = 3 * K.np * 8;
  if (!host_src || bytes != need) {
    c->err = "source size mismatch: need " + std::to_string(need);
    return PIC_EINVAL;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int s = c->cur;
  if (item == PIC_STATE_V && c->precision == PIC_FP64) {
    HIP_TRY(c, hipMemcpy(c->v[s], host_src, need, hipMemcpyHostToDevice));
    return check_flags(c);
  }
  // staged in the workspace's FP64 scratch (idle between steps)
  HIP_TRY(c, hipMemcpy(c->U, host_src, need, hipMemcpyHostToDevice));
  if (item == PIC_STATE_V) {
    k_set_velocities_mixed<<<grid_for(K.np), kBlock, 0, c->stream>>>(K, c->U, c->vf[s]);
    LAUNCH_CHECK(c, "set velocities");
  } else {
    // new cells, stable re-sort from the current order, deposit and field solve
    // at the current time, as at initialisation
    TRY(zero_counts(c));
    if (c->precision == PIC_FP64)
      k_set_positions_f64<<<grid_for(K.np), kBlock, 0, c->stream>>>(K, c->U, c->x[s], c->key,
                                                                    c->slot, c->count, c->flags);
    else
      k_set_positions_mixed<<<grid_for(K.np), kBlock, 0, c->stream>>>(K, c->U, c->off[s], c->key,
                                                                      c->slot, c->count, c->flags);
    LAUNCH_CHECK(c, "set positions");
    c->mom_ready = false;
    TRY(sort_particles(c));
    TRY(field_solve(c, (double)c->step * K.dt));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return check_flags(c);
}

int pic_use_graphs(pic_ctx* c, int enable) {
  if (!c || !c->ready) return PIC_ESTATE;
  if (!c->fused) {
    c->err = "captured steps need the fused step (not PIC_UNFUSED, not the collision-heavy FP64 mode)";
    return PIC_EINVAL;
  }
  c->graphs = enable != 0;
  if (!c->graphs) drop_graphs(c);
  return PIC_OK;
}

int pic_timing_stages(pic_ctx* c, uint32_t mask) {
  if (!c || !c->ready) return PIC_ESTATE;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  collect_timing(c);
  for (int i = 0; i < PIC_STAGE_COUNT; ++i) {
    c->stage_ms[i] = 0.0;
    c->stage_n[i] = 0;
  }
  c->timing_mask = mask & ((1u << PIC_STAGE_COUNT) - 1u);
  c->timing = c->timing_mask != 0;
  return PIC_OK;
}

int pic_timing_enable(pic_ctx* c, int enable) {
  return pic_timing_stages(c, enable ? (1u << PIC_STAGE_COUNT) - 1u : 0u);
}

int pic_timing_read(pic_ctx* c, double* ms, int64_t* launches) {
  if (!c || !c->ready) return PIC_ESTATE;
  if (!ms || !launches) return PIC_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  collect_timing(c);
  for (int i = 0; i < PIC_STAGE_COUNT; ++i) {
    ms[i] = c->stage_ms[i];
    launches[i] = c->stage_n[i];
  }
  return PIC_OK;
}

void pic_destroy(pic_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* pic_last_error(const pic_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
