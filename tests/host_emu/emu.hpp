// Workgroup emulator for running the library's kernels on the CPU (test
// harness only).  Each GPU thread of a workgroup is a fiber (ucontext); a
// fiber runs until it reaches a block barrier or a wave operation, where it
// yields to the scheduler.  The scheduler resumes the live fibers round by
// round in a chosen order (forward, reverse, or a fresh random permutation
// each round), so the code between two barriers of different threads runs in
// different interleavings from run to run: a result that depends on that
// order exposes a missing barrier or a race on shared memory.  A round in
// which no fiber makes progress is a deadlock (a barrier or wave operation
// that not every live thread reaches) and is reported.  Threads that have
// returned count as arrived, as exited waves do at a hardware barrier.
#pragma once

#include <ucontext.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <numeric>
#include <random>
#include <vector>

namespace emu {

struct Dim {
  unsigned x = 0, y = 0, z = 0;
};

inline Dim g_thread, g_block, g_blockdim, g_griddim;

enum Order { kForward = 0, kReverse = 1, kShuffle = 2 };

struct Fiber {
  ucontext_t ctx;
  std::vector<char> stack;
  bool done = false;
};

struct Wave {
  unsigned arrived = 0, gen = 0, live = 0;
  uint64_t buf[64];
};

struct State {
  std::vector<Fiber> fibers;
  std::vector<Wave> waves;
  ucontext_t sched;
  int cur = -1;
  unsigned live = 0, block_arrived = 0, block_gen = 0;
  bool progress = false, failed = false;
  const std::function<void()>* kernel = nullptr;
  uint64_t barriers = 0;
};
inline State g;

inline void fail(const char* what) {
  std::fprintf(stderr, "emu: %s (block %u, thread %u)\n", what, g_block.x, g_thread.x);
  std::abort();
}

inline void yield() { swapcontext(&g.fibers[g.cur].ctx, &g.sched); }

inline void flip_block() {
  g.block_arrived = 0;
  ++g.block_gen;
  g.progress = true;
}

inline void block_barrier() {
  const unsigned gen = g.block_gen;
  ++g.barriers;
  if (++g.block_arrived == g.live) flip_block();
  while (g.block_gen == gen) yield();
  g.progress = true;
}

inline Wave& my_wave() { return g.waves[g_thread.x / 64]; }

inline void flip_wave(Wave& W) {
  W.arrived = 0;
  ++W.gen;
  g.progress = true;
}

inline void wave_barrier(Wave& W) {
  const unsigned gen = W.gen;
  if (++W.arrived == W.live) flip_wave(W);
  while (W.gen == gen) yield();
  g.progress = true;
}

inline unsigned long long wave_ballot(bool p) {
  Wave& W = my_wave();
  const unsigned lane = g_thread.x & 63u;
  W.buf[lane] = p ? 1 : 0;
  wave_barrier(W);
  unsigned long long m = 0;
  const unsigned base = g_thread.x & ~63u;
  for (unsigned i = 0; i < 64 && base + i < g_blockdim.x; ++i)
    if (!g.fibers[base + i].done && W.buf[i]) m |= 1ull << i;
  wave_barrier(W);
  return m;
}

template <class T>
inline T wave_shfl(T v, int src) {
  static_assert(sizeof(T) <= 8, "wave_shfl moves at most 8 bytes");
  Wave& W = my_wave();
  const unsigned lane = g_thread.x & 63u, base = g_thread.x & ~63u;
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  W.buf[lane] = u;
  wave_barrier(W);
  const unsigned s = (unsigned)src & 63u;
  if (base + s >= g_blockdim.x || g.fibers[base + s].done) fail("shuffle from an inactive lane");
  T r;
  std::memcpy(&r, &W.buf[s], sizeof(T));
  wave_barrier(W);
  return r;
}

inline void fiber_entry() {
  g.progress = true;
  (*g.kernel)();
  Fiber& f = g.fibers[g.cur];
  f.done = true;
  g.progress = true;
  --g.live;
  Wave& W = my_wave();
  --W.live;
  // an exited thread no longer holds back the barriers it would have reached
  if (W.arrived > 0 && W.arrived == W.live) flip_wave(W);
  if (g.block_arrived > 0 && g.block_arrived == g.live) flip_block();
}

// Runs one workgroup of nthreads threads of `kernel` with the given order.
inline void run_block(unsigned nthreads, const std::function<void()>& kernel, int order,
                      std::mt19937_64& rng, size_t stack_bytes = 256u << 10) {
  if (g.fibers.size() != nthreads) {
    g.fibers.clear();
    g.fibers.resize(nthreads);
  }
  g.waves.assign((nthreads + 63) / 64, Wave{});
  for (unsigned w = 0; w < g.waves.size(); ++w) g.waves[w].live = std::min(64u, nthreads - 64 * w);
  g.kernel = &kernel;
  g.live = nthreads;
  g.block_arrived = 0;
  g.block_gen = 0;
  g_blockdim = Dim{nthreads, 1, 1};
  for (unsigned i = 0; i < nthreads; ++i) {
    Fiber& f = g.fibers[i];
    f.done = false;
    if (f.stack.size() != stack_bytes) f.stack.assign(stack_bytes, 0);
    getcontext(&f.ctx);
    f.ctx.uc_stack.ss_sp = f.stack.data();
    f.ctx.uc_stack.ss_size = f.stack.size();
    f.ctx.uc_link = &g.sched;
    makecontext(&f.ctx, fiber_entry, 0);
  }
  std::vector<int> ord(nthreads);
  std::iota(ord.begin(), ord.end(), 0);
  if (order == kReverse) std::reverse(ord.begin(), ord.end());
  while (g.live > 0) {
    if (order == kShuffle) std::shuffle(ord.begin(), ord.end(), rng);
    g.progress = false;
    for (int i : ord) {
      if (g.fibers[i].done) continue;
      g.cur = i;
      g_thread = Dim{(unsigned)i, 0, 0};
      swapcontext(&g.sched, &g.fibers[i].ctx);
    }
    if (!g.progress && g.live > 0) fail("deadlock: a barrier that not every live thread reaches");
  }
}

// Runs a grid of nblocks workgroups one after another.
inline void run_grid(unsigned nblocks, unsigned nthreads, const std::function<void()>& kernel,
                     int order, std::mt19937_64& rng) {
  g_griddim = Dim{nblocks, 1, 1};
  std::vector<unsigned> blocks(nblocks);
  std::iota(blocks.begin(), blocks.end(), 0u);
  if (order == kReverse) std::reverse(blocks.begin(), blocks.end());
  if (order == kShuffle) std::shuffle(blocks.begin(), blocks.end(), rng);
  for (unsigned b : blocks) {
    g_block = Dim{b, 0, 0};
    run_block(nthreads, kernel, order, rng);
  }
}

}  // namespace emu
