// Test harness: the library's particle kernels run on the CPU, one workgroup
// at a time, under the workgroup emulator (emu.hpp).  Three modes:
//   0  the fused particle kernel in its collide-only mode: one collision call
//      of Algorithm 1 averaged over N_avg outcomes and the manufactured source
//      for every particle of a cell-sorted state;
//   1  the fused particle pass of the FP64 form: call B of step s, the second
//      half kick, call A of step s + 1, the first half kick and the drift;
//   2  the same half step with the separate kernels (k_collide_f64,
//      k_kick_f64, k_drift_f64), which the fused pass must equal bit for bit.
//
// usage: particle_pass IN OUT
// IN  : pic_problem, pic_discretization, then the header below, then the
//       cell-sorted velocities v[3][np] (FP64), cell starts cs[nn + 1] (int32),
//       the cell of every particle key[np] (int32); modes 1 and 2 also
//       positions x[3][np], ids id[np] (int32) and the nodal field E[3][nn]
// OUT : mode 0: dv_avg[3][np], dv_src[3][np]; modes 1, 2: x[3][np], v[3][np],
//       key[np] (int32), count[nn] (int32); then counters[4] (uint64),
//       flags[4] (int32), the number of angle records (int64) and the records
//
// The tile tables are built from their definition (tile t holds the cells
// whose first particle lies in [t B, (t + 1) B)); everything else is the
// library's own code: the constants from pic_host.hpp and the kernels of
// pic_particle.hpp / pic_mixed.hpp.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hip/hip_runtime.h"
#include "pic_host.hpp"

using namespace pic;

struct Header {
  uint64_t seed;
  uint32_t rep, precision;  // 0 FP64, 1 mixed
  int64_t step;
  int32_t call, order;      // emu::Order
  double t;
  uint64_t rng_seed;
  int32_t full, mode;       // full: the instance with angle and pair logs
};

template <class T>
static void rd(FILE* f, T* p, size_t n) {
  if (std::fread(p, sizeof(T), n, f) != n) {
    std::fprintf(stderr, "short input\n");
    std::exit(2);
  }
}

template <class T>
static void wr(FILE* f, const T* p, size_t n) {
  if (std::fwrite(p, sizeof(T), n, f) != n) std::exit(3);
}

int main(int argc, char** argv) {
  if (argc != 3) return 1;
  FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 1;
  pic_problem prob;
  pic_discretization disc;
  Header h;
  rd(in, &prob, 1);
  rd(in, &disc, 1);
  rd(in, &h, 1);
  SimConst K = derive(&prob, &disc, h.seed, h.rep);
  const int64_t np = K.np;
  const int nn = K.nn;
  std::vector<double> v(3 * np);
  std::vector<int> cs(nn + 1), key(np);
  rd(in, v.data(), v.size());
  rd(in, cs.data(), cs.size());
  rd(in, key.data(), key.size());
  std::vector<double> x(3 * np, 0.0), E(3 * (size_t)nn, 0.0);
  std::vector<int> id(np);
  for (int64_t i = 0; i < np; ++i) id[i] = (int)i;
  if (h.mode != 0) {
    rd(in, x.data(), x.size());
    rd(in, id.data(), id.size());
    rd(in, E.data(), E.size());
  }
  std::fclose(in);
  // the time-independent velocity shape of every particle, as initialisation computes it
  std::vector<double> ash(3 * np);
  for (int64_t i = 0; i < np; ++i) {
    double xv[3], a3[3];
    velocity_uniforms(K, id[i], xv);
    velocity_shape(K, xv, a3);
    for (int d = 0; d < 3; ++d) ash[d * np + i] = a3[d];
  }

  const int ntiles = (int)((np + kTileB - 1) / kTileB);
  std::vector<int> tile_c0(ntiles + 2, nn), tile_s0(ntiles + 2, (int)np);
  for (int t = 0; t <= ntiles; ++t) {
    const int64_t want = (int64_t)t * kTileB;
    int c = (int)(std::lower_bound(cs.begin(), cs.end(), (int)std::min<int64_t>(want, np + 1)) - cs.begin());
    if (want > np || c > nn) continue;  // past the end: the scan's fill
    tile_c0[t] = c;
    tile_s0[t] = cs[c];
  }

  // global scratch and outputs, sized exactly (out-of-range accesses fault
  // under the address sanitizer)
  std::vector<double> gv0(3 * np), gu(3 * np), gD(3 * np), Dout(3 * np), Sout(3 * np);
  std::vector<int> gmark(np), gtl(np), slot(np), count(nn, 0);
  std::vector<unsigned long long> counters(kCntCount, 0);
  std::vector<int> flags(kFlagCount, 0);
  const int64_t angcap = 1 << 20;
  std::vector<double> angles(h.full ? 2 * angcap : 0);
  if (h.full) {
    K.anglog = angles.data();
    K.angcap = angcap;
  }
  std::vector<float> vf(3 * np), off(3 * np, 0.5f), ashf(3 * np, 0.0f), E32(3 * (size_t)nn, 0.0f);
  for (int64_t i = 0; i < 3 * np; ++i) vf[i] = (float)v[i];

  PartArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x.data();
  a.v = v.data();
  a.ash = ash.data();
  a.id = id.data();
  a.key = key.data();
  a.slot = slot.data();
  a.count = count.data();
  a.cstart = cs.data();
  a.tile_c0 = tile_c0.data();
  a.tile_s0 = tile_s0.data();
  a.E = E.data();
  a.gv0 = gv0.data();
  a.gu = gu.data();
  a.gD = gD.data();
  a.gmark = gmark.data();
  a.gtl = gtl.data();
  a.Dout = Dout.data();
  a.Sout = Sout.data();
  a.counters = counters.data();
  a.flags = flags.data();
  std::vector<int> defer(ntiles + 1, 0);
  int deferred = 0;
  a.defer = defer.data();
  a.ntiles = ntiles;
  a.defer_list = 0;
  if (h.mode == 0) {
    a.mode = kCollideOnly;
    a.na = h.step;
    a.callA = h.call;
    a.callB = 1;
    a.tB = h.t;
  } else {
    // modes 1 and 2: B then A; 3: A alone (the first pass of a pic_step call);
    // 4: B alone (its last pass)
    a.mode = h.mode == 3 ? kDoA : (h.mode == 4 ? kDoB : kDoB | kDoA);
    a.nb = h.step;
    a.na = h.mode == 3 ? h.step : h.step + 1;
    a.callB = 1;
    a.callA = 0;
  }

  const MixConst M = mix_const(K, a);
  std::mt19937_64 rng(h.rng_seed);
  // paper family: the drift's manufactured term, computed before the pass as
  // the library does (into a buffer of its own here)
  std::vector<double> mdrift;
  std::vector<float> mdrift32;
  if (K.family == 0 && (a.mode & kDoA) && !(a.mode & kCollideOnly) && h.mode != 2 && h.mode < 5) {
    const unsigned gp = (unsigned)((np + kBlock - 1) / kBlock);
    if (h.precision == 0) {
      mdrift.assign(3 * np, 0.0);
      a.mdrift = mdrift.data();
      emu::run_grid(gp, kBlock, [&] { k_paper_drift_f64(K, a, mdrift.data()); }, h.order, rng);
    } else {
      mdrift32.assign(3 * np, 0.0f);
      a.mdrift32 = mdrift32.data();
      emu::run_grid(gp, kBlock, [&] { k_paper_drift_mixed(K, a, off.data(), mdrift32.data()); },
                    h.order, rng);
    }
  }
  const int sig = K.sigma_model == 0 ? kSigPoly : (K.omega == 1.0 ? kSigMaxwell : kSigHS);
  // full: 1 the full instance alone; 0 the lean instance, then the general
  // one over the tiles it deferred (the library's default); 2 the general
  // lean instance alone
  std::function<void()> kern, kern_lean;
  PartArgs ag = a;
  ag.defer_list = h.full == 0 ? 1 : 0;
  if (h.precision == 0) {
    auto f64 = [&](auto kfull, auto kgen, auto kfast) {
      if (h.full == 1) kern = [&, kfull] { kfull(K, a); };
      else kern = [&, kgen] { kgen(K, ag); };
      kern_lean = [&, kfast] { kfast(K, a); };
    };
    if (K.family == 0 && sig == kSigPoly)
      f64(k_particles_f64<0, kSigPoly, true, false>, k_particles_f64<0, kSigPoly, false, false>,
          k_particles_f64<0, kSigPoly, false, true>);
    else if (K.family == 1 && sig == kSigHS)
      f64(k_particles_f64<1, kSigHS, true, false>, k_particles_f64<1, kSigHS, false, false>,
          k_particles_f64<1, kSigHS, false, true>);
    else
      return 4;
  } else {
    auto mixed = [&](auto kfull, auto kgen, auto kfast) {
      if (h.full == 1)
        kern = [&, kfull] { kfull(K, M, a, off.data(), vf.data(), ashf.data(), E32.data()); };
      else
        kern = [&, kgen] { kgen(K, M, ag, off.data(), vf.data(), ashf.data(), E32.data()); };
      kern_lean = [&, kfast] { kfast(K, M, a, off.data(), vf.data(), ashf.data(), E32.data()); };
    };
    if (K.family == 1 && sig == kSigHS)
      mixed(k_particles_mixed<1, kSigHS, true, false>, k_particles_mixed<1, kSigHS, false, false>,
            k_particles_mixed<1, kSigHS, false, true>);
    else if (K.family == 0 && sig == kSigPoly)
      mixed(k_particles_mixed<0, kSigPoly, true, false>, k_particles_mixed<0, kSigPoly, false, false>,
            k_particles_mixed<0, kSigPoly, false, true>);
    else
      return 4;
  }
  const bool lean = h.full == 0 && h.mode != 0;  // (collide-only runs the general instance)
  if (!lean) ag.defer_list = 0;
  if (h.mode == 5 || h.mode == 6) {
    // the separate kernels of an A-alone (5) or B-alone (6) pass
    if (h.precision != 0) return 4;
    std::vector<double> D(3 * np), U(3 * np);
    const int gn = (nn + kBlock - 1) / kBlock, gp = (int)((np + kBlock - 1) / kBlock);
    const double dt = K.dt, s = (double)h.step;
    auto collide = [&](int call, int64_t step) {
      emu::run_grid(gn, kBlock, [&] {
        k_collide_f64(K, call, step, v.data(), cs.data(), D.data(), U.data(), nullptr, 0,
                      counters.data(), flags.data());
      }, h.order, rng);
    };
    auto kick = [&](double t, double tf, double tt, double ts) {
      emu::run_grid(gp, kBlock, [&] {
        k_kick_f64(K, t, tf, tt, ts, x.data(), v.data(), ash.data(), id.data(), key.data(),
                   cs.data(), E.data(), D.data());
      }, h.order, rng);
    };
    if (h.mode == 5) {
      if (K.collisions) collide(0, h.step);
      kick(s * dt, s * dt, (s + 0.5) * dt, s * dt);
      emu::run_grid(gp, kBlock, [&] {
        k_drift_f64(K, s * dt, (s + 0.5) * dt, (s + 1.0) * dt, x.data(), v.data(), ash.data(),
                    id.data(), key.data(), slot.data(), count.data(), flags.data());
      }, h.order, rng);
    } else {
      if (K.collisions) collide(1, h.step);
      kick((s + 1.0) * dt, (s + 0.5) * dt, (s + 1.0) * dt, (s + 0.5) * dt);
    }
  } else if (h.mode == 2) {
    if (h.precision != 0) return 4;
    // the separate kernels of the same half step, as the unfused step runs them
    std::vector<double> D(3 * np), U(3 * np);
    const int gn = (nn + kBlock - 1) / kBlock, gp = (int)((np + kBlock - 1) / kBlock);
    const double dt = K.dt;
    const double thb = ((double)h.step + 0.5) * dt, t1b = ((double)h.step + 1.0) * dt;
    const double t0a = ((double)h.step + 1.0) * dt, tha = ((double)h.step + 1.5) * dt,
                 t1a = ((double)h.step + 2.0) * dt;
    auto collide = [&](int call, int64_t step) {
      emu::run_grid(gn, kBlock, [&] {
        k_collide_f64(K, call, step, v.data(), cs.data(), D.data(), U.data(), nullptr, 0,
                      counters.data(), flags.data());
      }, h.order, rng);
    };
    auto kick = [&](double t, double tf, double tt, double ts) {
      emu::run_grid(gp, kBlock, [&] {
        k_kick_f64(K, t, tf, tt, ts, x.data(), v.data(), ash.data(), id.data(), key.data(),
                   cs.data(), E.data(), D.data());
      }, h.order, rng);
    };
    if (K.collisions) collide(1, h.step);
    kick(t1b, thb, t1b, thb);
    if (K.collisions) collide(0, h.step + 1);
    kick(t0a, t0a, tha, t0a);
    emu::run_grid(gp, kBlock, [&] {
      k_drift_f64(K, t0a, tha, t1a, x.data(), v.data(), ash.data(), id.data(), key.data(),
                  slot.data(), count.data(), flags.data());
    }, h.order, rng);
  } else if (lean) {
    defer[0] = 0;  // the library clears the count before every lean launch
    emu::run_grid((unsigned)ntiles, kTileThreads, kern_lean, h.order, rng);
    deferred = defer[0];
    // the general instance over the deferred tiles, on fewer workgroups than
    // tiles so that each works through several; it only reads the list
    emu::run_grid((unsigned)std::max(1, std::min(ntiles, 7)), kTileThreads, kern, h.order, rng);
    if (defer[0] != deferred) return 5;
  } else {
    emu::run_grid((unsigned)ntiles, kTileThreads, kern, h.order, rng);
  }

  FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 1;
  if (h.mode == 0) {
    wr(out, Dout.data(), Dout.size());
    wr(out, Sout.data(), Sout.size());
  } else {
    wr(out, x.data(), x.size());
    wr(out, v.data(), v.size());
    wr(out, key.data(), key.size());
    wr(out, count.data(), count.size());
  }
  wr(out, counters.data(), counters.size());
  wr(out, flags.data(), flags.size());
  const int64_t nrec = h.full ? (int64_t)std::min<unsigned long long>(counters[kCntAngles], angcap) : 0;
  wr(out, &nrec, 1);
  if (nrec) wr(out, angles.data(), 2 * nrec);
  std::fclose(out);
  std::fprintf(stderr, "emu: %d tiles, %d deferred, %llu block barriers\n", ntiles, deferred,
               (unsigned long long)emu::g.barriers);
  return 0;
}
