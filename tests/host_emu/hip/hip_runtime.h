// Host stand-in for <hip/hip_runtime.h>, used only by the test harness that
// runs the library's device code on the CPU (tests/host_emu).  It maps the
// HIP keywords to plain C++ and the intrinsics the kernels use to the
// workgroup emulator in emu.hpp: every GPU thread of a workgroup is a fiber,
// __syncthreads() and the wave operations are barriers of the emulator, and
// atomics are plain read-modify-writes (one fiber runs at a time).
#pragma once

#include <math.h>
#include <stdint.h>

#include <cmath>
#include <cstring>

#include "../emu.hpp"

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __shared__ static
#define __launch_bounds__(...)

#define threadIdx (::emu::g_thread)
#define blockIdx (::emu::g_block)
#define blockDim (::emu::g_blockdim)
#define gridDim (::emu::g_griddim)

inline void __syncthreads() { ::emu::block_barrier(); }
inline int __lane_id() { return (int)(::emu::g_thread.x & 63u); }
inline unsigned long long __ballot(int pred) { return ::emu::wave_ballot(pred != 0); }
template <class T> inline T __shfl(T v, int src) { return ::emu::wave_shfl(v, src); }
template <class T> inline T __shfl_xor(T v, int mask) {
  return ::emu::wave_shfl(v, __lane_id() ^ mask);
}
inline int __ffsll(long long v) { return v ? __builtin_ctzll((unsigned long long)v) + 1 : 0; }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline uint64_t __umul64hi(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

template <class T, class U> inline T atomicAdd(T* p, U v) {
  T old = *p;
  *p = old + (T)v;
  return old;
}
template <class T, class U> inline T atomicOr(T* p, U v) {
  T old = *p;
  *p = old | (T)v;
  return old;
}

// memory-model builtins of the Poisson solver (not run by the harness)
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __hip_atomic_load(p, order, scope) (*(p))
#define __hip_atomic_store(p, v, order, scope) (*(p) = (v))
#define __builtin_amdgcn_fence(order, scope) ((void)0)
inline void __threadfence() {}
#define __builtin_amdgcn_s_sleep(n) ((void)0)

// device math with no standard C++ counterpart
inline double emu_sinpi(double x) { return std::sin(M_PI * x); }
inline double emu_cospi(double x) { return std::cos(M_PI * x); }
inline void emu_sincospi(double x, double* s, double* c) {
  *s = std::sin(M_PI * x);
  *c = std::cos(M_PI * x);
}
inline void emu_sincospif(float x, float* s, float* c) {
  *s = std::sin((float)M_PI * x);
  *c = std::cos((float)M_PI * x);
}
#define sinpi emu_sinpi
#define cospi emu_cospi
#define sincospif emu_sincospif
#define sincospi emu_sincospi

template <class A, class B> inline auto min(A a, B b) -> decltype(a < b ? a : b) {
  return a < b ? a : b;
}
template <class A, class B> inline auto max(A a, B b) -> decltype(a < b ? a : b) {
  return a < b ? b : a;
}
