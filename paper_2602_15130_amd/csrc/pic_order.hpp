// The move of the sort, optionally with the deposit of the moved tile.
#pragma once

#include <type_traits>

#include "pic_mixed.hpp"

namespace pic {

// Stable in-cell order by cell-aligned tiles: a tile's slots (the sort's
// scatter slots of its cells) load their source indices into LDS; each
// slot's rank among the source indices of its own cell, which is its place in
// the stable order, is counted in LDS, and the particle's state moves from its
// source to (cell start) + rank.  Same destinations as order_dst; tiles larger
// than the LDS slots use order_dst itself.  Every global load a slot needs
// (source index, cell, cell bounds, the state itself) is issued before the
// block waits for the LDS copy, so a tile costs two dependent load rounds.
//
// DEP: the same workgroup then deposits its tile: the eight cloud-in-cell
// weights of each moved particle go to LDS at its sorted place, and one lane
// per (cell, corner) sums its cell's weights in sorted order -- the sums of
// k_deposit_tiles_f64 / k_deposit_tiles_mixed, bit for bit, without reading
// the positions back.  T = double: absolute FP64 positions, moments in FP64;
// T = float: FP32 in-cell offsets, moments with Neumaier compensation.
template <class T, bool DEP>
__global__ void __launch_bounds__(kTileThreads) k_order_tiles(SimConst K, const int* tile_c0,
                                                              const int* tile_s0, const int* tidx,
                                                              const int* tkey, const int* cstart,
                                                              const T* xs, const T* vs,
                                                              const T* as, const int* ids, T* xd,
                                                              T* vd, T* ad, int* idd, int* keyd,
                                                              T* mom, int n, int* flags) {
  tile_c0 = mem(K, tile_c0);
  tile_s0 = mem(K, tile_s0);
  tidx = mem(K, tidx);
  tkey = mem(K, tkey);
  cstart = mem(K, cstart);
  xs = mem(K, xs);
  vs = mem(K, vs);
  as = mem(K, as);
  ids = mem(K, ids);
  xd = mem(K, xd);
  vd = mem(K, vd);
  ad = mem(K, ad);
  idd = mem(K, idd);
  keyd = mem(K, keyd);
  mom = mem(K, mom);
  flags = mem(K, flags);
  constexpr int kPer = (kLdsSlots + kTileThreads - 1) / kTileThreads;
  __shared__ int lidx[kLdsSlots];
  __shared__ T W[DEP ? 8 * kLdsSlots : 1];
  const int s0 = tile_s0[blockIdx.x], ns = tile_s0[blockIdx.x + 1] - s0;
  if (ns <= 0) return;
  const bool lds = ns <= kLdsSlots;
  if (!lds) {
    for (int j = threadIdx.x; j < ns; j += kTileThreads) {
      const int slot = s0 + j, my = tidx[slot];
      const int dst = order_dst(tidx, tkey, cstart, slot, flags);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        xd[(int64_t)d * n + dst] = xs[(int64_t)d * n + my];
        vd[(int64_t)d * n + dst] = vs[(int64_t)d * n + my];
        ad[(int64_t)d * n + dst] = as[(int64_t)d * n + my];
      }
      idd[dst] = ids[my];
      keyd[dst] = tkey[slot];
    }
    if (!DEP) return;
    __threadfence_block();  // the tile's moved positions, read back below
    __syncthreads();
  } else {
    int my[kPer], cc[kPer], cs[kPer], ce[kPer], idv[kPer];
    T sv[kPer][9];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = threadIdx.x + q * kTileThreads;
      if (j < ns) {
        my[q] = tidx[s0 + j];
        cc[q] = tkey[s0 + j];
      }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = threadIdx.x + q * kTileThreads;
      if (j < ns) {
        lidx[j] = my[q];
        cs[q] = cstart[cc[q]] - s0;
        ce[q] = cstart[cc[q] + 1] - s0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          sv[q][d] = xs[(int64_t)d * n + my[q]];
          sv[q][3 + d] = vs[(int64_t)d * n + my[q]];
          sv[q][6 + d] = as[(int64_t)d * n + my[q]];
        }
        idv[q] = ids[my[q]];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = threadIdx.x + q * kTileThreads;
      if (j < ns) {
        int r = 0;
        for (int k = cs[q]; k < ce[q]; ++k) r += lidx[k] < my[q];
        const int dst = s0 + cs[q] + r;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          xd[(int64_t)d * n + dst] = sv[q][d];
          vd[(int64_t)d * n + dst] = sv[q][3 + d];
          ad[(int64_t)d * n + dst] = sv[q][6 + d];
        }
        idd[dst] = idv[q];
        keyd[dst] = cc[q];
        if constexpr (DEP) {
          T w[8];
          if constexpr (std::is_same<T, float>::value) {
            const float o[3] = {sv[q][0], sv[q][1], sv[q][2]};
            cic_weights_mixed(o, w);
          } else {
            const double xp[3] = {sv[q][0], sv[q][1], sv[q][2]};
            cic_weights_f64(K, xp, w);
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) W[k * kLdsSlots + (dst - s0)] = w[k];
        }
      }
    }
    if (!DEP) return;
    __syncthreads();
  }
  if constexpr (DEP) {
    // the tile's cells: the first cell of this tile up to the first of the next
    const int c0 = min(tile_c0[blockIdx.x], K.nn);
    const int c1 = min(max(tile_c0[blockIdx.x + 1], c0), K.nn);
    for (int l = threadIdx.x; l < 8 * (c1 - c0); l += kTileThreads) {
      const int k = l & 7, c = c0 + (l >> 3);
      const int a = cstart[c] - s0, e = cstart[c + 1] - s0;
      if constexpr (std::is_same<T, float>::value) {
        float sum = 0.0f, comp = 0.0f;
        for (int j = a; j < e; ++j) {
          float wk;
          if (lds) {
            wk = W[k * kLdsSlots + j];
          } else {
            const int p = s0 + j;
            float o[3] = {xd[p], xd[n + p], xd[2 * (int64_t)n + p]}, w[8];
            cic_weights_mixed(o, w);
            wk = w[k];
          }
          neumaier_add(sum, comp, wk);
        }
        mom[(int64_t)k * K.nn + c] = sum;
        mom[(int64_t)(8 + k) * K.nn + c] = comp;
      } else {
        double m = 0.0;
        for (int j = a; j < e; ++j) {
          if (lds) {
            m += W[k * kLdsSlots + j];
          } else {
            const int p = s0 + j;
            double xp[3] = {xd[p], xd[n + p], xd[2 * (int64_t)n + p]}, w[8];
            cic_weights_f64(K, xp, w);
            m += w[k];
          }
        }
        mom[(int64_t)k * K.nn + c] = m;
      }
    }
  }
}

}  // namespace pic
