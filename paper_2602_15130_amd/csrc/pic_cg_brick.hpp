// Poisson CG with the iterate held on chip: the same single-reduction
// recurrence as k_cg (A = -L_h, A phi = -b, Chronopoulos and Gear), with the
// mesh split into bricks of bdim[0] x bdim[1] x bdim[2] nodes, one brick per
// persistent block.  A thread owns Q nodes of its brick and keeps x, r, w, s
// and p of those nodes in registers for the whole solve; the stencil reads
// r_{i+1} from a padded LDS copy of the brick.  Only the brick faces travel
// through global memory: after each sweep a block publishes w on its six faces
// into a packed per-brick buffer (ping-pong by iteration parity; r_0 once at
// the start), and the next sweep rebuilds the neighbours' r_{i+1} on the
// one-node halo with their owner's recurrence, s_i = w_i + beta s_{i-1},
// r_{i+1} = r_i - alpha s_i, from the published w_i and the halo's r_i and
// s_{i-1} kept in LDS: the same operations on the same values (no contraction
// into FMA), so the halo holds the owners' bits, and one grid-wide reduction
// per iteration is still the only synchronisation.  Per iteration a block
// moves (face nodes) x 8 bytes each way, in contiguous runs, instead of 80
// bytes per node.
//
// Published faces: pub[((brick * 2 + parity) * 3 + array) * nh + slot], array
// 0 = r (r_0 only), 1 = w, 2 unused; slots of face f start at foff[f] with faces ordered
// -x, +x, -y, +y, -z, +z; within an x face the slot is lj + by lk, within a y
// face li + bx lk, within a z face li + bx lj.  The halo uses the same order,
// so halo slot h of one brick reads slot h of the opposite face of the
// neighbour across it.
#pragma once

#include "pic_kernels.hpp"

namespace pic {

// Padded-brick stencil: (-L f) at padded index c with the same association as
// neg_lap.
__device__ inline double neg_lap_pad(const SimConst& K, const double* R, int c, int px, int pxy) {
  double v = R[c];
  double lx = R[c + 1] - 2.0 * v + R[c - 1];
  double ly = R[c + px] - 2.0 * v + R[c - px];
  double lz = R[c + pxy] - 2.0 * v + R[c - pxy];
  return -(lx * K.ih2[0] + ly * K.ih2[1] + lz * K.ih2[2]);
}

// Halo node h of a brick at origin (ox, oy, oz): its padded index and global
// node.  Halo nodes are the face neighbours only (the stencil has no edge or
// corner terms), ordered -x, +x, -y, +y, -z, +z.
__device__ inline void brick_halo(const SimConst& K, const int bd[3], int ox, int oy, int oz, int h,
                                  int& pidx, int& gidx) {
  const int bx = bd[0], by = bd[1], bz = bd[2];
  const int fx = by * bz, fy = bx * bz, fz = bx * by;
  int li, lj, lk;
  if (h < 2 * fx) {
    int hi = h >= fx, e = h - hi * fx;
    lj = e % by;
    lk = e / by;
    li = hi ? bx : -1;
  } else if (h < 2 * fx + 2 * fy) {
    h -= 2 * fx;
    int hi = h >= fy, e = h - hi * fy;
    li = e % bx;
    lk = e / bx;
    lj = hi ? by : -1;
  } else {
    h -= 2 * fx + 2 * fy;
    int hi = h >= fz, e = h - hi * fz;
    li = e % bx;
    lj = e / bx;
    lk = hi ? bz : -1;
  }
  pidx = ((lk + 1) * (by + 2) + (lj + 1)) * (bx + 2) + (li + 1);
  gidx = lin(K, ox + li, oy + lj, oz + lk);
}

// Start of each face's slots in a published face buffer (faces -x, +x, -y,
// +y, -z, +z) and the total nh.
__device__ inline void brick_face_offsets(const int bd[3], int foff[7]) {
  const int fx = bd[1] * bd[2], fy = bd[0] * bd[2], fz = bd[0] * bd[1];
  foff[0] = 0;
  foff[1] = fx;
  foff[2] = 2 * fx;
  foff[3] = 2 * fx + fy;
  foff[4] = 2 * fx + 2 * fy;
  foff[5] = 2 * fx + 2 * fy + fz;
  foff[6] = 2 * (fx + fy + fz);
}

// Halo slot h of brick (bi, bj, bk): where it goes in the padded brick and
// where its published value sits (brick-relative offset, without the
// parity/array term) in the neighbour's face buffer.
__device__ inline void brick_halo_src(const int bd[3], const int nbr[3], const int foff[7], int bi,
                                      int bj, int bk, int h, int& pidx, int& src) {
  const int bx = bd[0], by = bd[1], bz = bd[2];
  int part = 0;
  while (part < 5 && h >= foff[part + 1]) ++part;
  const int e = h - foff[part], up = part & 1;
  int li, lj, lk, ni = bi, nj = bj, nk = bk;
  if (part < 2) {
    lj = e % by;
    lk = e / by;
    li = up ? bx : -1;
    ni = wrapi(bi + (up ? 1 : -1), nbr[0]);
  } else if (part < 4) {
    li = e % bx;
    lk = e / bx;
    lj = up ? by : -1;
    nj = wrapi(bj + (up ? 1 : -1), nbr[1]);
  } else {
    li = e % bx;
    lj = e / bx;
    lk = up ? bz : -1;
    nk = wrapi(bk + (up ? 1 : -1), nbr[2]);
  }
  pidx = ((lk + 1) * (by + 2) + (lj + 1)) * (bx + 2) + (li + 1);
  const int nb = (nk * nbr[1] + nj) * nbr[0] + ni;
  src = nb * 6 * foff[6] + foff[part ^ 1] + e;
}

// Face values are exchanged between workgroups on different XCDs with
// device-scope relaxed atomic stores and loads, which the grid reduction's
// release/acquire pair orders; they travel to the device coherence point
// directly instead of being written back from and invalidated in each L2.
__device__ inline void face_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double face_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Writes v to every face slot of own node (li, lj, lk) in face buffer `fb`.
__device__ inline void brick_publish(double* fb, const int bd[3], const int foff[7], int li, int lj,
                                     int lk, double v) {
  const int bx = bd[0], by = bd[1], bz = bd[2];
  if (li == 0) face_store(&fb[foff[0] + lj + by * lk], v);
  if (li == bx - 1) face_store(&fb[foff[1] + lj + by * lk], v);
  if (lj == 0) face_store(&fb[foff[2] + li + bx * lk], v);
  if (lj == by - 1) face_store(&fb[foff[3] + li + bx * lk], v);
  if (lk == 0) face_store(&fb[foff[4] + li + bx * lj], v);
  if (lk == bz - 1) face_store(&fb[foff[5] + li + bx * lj], v);
}

// Bytes of dynamic LDS for a brick: the padded brick in doubles, then the
// halo table (padded index and global node of every halo node).
inline size_t brick_lds_bytes(const int bd[3]) {
  size_t pad = (size_t)(bd[0] + 2) * (bd[1] + 2) * (bd[2] + 2);
  size_t nh = 2 * ((size_t)bd[1] * bd[2] + (size_t)bd[0] * bd[2] + (size_t)bd[0] * bd[1]);
  return pad * sizeof(double) + 2 * nh * sizeof(int) + 2 * nh * sizeof(double);
}

// Bricks are NT columns (bdim[0] x bdim[1] = NT) of Q nodes along z: thread t
// owns the column (li, lj) = (t mod bdim[0], t / bdim[0]) and its nodes
// lk = 0..Q-1, so its node q sits at padded index pl0 + q pxy and mesh node
// gn0 + q nx ny (a brick never wraps inside).
template <int Q, int NT>
__global__ void __launch_bounds__(NT) k_cg_brick(SimConst K, CgArgs a) {
  a = member_view(K, a);
  extern __shared__ double R[];
  __shared__ double sh[3 * (NT / 64)];
  const int bd[3] = {a.bdim[0], a.bdim[1], Q};
  int foff[7];
  brick_face_offsets(bd, foff);
  const int px = bd[0] + 2, pxy = (bd[0] + 2) * (bd[1] + 2);
  const int nh = foff[6];
  const int bi = blockIdx.x % a.nbr[0], bj = (blockIdx.x / a.nbr[0]) % a.nbr[1],
            bk = blockIdx.x / (a.nbr[0] * a.nbr[1]);
  const int ox = bi * bd[0], oy = bj * bd[1], oz = bk * Q;
  const int tid = threadIdx.x;
  double* pub = a.pub;
  double* own = pub + (int64_t)blockIdx.x * 6 * nh;  // this brick's face buffers
  // halo table, built once per solve: padded index and published source
  int* hp = (int*)(R + pxy * (Q + 2));
  int* hs = hp + nh;
  // the halo's own r and s, carried by the owners' recurrence
  double* hrv = (double*)(hs + nh);
  double* hsv = hrv + nh;
  for (int h = tid; h < nh; h += NT) brick_halo_src(bd, a.nbr, foff, bi, bj, bk, h, hp[h], hs[h]);

  const int li = tid % bd[0], lj = tid / bd[0];
  const int pl0 = (bd[1] + 2 + lj + 1) * px + (li + 1);  // padded index of lk = 0
  const int plane = K.nc[0] * K.nc[1];
  const int gn0 = ((oz * K.nc[1]) + oy + lj) * K.nc[0] + ox + li;
  const bool side = li == 0 || li == bd[0] - 1 || lj == 0 || lj == bd[1] - 1;
  auto pl = [&](int q) { return pl0 + q * pxy; };
  auto gn = [&](int q) { return gn0 + q * plane; };
  auto face = [&](int q) { return side || q == 0 || q == Q - 1; };
  auto publish = [&](double* fb, int q, double v) { brick_publish(fb, bd, foff, li, lj, q, v); };
  // -L at own node q from its value v and its z neighbours zm, zp (own
  // registers inside the column, the LDS halo at its ends); the x and y
  // neighbours come from LDS.  Same association as neg_lap_pad.
  auto col_lap = [&](int q, double v, double zm, double zp) {
    const int c = pl(q);
    double lx = R[c + 1] - 2.0 * v + R[c - 1];
    double ly = R[c + px] - 2.0 * v + R[c - px];
    double lz = zp - 2.0 * v + zm;
    return -(lx * K.ih2[0] + ly * K.ih2[1] + lz * K.ih2[2]);
  };
  double xr[Q], rr[Q], wr[Q], sr[Q], pr[Q];
  unsigned gen = 0;
  // sum of the iterate, carried by each iteration's reduction (for the
  // zero-mean projection; summed in the same order as a reduction of its own)
  double xsum = 0.0;
  bool xsum_ok = false;

  // r_0 = -b - A x_0 from the stored iterate (own nodes and halo straight from x)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    xr[q] = a.x[gn(q)];
    R[pl(q)] = xr[q];
  }
  for (int h = tid; h < nh; h += NT) {
    int pi, gi;
    brick_halo(K, bd, ox, oy, oz, h, pi, gi);
    R[pi] = a.x[gi];
  }
  __syncthreads();
  double v2[kMaxRed] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double bv = a.b[gn(q)];
    double rv = -bv - neg_lap_pad(K, R, pl(q), px, pxy);
    rr[q] = rv;
    v2[0] += rv * rv;
    v2[1] += bv * bv;
    if (face(q)) publish(own, q, rv);  // parity 0, r
  }
  if (!grid_sum_t<NT>(a, v2, 2, ++gen, sh)) return;
  double gamma = v2[0];
  const double bnorm = sqrt(v2[1]);
  int it = 0;
  if (bnorm == 0.0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) xr[q] = 0.0;
    gamma = 0.0;
  } else if (sqrt(gamma) > a.tol * bnorm) {
    // w_0 = A r_0
#pragma unroll
    for (int q = 0; q < Q; ++q) R[pl(q)] = rr[q];
    for (int h = tid; h < nh; h += NT) {
      const double rv = face_load(pub + hs[h]);
      R[hp[h]] = rv;
      hrv[h] = rv;
      hsv[h] = 0.0;
    }
    __syncthreads();
    double v1[kMaxRed] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double wv = neg_lap_pad(K, R, pl(q), px, pxy);
      wr[q] = wv;
      v1[0] += wv * rr[q];
      if (face(q)) publish(own + nh, q, wv);  // parity 0, w
    }
    if (!grid_sum_t<NT>(a, v1, 1, ++gen, sh)) return;
    double alpha = gamma / v1[0], beta = 0.0;
    int cur = 0;
    while (true) {
      if (it >= a.max_iter) {
        if (blockIdx.x == 0 && tid == 0) atomicOr(&a.flags[kFlagCgNoConv], 1);
        break;
      }
      const bool first = it == 0;  // p_{-1} = s_{-1} = 0: never read
      // own nodes: p_i, s_i, x_{i+1}, r_{i+1}
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        double pv = first ? rr[q] : rr[q] + beta * pr[q];
        double sv = first ? wr[q] : wr[q] + beta * sr[q];
        pr[q] = pv;
        sr[q] = sv;
        xr[q] += alpha * pv;
        rr[q] = rr[q] - alpha * sv;
        R[pl(q)] = rr[q];
      }
      // halo: the neighbours' r_{i+1} by their own recurrence, from their
      // published w_i and the halo's r_i, s_{i-1} kept here (the same
      // operations on the same values as the owners', so the same bits)
      {
        const double* src = pub + (int64_t)cur * 3 * nh + nh;
#pragma unroll 4
        for (int h = tid; h < nh; h += NT) {
          const double wv = face_load(src + hs[h]);
          const double sv = first ? wv : wv + beta * hsv[h];
          const double rv = hrv[h] - alpha * sv;
          hsv[h] = sv;
          hrv[h] = rv;
          R[hp[h]] = rv;
        }
      }
      __syncthreads();
      double* dst = own + (int64_t)(cur ^ 1) * 3 * nh;
      double gd[kMaxRed] = {0.0, 0.0, 0.0};
      const double zlo = R[pl(0) - pxy], zhi = R[pl(Q - 1) + pxy];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        double wv = col_lap(q, rr[q], q > 0 ? rr[q > 0 ? q - 1 : 0] : zlo,
                            q < Q - 1 ? rr[q < Q - 1 ? q + 1 : 0] : zhi);
        wr[q] = wv;
        gd[0] += rr[q] * rr[q];
        gd[1] += wv * rr[q];
        gd[2] += xr[q];
        if (face(q)) publish(dst + nh, q, wv);
      }
      // (grid_sum's block barrier also orders these stencil reads of R before
      // the next sweep overwrites it)
      if (!grid_sum_t<NT>(a, gd, 3, ++gen, sh)) return;
      xsum = gd[2];
      xsum_ok = true;
      cur ^= 1;
      ++it;
      beta = gd[0] / gamma;
      alpha = gd[0] / (gd[1] - beta * gd[0] / alpha);
      gamma = gd[0];
      if (sqrt(gamma) <= a.tol * bnorm) break;
    }
  }
  // zero-mean projection (Sec. 2); the last iteration's reduction carried
  // the sum of the final iterate, else one more reduction
  if (!xsum_ok) {
    double s_x[kMaxRed] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) s_x[0] += xr[q];
    if (!grid_sum_t<NT>(a, s_x, 1, ++gen, sh)) return;
    xsum = s_x[0];
  }
  const double mean = xsum / (double)K.nn;
#pragma unroll
  for (int q = 0; q < Q; ++q) a.x[gn(q)] = xr[q] - mean;
  if (blockIdx.x == 0 && tid == 0) {
    *a.iters_out = it;
    *a.relres_out = bnorm == 0.0 ? 0.0 : sqrt(gamma) / bnorm;
  }
}

}  // namespace pic
