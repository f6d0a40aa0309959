// Forward and backward substitution on the stored FP64 LU factors of one
// macro with 16 NH right-hand sides, by one workgroup of NW wavefronts.
//
// The right-hand sides form an N x 16 NH block Y, cut into 16-row tiles;
// wavefront w holds tiles w, w + NW, w + 2 NW, ... (TPW of them) in the FP64
// MFMA accumulator layout (x[i][h]: tile w + NW i, right-hand sides
// 16 h .. 16 h + 15; element v of lane (li, lk) is row lk + 4 v, column li).
// Block step b of the forward sweep (L unit lower, column-major in place):
//   * the wavefront that owns tile b + 1 subtracts L[tile b + 1, block b] Y_b
//     from it, multiplies it by the inverse of the diagonal 16 x 16 block of
//     L (both on MFMA) and publishes it in LDS for the next step;
//   * every wavefront subtracts L[tile t, block b] Y_b from each of its other
//     tiles t > b + 1: four 16x16x4 FP64 MFMAs per tile and 16 right-hand
//     sides, with the L tile read once from HBM for all of them.
// A wavefront forms the inverse of the diagonal block of its next block (and
// loads that block's coupling tile) as soon as it has published its current
// one, NW steps before it is needed, so a step's critical path holds two
// chains of four MFMAs and no factor load.  The factor tiles of the last
// tiles of every wavefront are loaded one step ahead, before the barrier.
// The solved block goes to one of two LDS buffers, one workgroup barrier per
// block.  The backward sweep (U upper, non-unit diagonal) runs the same steps
// from the last block up.  Rows past N read as the identity.  The factor is
// read once per call for all 16 NH right-hand sides.
#pragma once
#include "macro_solve.h"
#include "mfma.h"

namespace mhdg {

// LDS of the sweeps: the double buffer of the published block (2 x 16 NH x 16)
// and one 16 x 16 work tile per wavefront (rows padded to 17)
__host__ __device__ constexpr int mrhs_lds_doubles(int nw, int nh) { return 2 * nh * 256 + nw * 16 * 17; }

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The factor tile at rows 16 t, columns 16 c in the MFMA A-operand layout:
// a[s] = F(16 t + li, 16 c + 4 s + lk).  Indices are clamped into the block
// and the value masked (identity past N), so every load is issued.
__device__ __forceinline__ void load_tile(double (&a)[4], const double* __restrict__ A, int ld,
                                          int N, int t, int c, int lane) {
  const int li = lane & 15, lk = lane >> 4;
  const int r = 16 * t + li;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int q = 16 * c + 4 * s + lk;
    const double v = A[size_t(min(q, N - 1)) * ld + min(r, N - 1)];
    a[s] = (r < N && q < N) ? v : (r == q ? 1.0 : 0.0);
  }
}

// Inverse of a diagonal factor tile dg (load_tile layout) in the A-operand
// layout: inv[s] = (F_cc^-1)[li][4 s + lk], F_cc unit lower (UPPER = false:
// its strict lower part) or upper with its diagonal.  One wavefront solves
// F_cc X = I column-parallel (16 sequential rows) in its LDS work tile sd.
template <bool UPPER>
__device__ __forceinline__ void inv_tile(const double (&dg)[4], double (*sd)[17], double (&inv)[4],
                                         int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) sd[li][4 * s + lk] = dg[s];
  wave_lds_sync();
  d4 y;
#pragma unroll
  for (int v = 0; v < 4; ++v) y[v] = lk + 4 * v == li ? 1.0 : 0.0;
  if (!UPPER) {
#pragma unroll
    for (int i = 0; i < 15; ++i) {
      double l[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) l[v] = lk + 4 * v > i ? sd[lk + 4 * v][i] : 0.0;
      const double yi = __shfl(y[i >> 2], li + 16 * (i & 3), 64);
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] -= l[v] * yi;
    }
  } else {
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      const double d = sd[i][i];
      if (lk == (i & 3)) y[i >> 2] = y[i >> 2] / d;
      if (i == 0) break;
      double u[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) u[v] = lk + 4 * v < i ? sd[lk + 4 * v][i] : 0.0;
      const double yi = __shfl(y[i >> 2], li + 16 * (i & 3), 64);
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] -= u[v] * yi;
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int v = 0; v < 4; ++v) sd[lk + 4 * v][li] = y[v];
  wave_lds_sync();
#pragma unroll
  for (int s = 0; s < 4; ++s) inv[s] = sd[li][4 * s + lk];
  wave_lds_sync();
}

// y <- F_cc^-1 y on MFMA (inv from inv_tile; the FP64 accumulator element s
// of a lane is the B operand of k-step s).
template <int NH>
__device__ __forceinline__ void apply_inv(d4 (&y)[NH], const double (&inv)[4]) {
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    d4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) z = Mfma<double>::run(inv[s], y[h][s], z);
    y[h] = z;
  }
}

// Publish tile y (16 x 16 NH) to buffer buf: buf[h][row][col].
template <int NH>
__device__ __forceinline__ void publish(const d4 (&y)[NH], double* buf, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int v = 0; v < 4; ++v) buf[h * 256 + (lk + 4 * v) * 16 + li] = y[h][v];
}

// tiles whose factor loads may be in flight together in the update loop
#ifndef MHDG_MRHS_GROUP
#define MHDG_MRHS_GROUP 4
#endif
constexpr int kTileGroup = MHDG_MRHS_GROUP;
// tiles of each wavefront whose next-step factor tiles are loaded before the
// step's barrier (the last ones in the forward sweep, the first ones in the
// backward sweep: those stay active longest)
#ifndef MHDG_MRHS_PREFETCH
#define MHDG_MRHS_PREFETCH 4
#endif

// The B operands of a published block: bs[h][s] = Y_b[4 s + lk][16 h + li].
template <int NH>
__device__ __forceinline__ void read_block(double (&bs)[NH][4], const double* buf, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int s = 0; s < 4; ++s) bs[h][s] = buf[h * 256 + (4 * s + lk) * 16 + li];
}

// x -= F[tile t, block b] Y_b with the factor tile a (load_tile) and the
// block's B operands bs.
template <int NH>
__device__ __forceinline__ void tile_mma(d4 (&x)[NH], const double (&a)[4],
                                         const double (&bs)[NH][4]) {
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int s = 0; s < 4; ++s) x[h] = Mfma<double>::run(-a[s], bs[h][s], x[h]);
}

// cur = x[i1] and back, with i1 a runtime index into the unrolled tile array
template <int TPW, int NH>
__device__ __forceinline__ void take_tile(d4 (&cur)[NH], const d4 (&x)[TPW][NH], int i1) {
#pragma unroll
  for (int i = 0; i < TPW; ++i)
    if (i == i1) {
#pragma unroll
      for (int h = 0; h < NH; ++h) cur[h] = x[i][h];
    }
}
template <int TPW, int NH>
__device__ __forceinline__ void put_tile(d4 (&x)[TPW][NH], const d4 (&cur)[NH], int i1) {
#pragma unroll
  for (int i = 0; i < TPW; ++i)
    if (i == i1) {
#pragma unroll
      for (int h = 0; h < NH; ++h) x[i][h] = cur[h];
    }
}

// Both sweeps.  x: this wavefront's tiles (zero rows past N), A: the factor
// block (ld), s: mrhs_lds_doubles(NW, NH) doubles of LDS.  Ends with a
// workgroup barrier.  (Loading the next block's tiles in the owner's step and
// inverting them one step later, off the owner's path, was slower: 611
// against 671 vector-applies/s at 16 vectors per call.)
template <int NW, int TPW, int NH, int PF = (MHDG_MRHS_PREFETCH < TPW ? MHDG_MRHS_PREFETCH : TPW)>
__device__ __forceinline__ void mrhs_sweeps(d4 (&x)[TPW][NH], const double* __restrict__ A, int N,
                                            int ld, double* s, int wid_in, int lane) {
  // the wavefront index as a uniform value: every branch below is taken by
  // whole wavefronts, which the MFMA updates need
  const int wid = __builtin_amdgcn_readfirstlane(wid_in);
  double* bufs = s;
  double(*sd)[17] = reinterpret_cast<double(*)[17]>(s + 2 * NH * 256 + wid * 16 * 17);
  const int T = (N + 15) >> 4;
  // this wavefront's next block c: its coupling tile F[c, c -/+ 1] and the
  // inverse of its diagonal tile
  double pa[4], pinv[4];
  auto prepare = [&](int c, int cprev, bool upper) {
    double dg[4];
    load_tile(pa, A, ld, N, c, cprev, lane);
    load_tile(dg, A, ld, N, c, c, lane);
    if (upper) inv_tile<true>(dg, sd, pinv, lane);
    else inv_tile<false>(dg, sd, pinv, lane);
  };
  // ---- forward: L unit lower
  if (wid == 0) {
    double dg[4];
    load_tile(dg, A, ld, N, 0, 0, lane);
    inv_tile<false>(dg, sd, pinv, lane);
    apply_inv<NH>(x[0], pinv);
    publish<NH>(x[0], bufs, lane);
    if (NW < T) prepare(NW, NW - 1, false);
  } else if (wid < T) {
    prepare(wid, wid - 1, false);
  }
  double ap[PF][4];   // factor tiles of the last PF tiles for the coming step
#pragma unroll
  for (int j = 0; j < PF; ++j) load_tile(ap[j], A, ld, N, wid + NW * (TPW - PF + j), 0, lane);
  for (int b = 0; b < T; ++b) {
    __syncthreads();
    double bs[NH][4];
    read_block<NH>(bs, bufs + (b & 1) * NH * 256, lane);
    const int nb = b + 1;
    if (nb < T && wid == nb % NW) {   // the next block's owner: update, solve, publish
      d4 cur[NH];
      take_tile<TPW, NH>(cur, x, nb / NW);
      tile_mma<NH>(cur, pa, bs);
      apply_inv<NH>(cur, pinv);
      publish<NH>(cur, bufs + (nb & 1) * NH * 256, lane);
      put_tile<TPW, NH>(x, cur, nb / NW);
      if (nb + NW < T) prepare(nb + NW, nb + NW - 1, false);
    }
#pragma unroll
    for (int i = 0; i < TPW - PF; ++i) {
      const int t = wid + NW * i;
      if (t > nb && t < T) {
        double a[4];
        load_tile(a, A, ld, N, t, b, lane);
        tile_mma<NH>(x[i], a, bs);
      }
      if (i % kTileGroup == kTileGroup - 1) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int t = wid + NW * (TPW - PF + j);
      if (t > nb && t < T) tile_mma<NH>(x[TPW - PF + j], ap[j], bs);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (b + 1 < T) {
#pragma unroll
      for (int j = 0; j < PF; ++j) load_tile(ap[j], A, ld, N, wid + NW * (TPW - PF + j), b + 1, lane);
    }
  }
  __syncthreads();   // the last block's buffer is read before the backward sweep reuses it
  // ---- backward: U upper; the first PF tiles are the ones loaded ahead
  {
    // this wavefront's first block below T - 1
    const int c0 = T - 2 - ((T - 2 - wid) % NW + NW) % NW;
    if (wid == (T - 1) % NW) {
      d4 cur[NH];
      double dg[4];
      take_tile<TPW, NH>(cur, x, (T - 1) / NW);
      load_tile(dg, A, ld, N, T - 1, T - 1, lane);
      inv_tile<true>(dg, sd, pinv, lane);
      apply_inv<NH>(cur, pinv);
      publish<NH>(cur, bufs + ((T - 1) & 1) * NH * 256, lane);
      put_tile<TPW, NH>(x, cur, (T - 1) / NW);
    }
    if (T >= 2 && c0 >= 0) prepare(c0, c0 + 1, true);
  }
#pragma unroll
  for (int j = 0; j < PF; ++j) load_tile(ap[j], A, ld, N, wid + NW * j, T - 1, lane);
  for (int b = T - 1; b > 0; --b) {
    __syncthreads();
    double bs[NH][4];
    read_block<NH>(bs, bufs + (b & 1) * NH * 256, lane);
    const int nb = b - 1;
    if (wid == nb % NW) {
      d4 cur[NH];
      take_tile<TPW, NH>(cur, x, nb / NW);
      tile_mma<NH>(cur, pa, bs);
      apply_inv<NH>(cur, pinv);
      publish<NH>(cur, bufs + (nb & 1) * NH * 256, lane);
      put_tile<TPW, NH>(x, cur, nb / NW);
      if (nb - NW >= 0) prepare(nb - NW, nb - NW + 1, true);
    }
#pragma unroll
    for (int i = PF; i < TPW; ++i) {
      const int t = wid + NW * i;
      if (t < nb) {
        double a[4];
        load_tile(a, A, ld, N, t, b, lane);
        tile_mma<NH>(x[i], a, bs);
      }
      if ((i - PF) % kTileGroup == kTileGroup - 1) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int t = wid + NW * j;
      if (t < nb) tile_mma<NH>(x[j], ap[j], bs);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (b > 1) {
#pragma unroll
      for (int j = 0; j < PF; ++j) load_tile(ap[j], A, ld, N, wid + NW * j, b - 1, lane);
    }
  }
  __syncthreads();
}

}  // namespace mhdg
