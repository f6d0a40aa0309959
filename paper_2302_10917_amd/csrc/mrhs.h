// Forward and backward substitution on the stored FP64 LU factors of one
// macro with 16 NH right-hand sides, by one workgroup of NW wavefronts.
//
// The right-hand sides form an N x 16 NH block Y, cut into 16-row tiles;
// wavefront w holds tiles w, w + NW, w + 2 NW, ... (TPW of them) in the FP64
// MFMA accumulator layout (x[i][h]: tile w + NW i, right-hand sides
// 16 h .. 16 h + 15; element v of lane (li, lk) is row lk + 4 v, column li).
// Block step b of the forward sweep (L unit lower, column-major in place):
//   * the wavefront that owns tile b has already solved it with the 16 x 16
//     diagonal block of L and published it in LDS;
//   * every wavefront subtracts L[tile t, block b] Y_b from each of its tiles
//     t > b: one 16 x 16 x 16 product = four 16x16x4 FP64 MFMAs per tile and
//     16 right-hand sides, with the L tile read once from HBM for all of them;
//   * the owner of tile b + 1 updates that tile first and solves it at once,
//     so the next block is published while the other wavefronts still update.
// The solved block goes to one of two LDS buffers, one workgroup barrier per
// block.  The backward sweep (U upper, non-unit diagonal) runs the same steps
// from the last block up.  Rows past N read as the identity.  The factor is
// read once per call for all 16 NH right-hand sides.
#pragma once
#include "macro_solve.h"
#include "mfma.h"

namespace mhdg {

// LDS of the sweeps: the double buffer of the published block (2 x 16 NH x 16)
// and the staged 16 x 16 diagonal block (rows padded to 17)
template <int NH> struct MrhsLds { static constexpr int doubles = 2 * NH * 256 + 16 * 17; };

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

// Stage a diagonal tile (loaded with load_tile) in LDS: sd[r][q] = F(16c + r, 16c + q).
__device__ __forceinline__ void stage_diag(const double (&dg)[4], double (*sd)[17], int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) sd[li][4 * s + lk] = dg[s];
  wave_lds_sync();
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

// Y_c <- L_cc^-1 Y_c (unit lower), one wavefront, L_cc staged in sd.
template <int NH>
__device__ __forceinline__ void solve_unit_lower16(d4 (&y)[NH], double (*sd)[17], int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 15; ++i) {
    double yi[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) yi[h] = __shfl(y[h][i >> 2], li + 16 * (i & 3), 64);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = lk + 4 * v;
      if (r > i) {
        const double l = sd[r][i];
#pragma unroll
        for (int h = 0; h < NH; ++h) y[h][v] -= l * yi[h];
      }
    }
    __builtin_amdgcn_sched_barrier(0);   // one row per step: nothing hoisted
  }
}

// Y_c <- U_cc^-1 Y_c (upper, non-unit), one wavefront, U_cc staged in sd.
template <int NH>
__device__ __forceinline__ void solve_upper16(d4 (&y)[NH], double (*sd)[17], int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 15; i >= 0; --i) {
    const double d = sd[i][i];
    if (lk == (i & 3)) {
#pragma unroll
      for (int h = 0; h < NH; ++h) y[h][i >> 2] = y[h][i >> 2] / d;
    }
    if (i == 0) break;
    double yi[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) yi[h] = __shfl(y[h][i >> 2], li + 16 * (i & 3), 64);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = lk + 4 * v;
      if (r < i) {
        const double u = sd[r][i];
#pragma unroll
        for (int h = 0; h < NH; ++h) y[h][v] -= u * yi[h];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// tiles whose factor loads may be in flight together in the update loop
#ifndef MHDG_MRHS_GROUP
#define MHDG_MRHS_GROUP 4
#endif
constexpr int kTileGroup = MHDG_MRHS_GROUP;

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
// block (ld), s: MrhsLds<NH>::doubles of LDS.  The wavefront that will own
// block b + 2 loads, during step b, the two factor tiles its own step b + 1
// needs first (the tile that couples its block to block b + 1, and its
// diagonal tile), so the critical path of a step carries no factor load.
// Ends with a workgroup barrier.
template <int NW, int TPW, int NH>
__device__ __forceinline__ void mrhs_sweeps(d4 (&x)[TPW][NH], const double* __restrict__ A, int N,
                                            int ld, double* s, int wid_in, int lane) {
  // the wavefront index as a uniform value: every branch below is taken by
  // whole wavefronts, which the MFMA updates need
  const int wid = __builtin_amdgcn_readfirstlane(wid_in);
  double* bufs = s;
  double(*sd)[17] = reinterpret_cast<double(*)[17]>(s + 2 * NH * 256);
  const int T = (N + 15) >> 4;
  double pa[4], pd[4];   // prefetched coupling and diagonal tiles of this wavefront's next block
  // ---- forward: L unit lower
  if (wid == 0) {
    load_tile(pd, A, ld, N, 0, 0, lane);
    stage_diag(pd, sd, lane);
    solve_unit_lower16<NH>(x[0], sd, lane);
    publish<NH>(x[0], bufs, lane);
  }
  if (1 < T && wid == 1 % NW) {
    load_tile(pa, A, ld, N, 1, 0, lane);
    load_tile(pd, A, ld, N, 1, 1, lane);
  }
  for (int b = 0; b < T; ++b) {
    __syncthreads();
    double bs[NH][4];
    read_block<NH>(bs, bufs + (b & 1) * NH * 256, lane);
    const int nb = b + 1;
    if (nb < T && wid == nb % NW) {   // the next block's owner: update, solve, publish
      d4 cur[NH];
      take_tile<TPW, NH>(cur, x, nb / NW);
      tile_mma<NH>(cur, pa, bs);
      stage_diag(pd, sd, lane);
      solve_unit_lower16<NH>(cur, sd, lane);
      publish<NH>(cur, bufs + (nb & 1) * NH * 256, lane);
      put_tile<TPW, NH>(x, cur, nb / NW);
    }
    if (nb + 1 < T && wid == (nb + 1) % NW) {
      load_tile(pa, A, ld, N, nb + 1, nb, lane);
      load_tile(pd, A, ld, N, nb + 1, nb + 1, lane);
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wid + NW * i;
      if (t > nb && t < T) {
        double a[4];
        load_tile(a, A, ld, N, t, b, lane);
        tile_mma<NH>(x[i], a, bs);
      }
      if (i % kTileGroup == kTileGroup - 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();   // the last block's buffer is read before the backward sweep reuses it
  // ---- backward: U upper
  if (wid == (T - 1) % NW) {
    d4 cur[NH];
    take_tile<TPW, NH>(cur, x, (T - 1) / NW);
    load_tile(pd, A, ld, N, T - 1, T - 1, lane);
    stage_diag(pd, sd, lane);
    solve_upper16<NH>(cur, sd, lane);
    publish<NH>(cur, bufs + ((T - 1) & 1) * NH * 256, lane);
    put_tile<TPW, NH>(x, cur, (T - 1) / NW);
  }
  if (T >= 2 && wid == (T - 2) % NW) {
    load_tile(pa, A, ld, N, T - 2, T - 1, lane);
    load_tile(pd, A, ld, N, T - 2, T - 2, lane);
  }
  for (int b = T - 1; b > 0; --b) {
    __syncthreads();
    double bs[NH][4];
    read_block<NH>(bs, bufs + (b & 1) * NH * 256, lane);
    const int nb = b - 1;
    if (wid == nb % NW) {
      d4 cur[NH];
      take_tile<TPW, NH>(cur, x, nb / NW);
      tile_mma<NH>(cur, pa, bs);
      stage_diag(pd, sd, lane);
      solve_upper16<NH>(cur, sd, lane);
      publish<NH>(cur, bufs + (nb & 1) * NH * 256, lane);
      put_tile<TPW, NH>(x, cur, nb / NW);
    }
    if (nb >= 1 && wid == (nb - 1) % NW) {
      load_tile(pa, A, ld, N, nb - 1, nb, lane);
      load_tile(pd, A, ld, N, nb - 1, nb - 1, lane);
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wid + NW * i;
      if (t < nb) {
        double a[4];
        load_tile(a, A, ld, N, t, b, lane);
        tile_mma<NH>(x[i], a, bs);
      }
      if (i % kTileGroup == kTileGroup - 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();
}

}  // namespace mhdg
