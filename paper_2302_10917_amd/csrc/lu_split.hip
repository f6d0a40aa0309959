// LU with partial pivoting, one launch per step of each 128-column panel, so
// that the trailing update runs as a batched GEMM over the whole chip instead
// of inside one workgroup per macro.
//
// The same factorisation as lu_kernel and lu_blocked_kernel (PA = LU, largest
// |a| pivots with ties to the smallest row, factors column-major on exit): the
// local matrices of section 3.3.2 are factored once and the factors serve every
// later local solve.  Per panel of W = 128 columns starting at column k0:
//   1. lu_panel_kernel (one workgroup per macro) factors the window
//      A[k0:N, k0:k0+W] with its row interchanges applied inside the window
//      only: two 64-column halves of 16-column sub-panels held in registers.
//      Each sub-panel's 16 x 16 unit lower diagonal block is inverted (15
//      parallel steps), so that every triangular solve of the panel and of
//      the next launch is a chain of MFMA products.  The kernel writes the
//      window's row moves (the composition of its interchanges as
//      (destination row, source row) pairs) and the eight inverse blocks to a
//      per-macro scratch;
//   2. lu_swap_u12_kernel (one workgroup per 64 columns outside the window)
//      applies those moves to the columns left and right of the window and,
//      on the right, solves U12 = L11^-1 A12: each wavefront holds 16 columns
//      of the window rows in registers and runs the block solve on MFMA;
//   3. lu_update_kernel (one workgroup per 64 x 64 tile of the trailing
//      matrix) computes A22 -= L21 U12 on MFMA through 16-deep slices of L21
//      and U12 staged in LDS.  All tiles of one macro run on one XCD, so its
//      L21 and U12 are read from that XCD's L2.
// A last launch stores the factors column-major, one 32 x 32 tile pair per
// workgroup.  The matrix is row-major (element (i, j) at i * ld + j) until then.
#include "internal.h"
#include "mfma.h"

namespace mhdg {

constexpr int kSplitW = 128;              // panel width: the rank of the trailing updates
constexpr int kSplitH = 64;               // a panel is factored as two halves
constexpr int kMoveInts = 1 + 4 * kSplitW;  // count, then up to 2W (destination, source) pairs
// per-macro scratch: the row moves, then the inverses of the window's eight
// 16 x 16 diagonal blocks of L11 (row-major, sized for FP64)
constexpr size_t kMoveBytes = 2304;
constexpr size_t kSplitScratch = kMoveBytes + size_t(kSplitW / 16) * 256 * sizeof(double);
static_assert(kMoveBytes >= kMoveInts * sizeof(int32_t), "row moves fit");

// The B operand of k-step s (rows 4 s .. 4 s + 3 of a 16 x 16 tile) from the
// tile held in the MFMA accumulator layout.  FP64: accumulator element v of
// lane (li, lk) is row lk + 4 v, so it is element s of the lane itself; FP32:
// row 4 lk + v, so it comes from lane (li, s), element lk.
__device__ __forceinline__ double b_from_acc(const d4& x, int s, int lane) { return x[s]; }
__device__ __forceinline__ float b_from_acc(const f4& x, int s, int lane) {
  const int src = (lane & 15) + 16 * s, lk = lane >> 4;
  const float t0 = __shfl(x[0], src, 64), t1 = __shfl(x[1], src, 64);
  const float t2 = __shfl(x[2], src, 64), t3 = __shfl(x[3], src, 64);
  return lk == 0 ? t0 : (lk == 1 ? t1 : (lk == 2 ? t2 : t3));
}

// X <- L^-1 X for one wavefront's 16 columns of a 16 nb x 16 block held in
// registers in the accumulator layout (x[t]: rows 16 t ..), L unit lower
// triangular: the diagonal blocks through their inverses, Li(b, i, p) =
// (L_bb^-1)[i][p], the rows below through L's off-diagonal entries L(i, p)
// (both relative to the block's first row).  No other wavefront is involved.
template <typename T, int NB, typename FLi, typename FL>
__device__ __forceinline__ void wave_trsm(typename Mfma<T>::acc (&x)[NB], int nb, FLi Li, FL L,
                                          int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b >= nb) break;
    T bx[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) bx[s] = b_from_acc(x[b], s, lane);
    typename Mfma<T>::acc y = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s) y = Mfma<T>::run(Li(b, li, 4 * s + lk), bx[s], y);
    x[b] = y;
#pragma unroll
    for (int s = 0; s < 4; ++s) bx[s] = b_from_acc(y, s, lane);
#pragma unroll
    for (int t = b + 1; t < NB; ++t) {
      if (t >= nb) break;
#pragma unroll
      for (int s = 0; s < 4; ++s)
        x[t] = Mfma<T>::run(-L(16 * t + li, 16 * b + 4 * s + lk), bx[s], x[t]);
    }
  }
}

// Inverse of the unit lower 16 x 16 block Lb (strict lower part, sb rows
// used) into Li: Li = (I - l_14 e_14^T) ... (I - l_0 e_0^T), one step per
// column, thread (i, c) updating Li[i][c] (the first 256 threads).
template <typename T, int NT>
__device__ __forceinline__ void invert_unit_lower16(const T (*Lb)[17], T (*Li)[17], int sb) {
  const int tid = threadIdx.x, i = tid >> 4, c = tid & 15;
  if (tid < 256) Li[i][c] = i == c ? T(1) : T(0);
  __syncthreads();
#pragma unroll 1
  for (int p = 0; p + 1 < sb; ++p) {
    if (tid < 256 && i > p && i < sb) Li[i][c] -= Lb[i][p] * Li[p][c];
    __syncthreads();
  }
}

// A[r0:N, c0:c1] -= A[r0:N, kc:kc+kw] A[kc:kc+kw, c0:c1] for c1 - c0 <= 64 and
// kw <= KW inside the panel: the U block is staged in LDS (Us, KW x 64), and
// wavefront w takes the row tiles w, w + NW, ... with all (at most four)
// column tiles of a row tile at once.
template <typename T, int KW, int NT>
__device__ __forceinline__ void band_update(T* __restrict__ A, int N, int ld, int r0, int c0,
                                            int c1, int kc, int kw, T* __restrict__ Us) {
  constexpr int S = KW / 4, NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nrt = (N - r0 + 15) >> 4, ncols = c1 - c0;
  for (int x = tid; x < KW * 64; x += NT) {
    const int k = x >> 6, c = x & 63;
    Us[x] = (k < kw && c < ncols) ? A[size_t(kc + k) * ld + c0 + c] : T(0);
  }
  __syncthreads();
  T an[S];
  typename Mfma<T>::acc cn[4];
  auto load = [&](int rt) {
    const int rr = r0 + 16 * rt;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = 4 * s + lk, row = rr + li;
      an[s] = (row < N && k < kw) ? -A[size_t(row) * ld + kc + k] : T(0);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rr + Mfma<T>::drow(lk, v), c = 16 * ct + li;
        cn[ct][v] = (row < N && c < ncols) ? A[size_t(row) * ld + c0 + c] : T(0);
      }
  };
#pragma unroll 1
  for (int rt = wid; rt < nrt; rt += NW) {
    load(rt);
    T a[S];
    typename Mfma<T>::acc acc[4];
#pragma unroll
    for (int s = 0; s < S; ++s) a[s] = an[s];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = cn[ct];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      if (16 * ct < ncols)
#pragma unroll
        for (int s = 0; s < S; ++s)
          acc[ct] = Mfma<T>::run(a[s], Us[(4 * s + lk) * 64 + 16 * ct + li], acc[ct]);
    const int rr = r0 + 16 * rt;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rr + Mfma<T>::drow(lk, v), c = 16 * ct + li;
        if (row < N && c < ncols) A[size_t(row) * ld + c0 + c] = acc[ct][v];
      }
  }
  __syncthreads();
}

// One workgroup of NT threads per macro factors the window of columns
// [k0, k0 + w).  Thread t holds the sub-panel rows c0 + t + q NT (q < RPT), so
// RPT * NT >= N - k0 is required.
template <typename T, int NT, int RPT, int SB>
__global__ __launch_bounds__(NT, 2) void lu_panel_kernel(T* fac, const MacroInfo* __restrict__ info,
                                                      const int32_t* __restrict__ order,
                                                      int64_t base, int k0, int32_t* perm_all,
                                                      int32_t* status, char* scratch) {
  static_assert(kSplitH % 16 == 0 && (SB == 8 || SB == 16), "sub-panels tile 16-row blocks");
  constexpr int NW = NT / 64, H = kSplitH;
  const int e = order[base + blockIdx.x];
  const MacroInfo& mi = info[e];
  const int N = mi.N, ld = mi.ld;
  T* A = fac + mi.fac_off;
  int32_t* perm = perm_all + mi.loc_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int w = min(kSplitW, N - k0), cw1 = k0 + w;

  __shared__ double s_red_v[NW];
  __shared__ int s_red_i[NW];
  __shared__ T s_row[2][SB];        // pivot rows (alternating slots per column)
  __shared__ T s_swap[2][SB];       // the rows they displace
  __shared__ T s_L[H * H];          // L11 of the first half; U blocks of the band updates
  __shared__ int s_piv[kSplitW];    // pivot row of each window column
  __shared__ int s_md[2 * SB], s_ms[2 * SB];   // a sub-panel's row moves (-1: none)
  // row k0 + r holds the content that row s_pos[r] had before the window
  // (s_sub: before the current sub-panel)
  __shared__ int s_pos[RPT * NT], s_sub[RPT * NT];
  __shared__ int s_cnt;
  __shared__ T s_Lb[16][17];        // a unit lower 16 x 16 block (strict lower part)
  __shared__ T s_Li[16][17];        // its inverse
  __shared__ T s_Lih[4][16][17];    // inverses of the first half's diagonal blocks
  __shared__ T s_Lh[SB == 8 ? 16 : 1][17];   // 8-column sub-panels: a whole block's inverse
  __shared__ int s_status;

  if (k0 == 0)
    for (int i = tid; i < N; i += NT) perm[i] = i;
  if (tid == 0) { s_status = k0 == 0 ? 0 : status[e]; s_cnt = 0; }
  for (int r = tid; r < N - k0; r += NT) s_pos[r] = k0 + r;
  __syncthreads();

  T pr[RPT][SB];
#pragma unroll 1
  for (int h0 = k0; h0 < cw1; h0 += H) {
    const int hw = min(H, cw1 - h0);
    if (h0 > k0) {
      // the first half's U rows in this half's columns, L11^-1 A12 on MFMA
      // (one wavefront per 16 columns, with the first half's inverse diagonal
      // blocks), then the rank-H update of the rows below
      if (wid < ((hw + 15) >> 4)) {
        const int li = lane & 15, lk = lane >> 4, col = h0 + 16 * wid + li;
        typename Mfma<T>::acc x[H / 16];
#pragma unroll
        for (int t = 0; t < H / 16; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = k0 + 16 * t + Mfma<T>::drow(lk, v);
            x[t][v] = col < h0 + hw ? A[size_t(row) * ld + col] : T(0);
          }
        wave_trsm<T, H / 16>(
            x, H / 16, [&](int b, int i, int q) { return s_Lih[b][i][q]; },
            [&](int i, int q) { return A[size_t(k0 + i) * ld + k0 + q]; }, lane);
#pragma unroll
        for (int t = 0; t < H / 16; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = k0 + 16 * t + Mfma<T>::drow(lk, v);
            if (col < h0 + hw) A[size_t(row) * ld + col] = x[t][v];
          }
      }
      __syncthreads();
      band_update<T, H, NT>(A, N, ld, k0 + H, h0, h0 + hw, k0, H, s_L);
    }
#pragma unroll 1
    for (int c0 = h0; c0 < h0 + hw; c0 += SB) {
      const int sb = min(SB, h0 + hw - c0);
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = c0 + tid + q * NT;
#pragma unroll
        for (int c = 0; c < SB; ++c)
          pr[q][c] = (row < N && c < sb) ? A[size_t(row) * ld + c0 + c] : T(0);
      }
#pragma unroll 1
      for (int j = 0; j < sb; ++j) {
        const int col = c0 + j;
        // candidates are rows col..N-1; a NaN counts as +inf so that it is
        // chosen and reported, and the chosen row always lies in [col, N)
        double best = -1.0;
        int bidx = col;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int row = c0 + tid + q * NT;
          T x = T(0);
#pragma unroll
          for (int c = 0; c < SB; ++c)
            if (c == j) x = pr[q][c];
          const double v = pivot_mag((double)x);
          if (row >= col && row < N && v > best) { best = v; bidx = row; }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          double ov = __shfl_xor(best, o, 64);
          int oi = __shfl_xor(bidx, o, 64);
          if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
        }
        if (lane == 0) { s_red_v[wid] = best; s_red_i[wid] = bidx; }
        __syncthreads();
        best = s_red_v[0];
        bidx = s_red_i[0];
#pragma unroll
        for (int w2 = 1; w2 < NW; ++w2) {
          double ov = s_red_v[w2];
          int oi = s_red_i[w2];
          if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
        }
        const int prow = min(max(bidx, col), N - 1);
        const int own_c = (col - c0) % NT, slot_c = (col - c0) / NT;
        const int own_p = (prow - c0) % NT, slot_p = (prow - c0) / NT;
        // the pivot row and the row it displaces through LDS, one barrier:
        // s_row (slot j & 1) holds the new row col, s_swap the old one
        T* prow_s = s_row[j & 1];
        T* crow_s = s_swap[j & 1];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (tid == own_p && q == slot_p)
#pragma unroll
            for (int c = 0; c < SB; ++c) prow_s[c] = pr[q][c];
          if (prow != col && tid == own_c && q == slot_c)
#pragma unroll
            for (int c = 0; c < SB; ++c) crow_s[c] = pr[q][c];
        }
        if (tid == 0) {
          s_piv[col - k0] = prow;
          if (s_status == 0) s_status = pivot_status(best, col);
        }
        __syncthreads();
        if (prow != col) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (tid == own_c && q == slot_c)
#pragma unroll
              for (int c = 0; c < SB; ++c) pr[q][c] = prow_s[c];
            if (tid == own_p && q == slot_p)
#pragma unroll
              for (int c = 0; c < SB; ++c) pr[q][c] = crow_s[c];
          }
        }
        if (best != 0.0) {
          const T piv = prow_s[j];
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            const int row = c0 + tid + q * NT;
            if (row > col && row < N) {
              T x = T(0);
#pragma unroll
              for (int c = 0; c < SB; ++c)
                if (c == j) x = pr[q][c];
              const T l = x / piv;   // one division per row
#pragma unroll
              for (int c = 0; c < SB; ++c) {
                if (c == j) pr[q][c] = l;
                if (c > j) pr[q][c] -= l * prow_s[c];
              }
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = c0 + tid + q * NT;
        if (row < N)
#pragma unroll
          for (int c = 0; c < SB; ++c)
            if (c < sb) A[size_t(row) * ld + c0 + c] = pr[q][c];
      }
      // the sub-panel's unit lower block (strict lower part, 16 x 16 frame)
      if (tid < 16)
#pragma unroll
        for (int c = 0; c < 16; ++c)
          s_Lb[tid][c] = (c < SB && tid < sb && c < tid) ? pr[0][c < SB ? c : 0] : T(0);
      __syncthreads();
      // the sub-panel's interchanges as row moves: thread 0 applies them to
      // the rows they touch (candidates: the sub-panel rows and the pivot
      // rows), then every candidate whose content changed is a move
      const int kc = tid % SB;
      const bool cand = tid < 2 * SB && kc < sb;
      const int cp = cand ? (tid < SB ? c0 + kc : s_piv[c0 - k0 + kc]) : 0;
      if (cand) s_sub[cp - k0] = cp;
      __syncthreads();
      if (tid == 0)
        for (int j = 0; j < sb; ++j) {
          const int a = c0 + j - k0, b = s_piv[c0 - k0 + j] - k0;
          const int ta = s_sub[a], tb = s_sub[b];
          s_sub[a] = tb;
          s_sub[b] = ta;
        }
      __syncthreads();
      int wpos = 0;
      if (tid < 2 * SB) {
        const int src = cand ? s_sub[cp - k0] : -1;
        s_md[tid] = (cand && src != cp) ? cp : -1;
        s_ms[tid] = src;
        if (cand) wpos = s_pos[src - k0];
      }
      __syncthreads();
      if (cand) s_pos[cp - k0] = wpos;   // the window's composition so far
      {
        // the moves in the other window columns: every moved value is read
        // before any is written
        constexpr int PARTS = NT / kSplitW, PV = (2 * SB + PARTS - 1) / PARTS;
        const int c = k0 + tid % kSplitW, part = tid / kSplitW;
        const bool act = c < cw1 && (c < c0 || c >= c0 + sb);
        T vals[PV];
#pragma unroll
        for (int q = 0; q < PV; ++q) {
          const int x = part + PARTS * q;
          vals[q] = (act && x < 2 * SB && s_md[x] >= 0) ? A[size_t(s_ms[x]) * ld + c] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PV; ++q) {
          const int x = part + PARTS * q;
          if (act && x < 2 * SB && s_md[x] >= 0) A[size_t(s_md[x]) * ld + c] = vals[q];
        }
      }
      __syncthreads();
      // the inverse of the sub-panel's unit lower block (in a 16 x 16 frame)
      invert_unit_lower16<T, NT>(s_Lb, s_Li, sb);
      // the inverse of the window's 16 x 16 diagonal block that ends here:
      // for the second half's solve (first-half blocks) and, when columns lie
      // right of the window, for the next launch
      const int gend = c0 + sb - k0;   // window columns done
      if ((gend & 15) == 0 || c0 + sb == cw1) {
        const int g0 = (gend - 1) & ~15;   // first window column of the block
        if constexpr (SB == 8) {
          if ((gend & 15) == 0) {   // two 8-column sub-panels: invert the whole block
            if (tid < 256) {
              const int i = tid >> 4, c = tid & 15;
              s_Lb[i][c] = c < i ? A[size_t(k0 + g0 + i) * ld + k0 + g0 + c] : T(0);
            }
            invert_unit_lower16<T, NT>(s_Lb, s_Lh, 16);
          }
        }
        T(*Lg)[17] = (SB == 8 && (gend & 15) == 0) ? s_Lh : s_Li;
        if (tid < 256) {
          const int i = tid >> 4, c = tid & 15;
          if (g0 < H) s_Lih[g0 >> 4][i][c] = Lg[i][c];
          if (cw1 < N && gend - g0 == 16)
            ((T*)(scratch + int64_t(blockIdx.x) * kSplitScratch + kMoveBytes))[g0 * 16 + tid] =
                Lg[i][c];
        }
        __syncthreads();
      }
      // the half's remaining columns: U rows of this sub-panel (MFMA with the
      // inverse block, one wavefront per 16 columns), then a rank-sb update
      const int b0 = c0 + sb, b1 = h0 + hw;
      if (b0 < b1) {
        if (wid < ((b1 - b0 + 15) >> 4)) {
          const int li = lane & 15, lk = lane >> 4, col = b0 + 16 * wid + li;
          typename Mfma<T>::acc y = {T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) {
            const int k = 4 * s2 + lk;
            const T bv = (col < b1 && c0 + k < N) ? A[size_t(c0 + k) * ld + col] : T(0);
            y = Mfma<T>::run(s_Li[li][k], bv, y);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = Mfma<T>::drow(lk, v);
            if (row < sb && col < b1) A[size_t(c0 + row) * ld + col] = y[v];
          }
        }
        __syncthreads();
        band_update<T, SB, NT>(A, N, ld, b0, b0, b1, c0, sb, s_L);
      }
    }
  }
  // The window's interchanges as row moves for the columns outside it, and
  // the permutation: row k0 + r now holds the old content of row s_pos[r]
  {
    int pv[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + q * NT;
      pv[q] = (r < N - k0 && s_pos[r] != k0 + r) ? perm[s_pos[r]] : 0;
    }
    __syncthreads();
    const bool outside = k0 > 0 || cw1 < N;
    int32_t* mv = (int32_t*)(scratch + int64_t(blockIdx.x) * kSplitScratch);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + q * NT;
      if (r < N - k0 && s_pos[r] != k0 + r) {
        perm[k0 + r] = pv[q];
        if (outside) {
          const int x = atomicAdd(&s_cnt, 1);
          mv[1 + 2 * x] = k0 + r;
          mv[2 + 2 * x] = s_pos[r];
        }
      }
    }
    __syncthreads();
    if (outside && tid == 0) mv[0] = s_cnt;
  }
  if (tid == 0) status[e] = s_status;
}

// One workgroup per 64 columns outside the window (blockIdx.x: the chunks left
// of the window, then those right of it; blockIdx.y: the macro).  Wavefront
// g holds the window rows of columns cb + 16 g .. cb + 16 g + 15 in registers
// (accumulator layout); right of the window it then solves U12 = L11^-1 A12
// for them on its own.
template <typename T>
__global__ __launch_bounds__(256, 4) void lu_swap_u12_kernel(T* fac, const MacroInfo* __restrict__ info,
                                                          const int32_t* __restrict__ order,
                                                          int64_t base, int k0,
                                                          const char* __restrict__ scratch) {
  constexpr int W = kSplitW, NB = W / 16;
  const int e = order[base + blockIdx.y];
  const MacroInfo& mi = info[e];
  const int N = mi.N, ld = mi.ld;
  T* A = fac + mi.fac_off;
  const char* scr = scratch + int64_t(blockIdx.y) * kSplitScratch;
  const int32_t* mv = (const int32_t*)scr;
  const T* lis = (const T*)(scr + kMoveBytes);
  const int w = min(W, N - k0), cw1 = k0 + w;
  const int nl = (k0 + 63) >> 6;
  const bool right = int(blockIdx.x) >= nl;
  const int cb = right ? cw1 + 64 * (int(blockIdx.x) - nl) : 64 * int(blockIdx.x);
  const int ce = right ? N : k0;
  if (cb >= ce) return;
  const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;

  __shared__ int s_src[W];          // source row of each window row's new content
  __shared__ int s_od[W], s_os[W];  // moves into rows below the window
  __shared__ int s_no;
  for (int t = tid; t < W; t += 256) s_src[t] = k0 + t;
  if (tid == 0) s_no = 0;
  __syncthreads();
  const int np = mv[0];
  for (int p = tid; p < np; p += 256) {
    const int d = mv[1 + 2 * p], s = mv[2 + 2 * p];
    if (d < cw1) {
      s_src[d - k0] = s;
    } else {
      const int q = atomicAdd(&s_no, 1);
      s_od[q] = d;
      s_os[q] = s;
    }
  }
  __syncthreads();
  // every source is read before any row is written
  const int col = cb + 16 * g + li;
  const bool cok = col < ce;
  typename Mfma<T>::acc x[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + Mfma<T>::drow(lk, v);
      x[t][v] = (cok && row < w) ? A[size_t(s_src[row]) * ld + col] : T(0);
    }
  __syncthreads();
  {
    // rows below the window take the old content of window rows
    const int no = s_no, c = cb + lane;
    if (c < ce)
      for (int q = g; q < no; q += 4)
        A[size_t(s_od[q]) * ld + c] = A[size_t(s_os[q]) * ld + c];
  }
  if (right)   // w == W here: the window is full when columns lie right of it
    wave_trsm<T, NB>(
        x, NB, [&](int b, int i, int q) { return lis[b * 256 + i * 16 + q]; },
        [&](int i, int q) { return A[size_t(k0 + i) * ld + k0 + q]; }, lane);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < NB; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + Mfma<T>::drow(lk, v);
      if (cok && row < w && (right || s_src[row] != k0 + row))
        A[size_t(k0 + row) * ld + col] = x[t][v];
    }
}

// A22 -= L21 U12 for one TM x TN tile of the trailing matrix (rows and
// columns from k0 + W).  Workgroups are dispatched to the XCDs in turn
// (block b runs on XCD b mod 8), so macro 8 m + x of the class takes the
// blocks b = 8 (m T2 + tile) + x: all its T2 tiles on XCD x, one after another.
// Wavefront v computes the (TM/2) x (TN/2) quarter (v / 2, v mod 2) of the
// tile as MFMA tiles; the next 16-deep slices of L21 and U12 are loaded into
// registers while the current ones are multiplied out of LDS.
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256, 4) void lu_update_kernel(T* fac, const MacroInfo* __restrict__ info,
                                                        const int32_t* __restrict__ order,
                                                        int64_t base, int count, int k0, int tpr,
                                                        int tpc) {
  constexpr int W = kSplitW, KC = 16;
  constexpr int PL = TM * KC / 256, PU = KC * TN / 256;   // prefetched values per thread
  constexpr int MI = TM / 32, NI = TN / 32;                // MFMA tiles per wavefront
  const int b = blockIdx.x, x = b & 7, i = b >> 3;
  const int T2 = tpr * tpc;
  const int mpos = (i / T2) * 8 + x;
  if (mpos >= count) return;
  const int tile = i % T2;
  const int e = order[base + mpos];
  const MacroInfo& mi = info[e];
  const int N = mi.N, ld = mi.ld;
  T* A = fac + mi.fac_off;
  const int r0 = k0 + W;
  const int row0 = r0 + TM * (tile / tpc), col0 = r0 + TN * (tile % tpc);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (TM / 2) * (wid >> 1), wc = (TN / 2) * (wid & 1);

  __shared__ T Ls[TM][KC + 1];
  __shared__ T Us[KC][TN + 1];
  T pl[PL], pu[PU];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int x2 = tid + 256 * q;
      const int r = x2 / KC, k = x2 % KC, row = row0 + r;
      pl[q] = row < N ? -A[size_t(row) * ld + k0 + kc + k] : T(0);
    }
#pragma unroll
    for (int q = 0; q < PU; ++q) {
      const int x2 = tid + 256 * q;
      const int kk = x2 / TN, cc = x2 % TN, col = col0 + cc;
      pu[q] = col < N ? A[size_t(k0 + kc + kk) * ld + col] : T(0);
    }
  };
  fetch(0);
  typename Mfma<T>::acc acc[MI][NI];
#pragma unroll
  for (int ti = 0; ti < MI; ++ti)
#pragma unroll
    for (int tj = 0; tj < NI; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wr + 16 * ti + Mfma<T>::drow(lk, v);
        const int col = col0 + wc + 16 * tj + li;
        acc[ti][tj][v] = (row < N && col < N) ? A[size_t(row) * ld + col] : T(0);
      }
#pragma unroll 1
  for (int kc = 0; kc < W; kc += KC) {
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int x2 = tid + 256 * q;
      Ls[x2 / KC][x2 % KC] = pl[q];
    }
#pragma unroll
    for (int q = 0; q < PU; ++q) {
      const int x2 = tid + 256 * q;
      Us[x2 / TN][x2 % TN] = pu[q];
    }
    __syncthreads();
    if (kc + KC < W) fetch(kc + KC);
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = 4 * s + lk;
      T a[MI], bb[NI];
#pragma unroll
      for (int ti = 0; ti < MI; ++ti) a[ti] = Ls[wr + 16 * ti + li][k];
#pragma unroll
      for (int tj = 0; tj < NI; ++tj) bb[tj] = Us[k][wc + 16 * tj + li];
#pragma unroll
      for (int ti = 0; ti < MI; ++ti)
#pragma unroll
        for (int tj = 0; tj < NI; ++tj) acc[ti][tj] = Mfma<T>::run(a[ti], bb[tj], acc[ti][tj]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < MI; ++ti)
#pragma unroll
    for (int tj = 0; tj < NI; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wr + 16 * ti + Mfma<T>::drow(lk, v);
        const int col = col0 + wc + 16 * tj + li;
        if (row < N && col < N) A[size_t(row) * ld + col] = acc[ti][tj][v];
      }
}

// In-place transpose to column-major: workgroup (p, macro) swaps the 32 x 32
// tiles (I, J) and (J, I) of the p-th pair I <= J.
template <typename T>
__global__ __launch_bounds__(256) void lu_transpose_kernel(T* fac, const MacroInfo* __restrict__ info,
                                                           const int32_t* __restrict__ order,
                                                           int64_t base, int nt) {
  const int e = order[base + blockIdx.y];
  const MacroInfo& mi = info[e];
  const int N = mi.N, ld = mi.ld;
  T* A = fac + mi.fac_off;
  int p = blockIdx.x, I = 0;
  while (p >= nt - I) { p -= nt - I; ++I; }
  const int J = I + p;
  __shared__ T t0[32][33];
  __shared__ T t1[32][33];
  const int tid = threadIdx.x;
  for (int x = tid; x < 1024; x += 256) {
    const int a = x >> 5, b = x & 31;
    const int r = 32 * I + a, c = 32 * J + b;
    t0[a][b] = (r < N && c < N) ? A[size_t(r) * ld + c] : T(0);
    const int r2 = 32 * J + a, c2 = 32 * I + b;
    t1[a][b] = (r2 < N && c2 < N) ? A[size_t(r2) * ld + c2] : T(0);
  }
  __syncthreads();
  for (int x = tid; x < 1024; x += 256) {
    const int a = x >> 5, b = x & 31;
    const int r = 32 * I + a, c = 32 * J + b;
    if (r < N && c < N) A[size_t(r) * ld + c] = t1[b][a];
    const int r2 = 32 * J + a, c2 = 32 * I + b;
    if (r2 < N && c2 < N) A[size_t(r2) * ld + c2] = t0[b][a];
  }
}

size_t lu_split_scratch_bytes(const SizeClass& c) {
  return c.N > kSplitW ? size_t(c.count) * kSplitScratch : 0;
}

template <typename T>
hipError_t lu_split_class(T* fac, const MacroInfo* info, const int32_t* order, const SizeClass& c,
                          int32_t* perm, int32_t* status, char* scratch, size_t scratch_bytes,
                          hipStream_t s) {
  const int N = c.N;
  const int64_t cnt = c.count;
  if (N > 4096) return hipErrorInvalidValue;
  if (lu_split_scratch_bytes(c) > scratch_bytes || (N > kSplitW && !scratch))
    return hipErrorInvalidValue;
  for (int k0 = 0; k0 < N; k0 += kSplitW) {
    const int w = std::min(kSplitW, N - k0);
    if (N - k0 <= 1024)
      hipLaunchKernelGGL((lu_panel_kernel<T, 256, 4, 16>), dim3((unsigned)cnt), dim3(256), 0, s,
                         fac, info, order, c.start, k0, perm, status, scratch);
    else
      hipLaunchKernelGGL((lu_panel_kernel<T, 512, 8, 8>), dim3((unsigned)cnt), dim3(512), 0, s,
                         fac, info, order, c.start, k0, perm, status, scratch);
    const int nl = (k0 + 63) / 64, nr = (N - k0 - w + 63) / 64;
    if (nl + nr > 0)
      hipLaunchKernelGGL(lu_swap_u12_kernel<T>, dim3((unsigned)(nl + nr), (unsigned)cnt), dim3(256),
                         0, s, fac, info, order, c.start, k0, (const char*)scratch);
    if (k0 + w < N) {
      const int tpd = (N - k0 - w + 63) / 64;
      const int64_t blocks = (cnt + 7) / 8 * 8 * int64_t(tpd) * tpd;
      hipLaunchKernelGGL((lu_update_kernel<T, 64, 64>), dim3((unsigned)blocks), dim3(256), 0, s,
                         fac, info, order, c.start, (int)cnt, k0, tpd, tpd);
    }
  }
  const int nt = (N + 31) / 32;
  hipLaunchKernelGGL(lu_transpose_kernel<T>, dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)cnt),
                     dim3(256), 0, s, fac, info, order, c.start, nt);
  return hipGetLastError();
}

template hipError_t lu_split_class<double>(double*, const MacroInfo*, const int32_t*,
                                           const SizeClass&, int32_t*, int32_t*, char*, size_t,
                                           hipStream_t);
template hipError_t lu_split_class<float>(float*, const MacroInfo*, const int32_t*,
                                          const SizeClass&, int32_t*, int32_t*, char*, size_t,
                                          hipStream_t);

}  // namespace mhdg
