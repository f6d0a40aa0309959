// Two-level blocked LU with partial pivoting for the larger local sizes.
//
// The same factorisation as lu_kernel (PA = LU, largest |a| pivots with
// ties to the smallest row, factors stored column-major on exit), organised
// to read the trailing matrix far fewer times: panels of NB columns, each
// factored as SB-column sub-panels held in registers (right-looking inside
// the panel, rank-SB MFMA updates of the panel's remaining columns only),
// then U12 = L11^-1 A12 by SB-row blocks against L11 in LDS, and one rank-NB
// MFMA update A22 -= L21 U12 per panel.  With NB = 64 the trailing matrix is
// read and written N/64 times instead of N/8 times.
#include "internal.h"
#include "lu_common.h"
#include "mfma.h"

namespace mhdg {

// The same update with the U slab shared through LDS: the workgroup walks
// groups of NW * RT row tiles; each wavefront keeps the L slab of its RT row
// tiles in registers, and every 16-column tile of U is loaded once per row
// group into LDS (Us: KW x 16 values) for all of them.  U is then read
// ceil(rows / (16 NW RT)) times instead of once per row tile, and every
// element of the updated block is still read and written once.
template <typename T, int KW, int NW, int RT>
__device__ __forceinline__ void slab_update_lds(T* __restrict__ A, int N, int ld, int r0, int c0,
                                                int c1, int kc, int kw, int wid, int lane,
                                                T* __restrict__ Us) {
  constexpr int S = KW / 4;
  const int nrt = (N - r0 + 15) >> 4, nct = (c1 - c0 + 15) >> 4;
  const int li = lane & 15, lk = lane >> 4;
  const int tid = wid * 64 + lane;
  for (int rg = 0; rg < nrt; rg += NW * RT) {
    T a[RT][S];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int row = r0 + 16 * (rg + wid * RT + t) + li;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int k = 4 * s + lk;
        a[t][s] = (row < N && k < kw) ? -A[size_t(row) * ld + kc + k] : T(0);
      }
    }
    for (int ct = 0; ct < nct; ++ct) {
      const int cb = c0 + 16 * ct;
      __syncthreads();   // the previous tile's readers are done
      for (int x = tid; x < KW * 16; x += NW * 64) {
        const int k = x >> 4, c = x & 15;
        Us[x] = (k < kw && cb + c < c1) ? A[size_t(kc + k) * ld + cb + c] : T(0);
      }
      __syncthreads();
      T b[S];
#pragma unroll
      for (int s = 0; s < S; ++s) b[s] = Us[(4 * s + lk) * 16 + li];
      const int col = cb + li;
      const bool cok = col < c1;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int rr = r0 + 16 * (rg + wid * RT + t);
        if (rr >= N) break;
        typename Mfma<T>::acc acc0, acc1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = rr + Mfma<T>::drow(lk, v);
          acc0[v] = (row < N && cok) ? A[size_t(row) * ld + col] : T(0);
          acc1[v] = T(0);
        }
#pragma unroll
        for (int s = 0; s < S; s += 2) {
          acc0 = Mfma<T>::run(a[t][s], b[s], acc0);
          if (s + 1 < S) acc1 = Mfma<T>::run(a[t][s + 1], b[s + 1], acc1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = rr + Mfma<T>::drow(lk, v);
          if (row < N && cok) A[size_t(row) * ld + col] = acc0[v] + acc1[v];
        }
      }
    }
  }
}

// One workgroup of NT threads per macro; thread t owns the sub-panel rows
// c0 + t + q NT (q < RPT), so RPT * NT >= N is required.  TRT: row tiles
// per wavefront in the trailing update with U tiles shared through LDS
// (slab_update_lds; each keeps NB / 4 L values per row tile in registers),
// or 0 for the update that streams U from memory per row tile.
template <typename T, int NT, int RPT, int NB, int SB, int TRT>
__global__ __launch_bounds__(NT) void lu_blocked_kernel(T* fac, const MacroInfo* __restrict__ info,
                                                        const int32_t* __restrict__ order,
                                                        int64_t base, int32_t* perm_all,
                                                        int32_t* status) {
  static_assert(NB % SB == 0 && SB % 4 == 0 && NB % 8 == 0, "panel shapes");
  constexpr int NW = NT / 64;
  const int e = order[base + blockIdx.x];
  const MacroInfo& mi = info[e];
  const int N = mi.N, ld = mi.ld;   // rows of the stored block are ld apart
  T* A = fac + mi.fac_off;
  int32_t* perm = perm_all + mi.loc_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  __shared__ double s_red_v[NW];
  __shared__ int s_red_i[NW];
  __shared__ T s_row[SB];
  __shared__ T s_swap[2][SB];
  __shared__ T s_L[NB * NB];   // L11 of the U12 solve; U tiles of the trailing update
  __shared__ int s_piv[SB];
  __shared__ int s_status;

  for (int i = tid; i < N; i += NT) perm[i] = i;
  if (tid == 0) s_status = 0;
  __syncthreads();

  T pr[RPT][SB];
  for (int k0 = 0; k0 < N; k0 += NB) {
    const int nb = min(NB, N - k0);
    // ---------------- panel: SB-column sub-panels, right-looking inside the panel
    for (int s0 = 0; s0 < nb; s0 += SB) {
      const int c0 = k0 + s0, sb = min(SB, nb - s0);
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = c0 + tid + q * NT;
#pragma unroll
        for (int c = 0; c < SB; ++c)
          pr[q][c] = (row < N && c < sb) ? A[size_t(row) * ld + c0 + c] : T(0);
      }
      for (int j = 0; j < sb; ++j) {
        const int col = c0 + j;
        // candidates are rows col..N-1; a NaN counts as +inf so that it is
        // chosen and reported, and the chosen row always lies in [col, N)
        double best = -1.0;
        int bidx = col;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int row = c0 + tid + q * NT;
          double v = -1.0;
#pragma unroll
          for (int c = 0; c < SB; ++c)
            if (c == j) v = pivot_mag((double)pr[q][c]);
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
        for (int w = 1; w < NW; ++w) {
          double ov = s_red_v[w];
          int oi = s_red_i[w];
          if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
        }
        const int prow = min(max(bidx, col), N - 1);
        const int own_c = (col - c0) % NT, slot_c = (col - c0) / NT;
        const int own_p = (prow - c0) % NT, slot_p = (prow - c0) / NT;
        if (prow != col) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (tid == own_p && q == slot_p)
              for (int c = 0; c < SB; ++c) s_swap[0][c] = pr[q][c];
            if (tid == own_c && q == slot_c)
              for (int c = 0; c < SB; ++c) s_swap[1][c] = pr[q][c];
          }
        }
        __syncthreads();
        if (prow != col) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (tid == own_c && q == slot_c)
              for (int c = 0; c < SB; ++c) pr[q][c] = s_swap[0][c];
            if (tid == own_p && q == slot_p)
              for (int c = 0; c < SB; ++c) pr[q][c] = s_swap[1][c];
          }
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (tid == own_c && q == slot_c)
            for (int c = 0; c < SB; ++c) s_row[c] = pr[q][c];
        if (tid == 0) {
          s_piv[j] = prow;
          if (s_status == 0) s_status = pivot_status(best, col);
        }
        __syncthreads();
        if (best != 0.0) {
          const T piv = s_row[j];
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            const int row = c0 + tid + q * NT;
            if (row > col && row < N) {
              T l = T(0);
#pragma unroll
              for (int c = 0; c < SB; ++c)
                if (c == j) { l = pr[q][c] / piv; pr[q][c] = l; }
#pragma unroll
              for (int c = 0; c < SB; ++c)
                if (c > j) pr[q][c] -= l * s_row[c];
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
      __syncthreads();
      // row interchanges in every column outside the sub-panel, in pivot order
      for (int c = tid; c < N; c += NT) {
        if (c >= c0 && c < c0 + sb) continue;
        for (int j = 0; j < sb; ++j) {
          const int prow = s_piv[j], col = c0 + j;
          if (prow != col) {
            T a = A[size_t(col) * ld + c], b = A[size_t(prow) * ld + c];
            A[size_t(col) * ld + c] = b;
            A[size_t(prow) * ld + c] = a;
          }
        }
      }
      if (tid == 0)
        for (int j = 0; j < sb; ++j) {
          const int prow = s_piv[j], col = c0 + j;
          if (prow != col) { int t = perm[col]; perm[col] = perm[prow]; perm[prow] = t; }
        }
      __syncthreads();
      // the panel's remaining columns: U rows of this sub-panel, then a rank-sb update
      const int b0 = c0 + sb, b1 = k0 + nb;
      if (b0 < b1) {
        for (int c = b0 + tid; c < b1; c += NT) {
          T v[SB];
#pragma unroll
          for (int jj = 0; jj < SB; ++jj) v[jj] = jj < sb ? A[size_t(c0 + jj) * ld + c] : T(0);
#pragma unroll
          for (int jj = 1; jj < SB; ++jj)
#pragma unroll
            for (int ii = 0; ii < jj; ++ii)
              if (jj < sb) v[jj] -= A[size_t(c0 + jj) * ld + c0 + ii] * v[ii];
#pragma unroll
          for (int jj = 0; jj < SB; ++jj)
            if (jj < sb) A[size_t(c0 + jj) * ld + c] = v[jj];
        }
        __syncthreads();
        slab_update<T, SB, NW>(A, N, ld, b0, b0, b1, c0, sb, wid, lane);
        __syncthreads();
      }
    }
    if (k0 + nb >= N) break;
    // ---------------- U12 = L11^-1 A12, SB-row blocks, L11 in LDS
    for (int i = tid; i < NB * NB; i += NT) {
      const int r = i / NB, c = i % NB;
      s_L[i] = (r < nb && c < r) ? A[size_t(k0 + r) * ld + k0 + c] : T(0);
    }
    __syncthreads();
    for (int c = k0 + nb + tid; c < N; c += NT) {
      for (int b = 0; b < nb; b += SB) {
        T v[SB];
#pragma unroll
        for (int jj = 0; jj < SB; ++jj) v[jj] = b + jj < nb ? A[size_t(k0 + b + jj) * ld + c] : T(0);
        for (int i = 0; i < b; ++i) {
          const T x = A[size_t(k0 + i) * ld + c];   // finished U entry (written by this thread)
#pragma unroll
          for (int jj = 0; jj < SB; ++jj) v[jj] -= s_L[(b + jj) * NB + i] * x;
        }
#pragma unroll
        for (int jj = 1; jj < SB; ++jj)
#pragma unroll
          for (int ii = 0; ii < jj; ++ii) v[jj] -= s_L[(b + jj) * NB + b + ii] * v[ii];
#pragma unroll
        for (int jj = 0; jj < SB; ++jj)
          if (b + jj < nb) A[size_t(k0 + b + jj) * ld + c] = v[jj];
      }
    }
    __syncthreads();
    // ---------------- A22 -= L21 U12 (rank nb)
    if constexpr (TRT > 0)
      slab_update_lds<T, NB, NW, TRT>(A, N, ld, k0 + nb, k0 + nb, N, k0, nb, wid, lane, s_L);
    else
      slab_update<T, NB, NW>(A, N, ld, k0 + nb, k0 + nb, N, k0, nb, wid, lane);
    __syncthreads();
  }
  // ---- store the factors column-major (in-place transpose by 32 x 32 tile pairs)
  {
    __shared__ T t0[32][33];
    __shared__ T t1[32][33];
    const int nt = (N + 31) / 32;
    for (int I = 0; I < nt; ++I)
      for (int J = I; J < nt; ++J) {
        for (int x = tid; x < 1024; x += NT) {
          const int a = x >> 5, b = x & 31;
          const int r = 32 * I + a, c = 32 * J + b;
          t0[a][b] = (r < N && c < N) ? A[size_t(r) * ld + c] : T(0);
          const int r2 = 32 * J + a, c2 = 32 * I + b;
          t1[a][b] = (r2 < N && c2 < N) ? A[size_t(r2) * ld + c2] : T(0);
        }
        __syncthreads();
        for (int x = tid; x < 1024; x += NT) {
          const int a = x >> 5, b = x & 31;
          const int r = 32 * I + a, c = 32 * J + b;
          if (r < N && c < N) A[size_t(r) * ld + c] = t1[b][a];
          const int r2 = 32 * J + a, c2 = 32 * I + b;
          if (r2 < N && c2 < N) A[size_t(r2) * ld + c2] = t0[b][a];
        }
        __syncthreads();
      }
  }
  if (tid == 0) status[e] = s_status;
}

// Blocked NB = 64 / SB = 8 with 256 threads (N <= 1024) or 512 threads
// (N <= 4096); TRT from the variant (LU_BLOCKED: 0, LU_BLOCKED_U2: 2,
// LU_BLOCKED_U4: 4).
template <typename T, int TRT>
static hipError_t lu_blocked_launch(T* fac, const MacroInfo* info, const int32_t* order,
                                    const SizeClass& c, int32_t* perm, int32_t* status,
                                    hipStream_t s) {
  const dim3 g((unsigned)c.count);
  if (c.N <= 1024)
    hipLaunchKernelGGL((lu_blocked_kernel<T, 256, 4, 64, 8, TRT>), g, dim3(256), 0, s, fac, info,
                       order, c.start, perm, status);
  else if (c.N <= 4096)   // 8 wavefronts
    hipLaunchKernelGGL((lu_blocked_kernel<T, 512, 8, 64, 8, TRT>), g, dim3(512), 0, s, fac, info,
                       order, c.start, perm, status);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t lu_blocked_class(int variant, T* fac, const MacroInfo* info, const int32_t* order,
                            const SizeClass& c, int32_t* perm, int32_t* status, hipStream_t s) {
  if (variant == LU_BLOCKED_U2) return lu_blocked_launch<T, 2>(fac, info, order, c, perm, status, s);
  if (variant == LU_BLOCKED_U4) return lu_blocked_launch<T, 4>(fac, info, order, c, perm, status, s);
  return lu_blocked_launch<T, 0>(fac, info, order, c, perm, status, s);
}

template hipError_t lu_blocked_class<double>(int, double*, const MacroInfo*, const int32_t*,
                                             const SizeClass&, int32_t*, int32_t*, hipStream_t);
template hipError_t lu_blocked_class<float>(int, float*, const MacroInfo*, const int32_t*,
                                            const SizeClass&, int32_t*, int32_t*, hipStream_t);

}  // namespace mhdg
