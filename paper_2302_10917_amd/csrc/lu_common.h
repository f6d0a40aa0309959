// Device helpers shared by the blocked factorisation kernels.
#pragma once
#include "internal.h"
#include "mfma.h"

namespace mhdg {

// A[r0:N, c0:c1] -= A[r0:N, kc:kc+kw] A[kc:kc+kw, c0:c1] (row-major, leading
// dimension ld, kw <= KW) on 16 x 16 MFMA tiles.  Wavefront w takes the row
// tiles w, w + NW, ...; a row tile keeps its K-slab of L in registers while
// the column tiles stream through, so the wavefronts of the workgroup read
// the same U tiles at about the same time (cache hits) and every element of
// the updated block is read and written once.
template <typename T, int KW, int NW>
__device__ __forceinline__ void slab_update(T* __restrict__ A, int N, int ld, int r0, int c0,
                                            int c1, int kc, int kw, int wid, int lane) {
  constexpr int S = KW / 4;
  const int nrt = (N - r0 + 15) >> 4, nct = (c1 - c0 + 15) >> 4;
  const int li = lane & 15, lk = lane >> 4;
  for (int rt = wid; rt < nrt; rt += NW) {
    const int rr = r0 + 16 * rt;
    T a[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = 4 * s + lk, row = rr + li;
      a[s] = (row < N && k < kw) ? -A[size_t(row) * ld + kc + k] : T(0);
    }
    for (int ct = 0; ct < nct; ++ct) {
      const int col = c0 + 16 * ct + li;
      const bool cok = col < c1;
      typename Mfma<T>::acc acc0, acc1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rr + Mfma<T>::drow(lk, v);
        acc0[v] = (row < N && cok) ? A[size_t(row) * ld + col] : T(0);
        acc1[v] = T(0);
      }
      // the U slab in chunks of CH k-steps (bounded registers); two
      // accumulation chains so that independent MFMAs overlap
      constexpr int CH = S < 8 ? S : 8;
#pragma unroll
      for (int h = 0; h < S; h += CH) {
        T b[CH];
#pragma unroll
        for (int s = 0; s < CH; ++s) {
          const int k = 4 * (h + s) + lk;
          b[s] = (cok && k < kw) ? A[size_t(kc + k) * ld + col] : T(0);
        }
#pragma unroll
        for (int s = 0; s < CH; s += 2) {
          acc0 = Mfma<T>::run(a[h + s], b[s], acc0);
          if (s + 1 < CH) acc1 = Mfma<T>::run(a[h + s + 1], b[s + 1], acc1);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rr + Mfma<T>::drow(lk, v);
        if (row < N && cok) A[size_t(row) * ld + col] = acc0[v] + acc1[v];
      }
    }
  }
}

}  // namespace mhdg
