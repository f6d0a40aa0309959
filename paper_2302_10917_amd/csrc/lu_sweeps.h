// Triangular sweeps with several right-hand sides at once on a macro's
// stored FP64 LU factors (used by the folded-operator build and the
// many-vector apply).
#pragma once
#include "macro_solve.h"

namespace mhdg {

// Forward and backward substitution with NR right-hand sides at once, on the
// FP64 factors of one macro (unit lower L and upper U stored column-major in
// place, leading dimension ld, N rows).  Lane l holds rows l + 64 q of every
// right-hand side in y[q][.]; the rows are already permuted.  Each factor
// column is loaded once and used for all NR right-hand sides.  NQ may exceed
// ceil(N / 64): row indices are clamped to the column and rows past N take no
// part.
template <int NQ, int NR>
__device__ __forceinline__ void lu_sweeps_nr(double (&y)[NQ][NR], const double* __restrict__ A,
                                             int N, int ld, int lane) {
  constexpr int kLG = kLoadGroup;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jend = min(64, N - 64 * q);
    for (int jj = 0; jj < jend; ++jj) {
      const int j = 64 * q + jj;
      double yj[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) yj[r] = readlane_d(y[q][r], jj);
      const double* col = A + size_t(j) * ld;
#pragma unroll
      for (int g = q; g < NQ; g += kLG) {
        double a[kLG];
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int rw = lane + 64 * (g + t);
          int rr = (g + t == q && rw <= j) ? j + 1 : rw;
          rr = rr < N ? rr : N - 1;
          a[t] = (g + t < NQ) ? col[rr] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int rw = lane + 64 * (g + t);
          if (g + t < NQ) {
            const double av = (rw > j && rw < N) ? a[t] : 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) y[g + t][r] -= av * yj[r];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
#pragma unroll
  for (int q = NQ - 1; q >= 0; --q) {
    const int jend = min(64, N - 64 * q);
    for (int jj = jend - 1; jj >= 0; --jj) {
      const int j = 64 * q + jj;
      const double* col = A + size_t(j) * ld;
      const double dj = col[j];
      double zj[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        zj[r] = readlane_d(y[q][r], jj) / dj;
        if (lane == jj) y[q][r] = zj[r];
      }
#pragma unroll
      for (int g = 0; g <= q; g += kLG) {
        double a[kLG];
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int rw = lane + 64 * (g + t);
          const int rr = (g + t == q && rw >= j) ? (j > 0 ? j - 1 : 0) : rw;
          a[t] = (g + t <= q) ? col[rr] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int rw = lane + 64 * (g + t);
          if (g + t <= q) {
            const double av = rw < j ? a[t] : 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) y[g + t][r] -= av * zj[r];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

}  // namespace mhdg
