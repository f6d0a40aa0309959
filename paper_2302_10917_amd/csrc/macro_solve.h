// Per-macro solve kernel of the trace operator (steps 1-3), the local
// right-hand-side solve and the local recovery.  Included by the translation
// units that instantiate it for each register-block count NQ (split so the
// fully unrolled instances compile in parallel).
#pragma once
#include "internal.h"

namespace mhdg {

__device__ __forceinline__ const int32_t* ints_(const double* base, int64_t off) {
  return reinterpret_cast<const int32_t*>(base + off);
}

// ------------------------------------------------------------------ per-macro solves
// Boundary entries of a macro's local vectors are kept compactly: field f
// (q_x, q_y, u), boundary position b = kP + s (edge k, position s < P along
// it), index f * 3P + b.  Only these rows of x = B lam and of C y are nonzero.
__device__ __forceinline__ int bpos(int k, int s, int P) { return s < P ? k * P + s : ((k + 1) % 3) * P; }

__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// xc += sgn * B_k lam_F (step 1): the rows v_x, v_y, w of the boundary nodes
// of edge k receive n_x g, n_y g, (a.n - tau) g with g_s = |F| sum_l
// T1[s][l] lam_l, T1 coupling the level-r edge space with the face's trace
// space, both in the face's canonical direction.
__device__ inline void edge_B(const MacroInfo& mi, int k, const double* tm, const Templates& Tp,
                       const double* lamF, double sgn, double bx, double by, double tau,
                       double* xc) {
  const LevelTemplates& L = Tp.lev[mi.level];
  const int P = mi.P, NBD = 3 * P, fl = mi.flevel[k];
  const int nF = (1 << fl) * Tp.p + 1;
  const double* T1 = tm + L.T1[fl];
  const double nx = mi.nrm[2 * k], ny = mi.nrm[2 * k + 1];
  const double an = bx * nx + by * ny - tau;
  for (int s = threadIdx.x; s <= P; s += blockDim.x) {
    const int sc = mi.orient[k] > 0 ? s : P - s;
    double g = 0.0;
    for (int l = 0; l < nF; ++l) g += T1[size_t(sc) * nF + l] * lamF[l];
    g *= sgn * mi.len[k];
    const int b = bpos(k, s, P);
    xc[b] += nx * g;
    xc[NBD + b] += ny * g;
    xc[2 * NBD + b] += an * g;
  }
}

// out_l = (C_k z)_l = |F| sum_s T1[s][l] (kappa n.q + tau u)(boundary node s) (step 3)
__device__ inline void edge_C(const MacroInfo& mi, int k, const double* tm, const Templates& Tp,
                       const double* zc, double tau, double* out) {
  const LevelTemplates& L = Tp.lev[mi.level];
  const int P = mi.P, NBD = 3 * P, fl = mi.flevel[k];
  const int nF = (1 << fl) * Tp.p + 1;
  const double* T1 = tm + L.T1[fl];
  const double kx = mi.kappa * mi.nrm[2 * k], ky = mi.kappa * mi.nrm[2 * k + 1];
  for (int l = threadIdx.x; l < nF; l += blockDim.x) {
    double v = 0.0;
    for (int sc = 0; sc <= P; ++sc) {
      const int b = bpos(k, mi.orient[k] > 0 ? sc : P - sc, P);
      v += T1[size_t(sc) * nF + l] * (kx * zc[b] + ky * zc[NBD + b] + tau * zc[2 * NBD + b]);
    }
    out[l] = mi.len[k] * v;
  }
}

// One wavefront per macro.  The permuted right-hand side and then the
// solution live in registers, lane l holding entries l + 64 q.  Forward and
// backward substitution run column by column over the column-major factors:
// each step broadcasts one solved entry (readlane) and updates the remaining
// entries with one contiguous column of L or U, so the loads of a column do
// not wait on any reduction and the factor streams from HBM exactly once.
// Resident wavefronts per SIMD the register budget is sized for: all macros
// of a large mesh should be resident at once (8 waves/SIMD = 64 VGPRs).
constexpr int kLoadGroup = 8;
template <int NQ> struct SolveOccupancy { static constexpr int waves = NQ <= 16 ? 8 : (NQ <= 27 ? 4 : 2); };

template <typename T, int NQ>
__global__ __launch_bounds__(64, SolveOccupancy<NQ>::waves) void macro_solve_kernel(int mode, const T* __restrict__ fac,
                                                         const MacroInfo* __restrict__ info,
                                                         const int32_t* __restrict__ perm_all,
                                                         const double* __restrict__ tm, Templates Tp,
                                                         double bx, double by, double tau,
                                                         const double* __restrict__ lam,
                                                         const double* xin, double* yout,
                                                         double* __restrict__ slots) {
  extern __shared__ double sm[];
  const MacroInfo& mi = info[blockIdx.x];
  const int N = mi.N, Q = mi.Q, P = mi.P, NBD = 3 * P, lane = threadIdx.x;
  double* xc = sm;             // compact boundary rows of the right-hand side
  double* zc = sm + 3 * NBD;   // compact boundary rows of the solution
  const int32_t* bidx = ints_(tm, Tp.lev[mi.level].bnd_index);
  const T* A = fac + mi.fac_off;
  const int32_t* perm = perm_all + mi.loc_off;
  const bool with_B = mode == MODE_APPLY || mode == MODE_RECOVER;
  if (with_B) {
    for (int i = lane; i < 3 * NBD; i += 64) xc[i] = 0.0;
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
      if (mi.tr_off[k] >= 0)
        edge_B(mi, k, tm, Tp, lam + mi.tr_off[k], mode == MODE_APPLY ? 1.0 : -1.0, bx, by, tau, xc);
      __syncthreads();
    }
  }
  double y[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    double v = 0.0;
    if (i < N) {
      const int r = perm[i];
      if (mode != MODE_APPLY) v = xin[mi.loc_off + r];
      if (with_B) {
        const int f = r / Q;
        const int b = bidx[r - f * Q];
        if (b >= 0) v += xc[f * NBD + b];
      }
    }
    y[q] = v;
  }
  // ---- forward substitution with the unit lower factor (step 2)
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jend = min(64, N - 64 * q);
    for (int jj = 0; jj < jend; ++jj) {
      const int j = 64 * q + jj;
      const double yj = readlane_d(y[q], jj);
      const T* col = A + size_t(j) * N;
      // loads are unconditional and issued in groups of kLoadGroup chunks, so a
      // column costs one or two memory latencies and the in-flight values fit
      // the register budget.  Rows past N land in the next macro's block or in
      // the workspace's guard tail; values outside the triangle are discarded
      // by the select.
#pragma unroll
      for (int g = q; g < NQ; g += kLoadGroup) {
        double a[kLoadGroup];
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
          const int r = lane + 64 * (g + t);
          // lanes outside the triangle of the first chunk, and past N in the
          // last chunk, re-read a row whose cache line is fetched anyway
          int rr = r;
          if (g + t == q) rr = r > j ? r : j + 1;
          if (g + t == NQ - 1) rr = rr < N ? rr : N - 1;
          a[t] = (g + t < NQ) ? (double)col[rr] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
          const int r = lane + 64 * (g + t);
          if (g + t < NQ) y[g + t] -= ((r > j && r < N) ? a[t] : 0.0) * yj;
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // ---- backward substitution with the upper factor
#pragma unroll
  for (int q = NQ - 1; q >= 0; --q) {
    const int jend = min(64, N - 64 * q);
    for (int jj = jend - 1; jj >= 0; --jj) {
      const int j = 64 * q + jj;
      const T* col = A + size_t(j) * N;
      const double zj = readlane_d(y[q], jj) / (double)col[j];
      if (lane == jj) y[q] = zj;
#pragma unroll
      for (int g = 0; g <= q; g += kLoadGroup) {
        double a[kLoadGroup];
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
          const int r = lane + 64 * (g + t);
          int rr = r;
          if (g + t == q) rr = r < j ? r : (j > 0 ? j - 1 : 0);
          a[t] = (g + t <= q) ? (double)col[rr] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
          const int r = lane + 64 * (g + t);
          if (g + t <= q) y[g + t] -= (r < j ? a[t] : 0.0) * zj;
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // ---- outputs
  if (mode == MODE_RECOVER || mode == MODE_LOCAL) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      if (i < N) yout[mi.loc_off + i] = y[q];
    }
  }
  if (mode != MODE_LOCAL) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      if (i < N) {
        const int f = i / Q;
        const int b = bidx[i - f * Q];
        if (b >= 0) zc[f * NBD + b] = y[q];
      }
    }
    __syncthreads();
    for (int k = 0; k < 3; ++k)
      if (mi.tr_off[k] >= 0) edge_C(mi, k, tm, Tp, zc, tau, slots + mi.slot_off[k]);
  }
}

template <typename T, int NQ>
void macro_solve_launch(int mode, const void* fac, const MacroInfo* info, int64_t n,
                               size_t lds, const int32_t* perm, const double* tmpl,
                               const Templates& Tp, double bx, double by, double tau,
                               const double* lam, const double* xin, double* yout, double* slots,
                               hipStream_t s) {
  hipLaunchKernelGGL((macro_solve_kernel<T, NQ>), dim3((unsigned)n), dim3(64), lds, s, mode,
                     (const T*)fac, info, perm, tmpl, Tp, bx, by, tau, lam, xin, yout, slots);
}

}  // namespace mhdg
