// Per-macro solve kernel of the trace operator (steps 1-3), the local
// right-hand-side solve and the local recovery.  Included by the translation
// units that instantiate it for each register-block count NQ (split so the
// fully unrolled instances compile in parallel).
#pragma once
#include "internal.h"

namespace mhdg {

// BF16 storage of factors (8-bit mantissa): the upper half of an FP32 word,
// widened exactly on load.
struct bf16_t {
  uint16_t bits;
  bf16_t() = default;
  __host__ __device__ constexpr explicit bf16_t(int) : bits(0) {}
  __device__ __forceinline__ operator double() const {
    return (double)__uint_as_float(uint32_t(bits) << 16);
  }
};

__device__ __forceinline__ const int32_t* ints_(const double* base, int64_t off) {
  return reinterpret_cast<const int32_t*>(base + off);
}

// ------------------------------------------------------------------ per-macro solves
// Boundary entries of a macro's local vectors are kept compactly: field f
// (q_x, q_y, u), boundary position b = kP + s (edge k, position s < P along
// it), index f * 3P + b.  Only these rows of x = B lam and of C y are nonzero.
__device__ __forceinline__ double wave_sum_(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int bpos(int k, int s, int P) { return s < P ? k * P + s : ((k + 1) % 3) * P; }

__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Boundary-row couplings of local edge k.  With G[i][l] = <mu_l, phi_i>_F =
// |F| T1[s][l] (T1 couples the level-r edge space with the face's trace
// space, both in the face's canonical direction, s the canonical position of
// boundary node i) every trace coupling of the method has the form
//   scatter: x[f][b(i)] += sgn c_f sum_l G[i][l] v_l      (B v: c = (n_x, n_y, a.n - tau);
//                                                         C^T v: c = (kappa n_x, kappa n_y, tau))
//   gather:  out_l = sum_i G[i][l] (c_0 z_0 + c_1 z_1 + c_2 z_2)(i)
//                                                        (C z: c = (kappa n_x, kappa n_y, tau);
//                                                         B^T z: c = (n_x, n_y, a.n - tau))
struct EdgeCoef { double c0, c1, c2; };

__device__ __forceinline__ EdgeCoef coef_B(const MacroInfo& mi, int k, double tau) {
  const double nx = mi.nrm[2 * k], ny = mi.nrm[2 * k + 1];
  return {nx, ny, mi.bx * nx + mi.by * ny - tau};
}
__device__ __forceinline__ EdgeCoef coef_C(const MacroInfo& mi, int k, double tau) {
  return {mi.kappa * mi.nrm[2 * k], mi.kappa * mi.nrm[2 * k + 1], tau};
}

__device__ inline void edge_scatter(const MacroInfo& mi, int k, const double* tm, const Templates& Tp,
                                    const double* vF, double sgn, EdgeCoef c, double* xc) {
  const LevelTemplates& L = Tp.lev[mi.level];
  const int P = mi.P, NBD = 3 * P, fl = mi.flevel[k];
  const int nF = (1 << fl) * Tp.p + 1;
  const double* T1 = tm + L.T1[fl];
  for (int s = threadIdx.x; s <= P; s += blockDim.x) {
    const int sc = mi.orient[k] > 0 ? s : P - s;
    double g = 0.0;
    for (int l = 0; l < nF; ++l) g += T1[size_t(sc) * nF + l] * vF[l];
    g *= sgn * mi.len[k];
    const int b = bpos(k, s, P);
    xc[b] += c.c0 * g;
    xc[NBD + b] += c.c1 * g;
    xc[2 * NBD + b] += c.c2 * g;
  }
}

__device__ inline void edge_gather(const MacroInfo& mi, int k, const double* tm, const Templates& Tp,
                                   const double* zc, EdgeCoef c, double* out) {
  const LevelTemplates& L = Tp.lev[mi.level];
  const int P = mi.P, NBD = 3 * P, fl = mi.flevel[k];
  const int nF = (1 << fl) * Tp.p + 1;
  const double* T1 = tm + L.T1[fl];
  for (int l = threadIdx.x; l < nF; l += blockDim.x) {
    double v = 0.0;
    for (int sc = 0; sc <= P; ++sc) {
      const int b = bpos(k, mi.orient[k] > 0 ? sc : P - sc, P);
      v += T1[size_t(sc) * nF + l] * (c.c0 * zc[b] + c.c1 * zc[NBD + b] + c.c2 * zc[2 * NBD + b]);
    }
    out[l] = mi.len[k] * v;
  }
}

// xc += sgn * B_k lam_F (step 1)
__device__ inline void edge_B(const MacroInfo& mi, int k, const double* tm, const Templates& Tp,
                              const double* lamF, double sgn, double tau,
                              double* xc) {
  edge_scatter(mi, k, tm, Tp, lamF, sgn, coef_B(mi, k, tau), xc);
}

// out = C_k z (step 3)
__device__ inline void edge_C(const MacroInfo& mi, int k, const double* tm, const Templates& Tp,
                              const double* zc, double tau, double* out) {
  edge_gather(mi, k, tm, Tp, zc, coef_C(mi, k, tau), out);
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

template <typename T, int NQ, int W = SolveOccupancy<NQ>::waves, int LG = kLoadGroup>
__global__ __launch_bounds__(64, W) void macro_solve_kernel(int mode, const T* __restrict__ fac,
                                                         const MacroInfo* __restrict__ info,
                                                         const int32_t* __restrict__ order, int64_t base,
                                                         const int32_t* __restrict__ perm_all,
                                                         const double* __restrict__ tm, Templates Tp,
                                                         const int32_t* __restrict__ skip, double tau,
                                                         const double* __restrict__ lam,
                                                         const double* xin, double* yout,
                                                         double* __restrict__ slots) {
  // loads in flight per group: the same number of bytes for FP32 factors,
  // half of them for BF16 (a wider group does not fit the register budget)
  constexpr int kLG = sizeof(T) == 8 ? LG : 2 * LG;
  extern __shared__ double sm[];
  const MacroInfo& mi = info[order[base + blockIdx.x]];
  if (skip && skip[mi.inst]) return;   // instance already converged: no work, outputs untouched
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
        edge_B(mi, k, tm, Tp, lam + mi.tr_off[k], mode == MODE_APPLY ? 1.0 : -1.0, tau, xc);
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
      const T* col = A + size_t(j) * mi.ld;
      // loads are unconditional and issued in groups of kLoadGroup chunks, so a
      // column costs one or two memory latencies and the in-flight values fit
      // the register budget.  Rows past N land in the next macro's block or in
      // the workspace's guard tail; values outside the triangle are discarded
      // by the select.
#pragma unroll
      for (int g = q; g < NQ; g += kLG) {
        T a[kLG];
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int r = lane + 64 * (g + t);
          // lanes outside the triangle of the first chunk, and past N in the
          // last chunk, re-read a row whose cache line is fetched anyway
          int rr = r;
          if (g + t == q) rr = r > j ? r : j + 1;
          if (g + t == NQ - 1) rr = rr < N ? rr : N - 1;
          a[t] = (g + t < NQ) ? col[rr] : T(0);
        }
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int r = lane + 64 * (g + t);
          if (g + t < NQ) y[g + t] -= ((r > j && r < N) ? (double)a[t] : 0.0) * yj;
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
      const T* col = A + size_t(j) * mi.ld;
      const double zj = readlane_d(y[q], jj) / (double)col[j];
      if (lane == jj) y[q] = zj;
#pragma unroll
      for (int g = 0; g <= q; g += kLG) {
        T a[kLG];
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int r = lane + 64 * (g + t);
          int rr = r;
          if (g + t == q) rr = r < j ? r : (j > 0 ? j - 1 : 0);
          a[t] = (g + t <= q) ? col[rr] : T(0);
        }
#pragma unroll
        for (int t = 0; t < kLG; ++t) {
          const int r = lane + 64 * (g + t);
          if (g + t <= q) y[g + t] -= (r < j ? (double)a[t] : 0.0) * zj;
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

// Per-macro solve for large local sizes: a workgroup of NW wavefronts per
// macro, 64-row chunk qq owned by wavefront qq % NW (register slot qq / NW).
// Every wavefront also keeps its own copy of the current diagonal chunk (the
// 64 rows holding the entries being solved) and updates it with the same
// operations in the same order, so each solved entry is available in every
// wavefront by a lane read, without a workgroup barrier per column.  The
// chunk owner publishes the next diagonal chunk through LDS once per 64
// columns.  Each wavefront streams, per column, its own chunks below (above,
// for the backward sweep) the diagonal chunk plus the diagonal rows (read by
// all NW wavefronts, mostly from cache).
template <typename T, int NQ, int NW>
__global__ __launch_bounds__(64 * NW) void macro_solve_mw_kernel(
    int mode, const T* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, const int32_t* __restrict__ perm_all,
    const double* __restrict__ tm, Templates Tp, const int32_t* __restrict__ skip, double tau,
    const double* __restrict__ lam, const double* xin, double* yout, double* __restrict__ slots) {
  constexpr int NL = (NQ + NW - 1) / NW;   // chunks per wavefront
  extern __shared__ double sm[];
  __shared__ double dch[2][64];            // published diagonal chunk (double-buffered)
  const MacroInfo& mi = info[order[base + blockIdx.x]];
  if (skip && skip[mi.inst]) return;   // instance already converged: no work, outputs untouched
  const int N = mi.N, Q = mi.Q, P = mi.P, NBD = 3 * P;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double* xc = sm;
  double* zc = sm + 3 * NBD;
  const int32_t* bidx = ints_(tm, Tp.lev[mi.level].bnd_index);
  const T* A = fac + mi.fac_off;
  const int32_t* perm = perm_all + mi.loc_off;
  const bool with_B = mode == MODE_APPLY || mode == MODE_RECOVER;
  if (with_B) {
    for (int i = threadIdx.x; i < 3 * NBD; i += blockDim.x) xc[i] = 0.0;
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
      if (mi.tr_off[k] >= 0)
        edge_B(mi, k, tm, Tp, lam + mi.tr_off[k], mode == MODE_APPLY ? 1.0 : -1.0, tau, xc);
      __syncthreads();
    }
  }
  double y[NL];
#pragma unroll
  for (int t = 0; t < NL; ++t) {
    const int i = lane + 64 * (wv + NW * t);
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
    y[t] = v;
  }
  const int nq = (N + 63) / 64;
  // the owner of chunk q hands its current values to every wavefront
  auto publish = [&](int q) -> double {
    if (wv == q % NW) {
#pragma unroll
      for (int t = 0; t < NL; ++t)
        if (t == q / NW) dch[q & 1][lane] = y[t];
    }
    __syncthreads();
    return dch[q & 1][lane];
  };
  auto retire = [&](int q, double d) {
    if (wv == q % NW) {
#pragma unroll
      for (int t = 0; t < NL; ++t)
        if (t == q / NW) y[t] = d;
    }
  };
  // ---- forward substitution (unit lower factor)
  for (int q = 0; q < nq; ++q) {
    double d = publish(q);
    const int rd = 64 * q + lane;
    const int jend = min(64, N - 64 * q);
    for (int jj = 0; jj < jend; ++jj) {
      const int j = 64 * q + jj;
      const double yj = readlane_d(d, jj);
      const T* col = A + size_t(j) * mi.ld;
      const int rdc = rd > j ? (rd < N ? rd : N - 1) : j;   // in-bounds address for every lane
      double a[NL];
#pragma unroll
      for (int t = 0; t < NL; ++t) {
        const int qq = wv + NW * t;
        const int r = lane + 64 * qq;
        a[t] = (qq > q && qq < nq) ? (double)col[r < N ? r : N - 1] : 0.0;
      }
      const double ad = (double)col[rdc];
      d -= ((rd > j && rd < N) ? ad : 0.0) * yj;
#pragma unroll
      for (int t = 0; t < NL; ++t) {
        const int qq = wv + NW * t;
        const int r = lane + 64 * qq;
        if (qq > q && qq < nq) y[t] -= (r < N ? a[t] : 0.0) * yj;
      }
    }
    retire(q, d);
  }
  // every wavefront has read the last forward chunk before it is republished
  __syncthreads();
  // ---- backward substitution (upper factor)
  for (int q = nq - 1; q >= 0; --q) {
    double d = publish(q);
    const int rd = 64 * q + lane;
    const int jst = min(63, N - 1 - 64 * q);
    for (int jj = jst; jj >= 0; --jj) {
      const int j = 64 * q + jj;
      const T* col = A + size_t(j) * mi.ld;
      double a[NL];
#pragma unroll
      for (int t = 0; t < NL; ++t) {
        const int qq = wv + NW * t;
        a[t] = qq < q ? (double)col[lane + 64 * qq] : 0.0;
      }
      const double cd = (double)col[rd < j ? rd : j];   // lanes above the diagonal read U[j][j]
      const double zj = readlane_d(d, jj) / readlane_d(cd, jj);
      d = lane == jj ? zj : d - (rd < j ? cd : 0.0) * zj;
#pragma unroll
      for (int t = 0; t < NL; ++t) {
        const int qq = wv + NW * t;
        if (qq < q) y[t] -= a[t] * zj;
      }
    }
    retire(q, d);
  }
  // ---- outputs
  if (mode == MODE_RECOVER || mode == MODE_LOCAL) {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int i = lane + 64 * (wv + NW * t);
      if (i < N) yout[mi.loc_off + i] = y[t];
    }
  }
  if (mode != MODE_LOCAL) {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int i = lane + 64 * (wv + NW * t);
      if (i < N) {
        const int f = i / Q;
        const int b = bidx[i - f * Q];
        if (b >= 0) zc[f * NBD + b] = y[t];
      }
    }
    __syncthreads();
    for (int k = 0; k < 3; ++k)
      if (mi.tr_off[k] >= 0) edge_C(mi, k, tm, Tp, zc, tau, slots + mi.slot_off[k]);
  }
}

template <typename T, int NQ, int NW>
void macro_solve_mw_launch(int mode, const void* fac, const MacroInfo* info, const int32_t* order,
                           int64_t base, int64_t n, size_t lds, const int32_t* perm,
                           const double* tmpl, const Templates& Tp, const int32_t* skip,
                           double tau, const double* lam, const double* xin, double* yout,
                           double* slots, hipStream_t s) {
  hipLaunchKernelGGL((macro_solve_mw_kernel<T, NQ, NW>), dim3((unsigned)n), dim3(64 * NW), lds, s, mode,
                     (const T*)fac, info, order, base, perm, tmpl, Tp, skip, tau, lam, xin, yout,
                     slots);
}

// Transposed per-macro solve y = A^-T x (adjoint), one wavefront per macro.
// With P A = L U held column-major: U^T w = x uses column i of U for row i
// of the forward sweep, L^T v = w column i of L for the backward sweep (each
// a dot product over contiguous memory and one wavefront reduction), then
// z[perm[i]] = v[i].  Modes as the forward solve, with C^T in place of B on
// input and B^T in place of C on output.
template <typename T, int NQ>
__global__ __launch_bounds__(64) void macro_solve_t_kernel(
    int mode, const T* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base,
    const int32_t* __restrict__ perm_all, const double* __restrict__ tm, Templates Tp,
    const int32_t* __restrict__ skip, double tau, const double* __restrict__ mu, const double* xin, double* yout,
    double* __restrict__ slots) {
  extern __shared__ double sm[];
  const MacroInfo& mi = info[order[base + blockIdx.x]];
  if (skip && skip[mi.inst]) return;   // instance already converged: no work, outputs untouched
  const int N = mi.N, Q = mi.Q, P = mi.P, NBD = 3 * P, lane = threadIdx.x;
  double* xc = sm;
  double* zc = sm + 3 * NBD;
  const int32_t* bidx = ints_(tm, Tp.lev[mi.level].bnd_index);
  const T* A = fac + mi.fac_off;
  const int32_t* perm = perm_all + mi.loc_off;
  const bool with_Ct = mode == MODE_APPLY || mode == MODE_RECOVER;
  if (with_Ct) {
    for (int i = lane; i < 3 * NBD; i += 64) xc[i] = 0.0;
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
      if (mi.tr_off[k] >= 0)
        edge_scatter(mi, k, tm, Tp, mu + mi.tr_off[k], mode == MODE_APPLY ? 1.0 : -1.0,
                     coef_C(mi, k, tau), xc);
      __syncthreads();
    }
  }
  double y[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    double v = 0.0;
    if (i < N) {
      if (mode != MODE_APPLY) v = xin[mi.loc_off + i];
      if (with_Ct) {
        const int f = i / Q;
        const int b = bidx[i - f * Q];
        if (b >= 0) v += xc[f * NBD + b];
      }
    }
    y[q] = v;
  }
  // ---- U^T w = x
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jend = min(64, N - 64 * q);
    for (int jj = 0; jj < jend; ++jj) {
      const int i = 64 * q + jj;
      const T* col = A + size_t(i) * mi.ld;
      double part = 0.0;
#pragma unroll
      for (int t = 0; t <= q; ++t) {
        const int r = lane + 64 * t;
        const double a = (double)col[r];
        part += (r < i ? a : 0.0) * y[t];
      }
      const double tot = wave_sum_(part);
      const double wi = (readlane_d(y[q], jj) - tot) / (double)col[i];
      if (lane == jj) y[q] = wi;
    }
  }
  // ---- L^T v = w
#pragma unroll
  for (int q = NQ - 1; q >= 0; --q) {
    const int jend = min(64, N - 64 * q);
    for (int jj = jend - 1; jj >= 0; --jj) {
      const int i = 64 * q + jj;
      const T* col = A + size_t(i) * mi.ld;
      double part = 0.0;
#pragma unroll
      for (int t = q; t < NQ; ++t) {
        const int r = lane + 64 * t;
        const double a = (double)col[r];
        part += ((r > i && r < N) ? a : 0.0) * y[t];
      }
      const double tot = wave_sum_(part);
      const double vi = readlane_d(y[q], jj) - tot;
      if (lane == jj) y[q] = vi;
    }
  }
  // ---- z[perm[i]] = v[i]; outputs
  if (mode == MODE_RECOVER || mode == MODE_LOCAL) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      if (i < N) yout[mi.loc_off + perm[i]] = y[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      if (i < N) {
        const int r = perm[i];
        const int f = r / Q;
        const int b = bidx[r - f * Q];
        if (b >= 0) zc[f * NBD + b] = y[q];
      }
    }
    __syncthreads();
    for (int k = 0; k < 3; ++k)
      if (mi.tr_off[k] >= 0)
        edge_gather(mi, k, tm, Tp, zc, coef_B(mi, k, tau), slots + mi.slot_off[k]);
  }
}

template <int NQ>
void macro_solve_t_launch(int mode, const void* fac, const MacroInfo* info, const int32_t* order,
                          int64_t base, int64_t n, size_t lds, const int32_t* perm,
                          const double* tmpl, const Templates& Tp, const int32_t* skip, double tau,
                          const double* mu, const double* xin, double* yout, double* slots,
                          hipStream_t s) {
  hipLaunchKernelGGL((macro_solve_t_kernel<double, NQ>), dim3((unsigned)n), dim3(64), lds, s, mode,
                     (const double*)fac, info, order, base, perm, tmpl, Tp, skip, tau, mu, xin,
                     yout, slots);
}

template <typename T, int NQ, int W = SolveOccupancy<NQ>::waves, int LG = kLoadGroup>
void macro_solve_launch(int mode, const void* fac, const MacroInfo* info, const int32_t* order,
                        int64_t base, int64_t n, size_t lds, const int32_t* perm,
                        const double* tmpl, const Templates& Tp, const int32_t* skip, double tau,
                        const double* lam, const double* xin, double* yout, double* slots,
                        hipStream_t s) {
  hipLaunchKernelGGL((macro_solve_kernel<T, NQ, W, LG>), dim3((unsigned)n), dim3(64), lds, s, mode,
                     (const T*)fac, info, order, base, perm, tmpl, Tp, skip, tau, lam, xin, yout,
                     slots);
}

}  // namespace mhdg
