// Folded (boundary-to-boundary) macro operators T_K = C_K A_K^-1 B_K.
//
// The global operator is S = D - sum_K C_K A_K^-1 B_K (eq. global_problem);
// steps 1-3 of the matrix-free method (section 3.3.2) apply the product
// C_K A_K^-1 B_K to lambda_K through the stored LU factors.  Folding stores the
// product itself, a dense L_K x L_K matrix over the macro's interior-face
// trace dofs (L_K = sum of n_F over its interior faces), so an apply reads
// L_K^2 values per macro instead of N_K^2.  T_K is built from the stored
// factors by triangular solves with many right-hand sides: the columns of B_K.
//
// Local numbering of a macro's trace dofs: its interior edges k = 0, 1, 2 in
// order, position i along the face (face canonical direction) within each,
// the same order as its contribution slots.  T_K is column-major.
#include "lu_sweeps.h"

namespace mhdg {

__device__ __forceinline__ int face_nodes(const MacroInfo& mi, int k, int p) {
  return (1 << mi.flevel[k]) * p + 1;
}

// Build of T_K.  One wavefront takes NR consecutive columns col0 .. col0+NR-1
// of B_K (column col = trace position i of interior edge k: the boundary-row
// lift of a unit trace value, one column of the edge template), runs the
// forward and backward sweeps with the NR right-hand sides in registers
// (lane l holding rows l + 64 q, as in the single-right-hand-side solve; each
// factor column is loaded once and used NR times), and restricts the NR
// solutions with C_K into NR columns of T_K.  The ceil(L_K / NR) wavefronts of
// a macro are consecutive in the dispatch of one XCD (block b runs on XCD
// b mod 8), so they start together and stream the same factor columns
// through that XCD's L2.  NQ may exceed ceil(N_K / 64): every row index is
// clamped to the macro's column and rows past N_K take no part.
template <int NQ, int NR>
__global__ __launch_bounds__(64) void fold_build_kernel(
    const double* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, int64_t count, int nch,
    const int32_t* __restrict__ perm_all, const double* __restrict__ tm, Templates Tp,
    double tau, const int64_t* __restrict__ toff, double* __restrict__ T) {
  extern __shared__ double sm[];   // NR compact boundary vectors of 3 NBD entries
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int64_t m = int64_t(seq / nch) * 8 + xcd;
  const int chunk = seq % nch;
  if (m >= count) return;
  const int e = order[base + m];
  const MacroInfo& mi = info[e];
  const int N = mi.N, Q = mi.Q, P = mi.P, NBD = 3 * P, lane = threadIdx.x, p = Tp.p;
  int lo[3], nk[3], L = 0;
  for (int k = 0; k < 3; ++k) {
    lo[k] = L;
    nk[k] = mi.tr_off[k] >= 0 ? face_nodes(mi, k, p) : 0;
    L += nk[k];
  }
  const int col0 = chunk * NR;
  if (col0 >= L) return;
  const LevelTemplates& LT = Tp.lev[mi.level];
  // ---- columns of B_K on the compact boundary rows (step 1 for a unit trace value)
  for (int t = lane; t < NR * 3 * NBD; t += 64) sm[t] = 0.0;
  __syncthreads();
  for (int r = 0; r < NR && col0 + r < L; ++r) {
    const int col = col0 + r;
    const int k = col < lo[1] ? 0 : (col < lo[2] ? 1 : 2);
    const int i = col - lo[k], nF = nk[k];
    const double* T1 = tm + LT.T1[mi.flevel[k]];
    const EdgeCoef c = coef_B(mi, k, tau);
    double* xc = sm + r * 3 * NBD;
    for (int s = lane; s <= P; s += 64) {
      const int sc = mi.orient[k] > 0 ? s : P - s;
      const double g = T1[size_t(sc) * nF + i] * mi.len[k];
      const int b = bpos(k, s, P);
      xc[b] = c.c0 * g;
      xc[NBD + b] = c.c1 * g;
      xc[2 * NBD + b] = c.c2 * g;
    }
  }
  __syncthreads();
  const int32_t* bidx = ints_(tm, LT.bnd_index);
  const int32_t* perm = perm_all + mi.loc_off;
  double y[NQ][NR];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    int b = -1, f = 0;
    if (i < N) {
      const int rw = perm[i];
      f = rw / Q;
      b = bidx[rw - f * Q];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) y[q][r] = b >= 0 ? sm[r * 3 * NBD + f * NBD + b] : 0.0;
  }
  lu_sweeps_nr<NQ, NR>(y, fac + mi.fac_off, N, mi.ld, lane);
  // ---- restriction with C_K (step 3): boundary rows of the solutions, then
  // per interior edge the trace moments, into columns col0 .. of T_K
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    if (i < N) {
      const int f = i / Q;
      const int b = bidx[i - f * Q];
      if (b >= 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) sm[r * 3 * NBD + f * NBD + b] = y[q][r];
      }
    }
  }
  __syncthreads();
  double* Tm = T + toff[e];
  for (int r = 0; r < NR && col0 + r < L; ++r) {
    const double* zc = sm + r * 3 * NBD;
    double* Tc = Tm + int64_t(col0 + r) * L;
    for (int k = 0; k < 3; ++k)
      if (nk[k] > 0) edge_C(mi, k, tm, Tp, zc, tau, Tc + lo[k]);
  }
}

hipError_t launch_fold_build(const double* fac, const MacroInfo* info, const int32_t* order,
                             const SizeClass* classes, int n_classes, const int32_t* perm,
                             const double* tmpl, const Templates& T, double tau, int max_L,
                             const int64_t* toff, double* out, hipStream_t s) {
  for (int c = 0; c < n_classes; ++c) {
    const SizeClass& sc = classes[c];
    if (sc.count == 0) continue;
    const int nq = (sc.N + 63) / 64;
    const int nr = nq <= 16 ? 4 : (nq <= 32 ? 2 : 1);
    const int nch = (max_L + nr - 1) / nr;
    const int64_t nblk = (sc.count + 7) / 8 * 8 * int64_t(nch);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = size_t(nr) * 9 * sc.P * sizeof(double);
    const dim3 g((unsigned)nblk), b(64);
#define MHDG_FOLD_BUILD(NQ_, NR_)                                                              \
  hipLaunchKernelGGL((fold_build_kernel<NQ_, NR_>), g, b, lds, s, fac, info, order, sc.start,  \
                     sc.count, nch, perm, tmpl, T, tau, toff, out)
    if (nq <= 4) MHDG_FOLD_BUILD(4, 4);
    else if (nq <= 8) MHDG_FOLD_BUILD(8, 4);
    else if (nq <= 16) MHDG_FOLD_BUILD(16, 4);
    else if (nq <= 32) MHDG_FOLD_BUILD(32, 2);
    else if (nq <= 58) MHDG_FOLD_BUILD(58, 1);
    else return hipErrorInvalidValue;
#undef MHDG_FOLD_BUILD
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Steps 1-3 with the folded operators: slots of macro K = T_K lambda_K, or
// T_K^T lambda_K for the transposed operator S^T (adjoint solves).  One
// workgroup of NW wavefronts per macro with lambda_K gathered into LDS; lane
// l owns rows l + 64 t (t < NT, L_K <= 64 NT).  Wavefront w takes the w-th of
// NW consecutive column ranges of T_K and reads it column by column,
// coalesced across the lanes, in batches of CB columns whose loads are all
// issued before any of them is used, so a macro's T_K is read in about
// ceil(L_K / (NW CB)) memory round trips.  Forward: row r accumulates
// T[r][c] lambda_c, and the wavefronts' partial sums meet in LDS.
// Transposed: column c's dot product with lambda is summed across the
// wavefront that holds the column and stored for row c.
template <int NT, int NW>
__global__ __launch_bounds__(64 * NW) void fold_apply_kernel(const MacroInfo* __restrict__ info,
                                                             const int64_t* __restrict__ toff,
                                                             const double* __restrict__ T, int p,
                                                             const int32_t* __restrict__ skip,
                                                             int transpose,
                                                             const double* __restrict__ lam,
                                                             double* __restrict__ slots) {
  constexpr int CB = NT == 3 ? 8 : 16;
  __shared__ double xl[64 * NT];
  __shared__ double red[NW][64 * NT];
  const MacroInfo& mi = info[blockIdx.x];
  if (skip && skip[mi.inst]) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int L = 0;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
    for (int l = tid; l < nF; l += 64 * NW) xl[L + l] = lam[mi.tr_off[k] + l];
    L += nF;
  }
  if (L == 0) return;
  __syncthreads();
  const double* Tm = T + toff[blockIdx.x];
  const int span = (L + NW - 1) / NW;
  const int cbeg = wid * span, cend = min(L, cbeg + span);
  double xr[NT], acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = lane + 64 * t;
    xr[t] = r < L ? xl[r] : 0.0;
    acc[t] = 0.0;
  }
  for (int c0 = cbeg; c0 < cend; c0 += CB) {
    double a[CB][NT];
#pragma unroll
    for (int cc = 0; cc < CB; ++cc)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = c0 + cc, r = lane + 64 * t;
        a[cc][t] = (c < cend && r < L) ? Tm[int64_t(c) * L + r] : 0.0;
      }
    if (!transpose) {
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        const double x = c0 + cc < cend ? xl[c0 + cc] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] += a[cc][t] * x;
      }
    } else {
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) v += a[cc][t] * xr[t];
        v = wave_sum_(v);
        const int c = c0 + cc;
        if (lane == 0 && c < cend) red[0][c] = v;   // row c of T_K^T lambda
      }
    }
  }
  if (!transpose) {
#pragma unroll
    for (int t = 0; t < NT; ++t) red[wid][lane + 64 * t] = acc[t];
  }
  __syncthreads();
  int r0 = 0;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
    for (int l = tid; l < nF; l += 64 * NW) {
      double v = red[0][r0 + l];
      if (!transpose)
#pragma unroll
        for (int w = 1; w < NW; ++w) v += red[w][r0 + l];
      slots[mi.slot_off[k] + l] = v;
    }
    r0 += nF;
  }
}

// Folded steps 1-3 for n_rhs trace vectors: workgroup (macro, group of NR
// consecutive vectors) reads T_K once for the NR vectors of its group, in the
// same column batches as the single-vector kernel.  Vector v reads
// lam + v * ld_lam and writes its slots at slots + v * ld_slots.
template <int NT, int NR>
__global__ __launch_bounds__(64) void fold_apply_many_kernel(const MacroInfo* __restrict__ info,
                                                             const int64_t* __restrict__ toff,
                                                             const double* __restrict__ T, int p,
                                                             int n_rhs,
                                                             const double* __restrict__ lam,
                                                             int64_t ld_lam,
                                                             double* __restrict__ slots,
                                                             int64_t ld_slots) {
  constexpr int CB = 8;
  __shared__ double xl[NR][64 * NT];
  const MacroInfo& mi = info[blockIdx.x];
  const int lane = threadIdx.x;
  const int v0 = blockIdx.y * NR, nv = min(NR, n_rhs - v0);
  int L = 0;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
    for (int r = 0; r < NR; ++r)
      for (int l = lane; l < nF; l += 64)
        xl[r][L + l] = r < nv ? lam[int64_t(v0 + r) * ld_lam + mi.tr_off[k] + l] : 0.0;
    L += nF;
  }
  if (L == 0) return;
  __syncthreads();
  const double* Tm = T + toff[blockIdx.x];
  double acc[NT][NR];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[t][r] = 0.0;
  for (int c0 = 0; c0 < L; c0 += CB) {
    double a[CB][NT];
#pragma unroll
    for (int cc = 0; cc < CB; ++cc)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = c0 + cc, rw = lane + 64 * t;
        a[cc][t] = (c < L && rw < L) ? Tm[int64_t(c) * L + rw] : 0.0;
      }
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) {
      const int c = min(c0 + cc, 64 * NT - 1);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double x = c0 + cc < L ? xl[r][c] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t][r] += a[cc][t] * x;
      }
    }
  }
  int r0 = 0;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int rw = lane + 64 * t;
      if (rw >= r0 && rw < r0 + nF)
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nv) slots[int64_t(v0 + r) * ld_slots + mi.slot_off[k] + (rw - r0)] = acc[t][r];
    }
    r0 += nF;
  }
}

hipError_t launch_fold_apply_many(const MacroInfo* info, int64_t n, const int64_t* toff,
                                  const double* T, int p, int max_L, int n_rhs, const double* lam,
                                  int64_t ld_lam, double* slots, int64_t ld_slots, hipStream_t s) {
  constexpr int NR = 8;
  const dim3 g((unsigned)n, (unsigned)((n_rhs + NR - 1) / NR)), b(64);
  if (max_L <= 64)
    hipLaunchKernelGGL((fold_apply_many_kernel<1, NR>), g, b, 0, s, info, toff, T, p, n_rhs, lam,
                       ld_lam, slots, ld_slots);
  else if (max_L <= 128)
    hipLaunchKernelGGL((fold_apply_many_kernel<2, NR>), g, b, 0, s, info, toff, T, p, n_rhs, lam,
                       ld_lam, slots, ld_slots);
  else if (max_L <= kFoldMaxL)
    hipLaunchKernelGGL((fold_apply_many_kernel<3, NR>), g, b, 0, s, info, toff, T, p, n_rhs, lam,
                       ld_lam, slots, ld_slots);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fold_apply(const MacroInfo* info, int64_t n, const int64_t* toff, const double* T,
                             int p, int max_L, const int32_t* skip, int transpose,
                             const double* lam, double* slots, hipStream_t s) {
#ifndef MHDG_FOLD_APPLY_WAVES
#define MHDG_FOLD_APPLY_WAVES 2
#endif
  constexpr int NW = MHDG_FOLD_APPLY_WAVES;
  const dim3 g((unsigned)n), b(64 * NW);
  if (max_L <= 64)
    hipLaunchKernelGGL((fold_apply_kernel<1, NW>), g, b, 0, s, info, toff, T, p, skip, transpose, lam, slots);
  else if (max_L <= 128)
    hipLaunchKernelGGL((fold_apply_kernel<2, NW>), g, b, 0, s, info, toff, T, p, skip, transpose, lam, slots);
  else if (max_L <= kFoldMaxL)
    hipLaunchKernelGGL((fold_apply_kernel<3, NW>), g, b, 0, s, info, toff, T, p, skip, transpose, lam, slots);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mhdg
