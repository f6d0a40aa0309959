// Folded (boundary-to-boundary) macro operators T_K = C_K A_K^-1 B_K.
//
// The global operator is S = D - sum_K C_K A_K^-1 B_K (eq. global_problem);
// steps 1-3 of the matrix-free method (section 3.3.2) apply the product
// C_K A_K^-1 B_K to lambda_K through the stored LU factors.  Folding stores the
// product itself, a dense L_K x L_K matrix over the macro's interior-face
// trace dofs (L_K = sum of n_F over its interior faces), so an apply reads
// L_K^2 values per macro instead of N_K^2.  T_K is built column by column with
// the same per-macro solves: with the interior faces coloured so that no macro
// has two faces of one colour, one apply of the indicator of (colour c,
// position i) leaves in every macro's contribution slots exactly one column
// of its T_K.
//
// Local numbering of a macro's trace dofs: its interior edges k = 0, 1, 2 in
// order, position i along the face (face canonical direction) within each,
// the same order as its contribution slots.
#include "internal.h"

namespace mhdg {

__device__ __forceinline__ int face_nodes(const MacroInfo& mi, int k, int p) {
  return (1 << mi.flevel[k]) * p + 1;
}

// lam = indicator of position i on every interior face of colour c
__global__ void fold_indicator_kernel(const FaceInfo* __restrict__ fi, int64_t nf,
                                      const int32_t* __restrict__ icolor, int c, int i,
                                      double* __restrict__ lam) {
  const int64_t f = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (f >= nf) return;
  const FaceInfo& F = fi[f];
  for (int l = 0; l < F.nF; ++l) lam[F.tr_off + l] = (icolor[f] == c && l == i) ? 1.0 : 0.0;
}

// Column (colour c, position i) of every T_K from the contribution slots.
// fcolor: colour of each face (by face id), -1 on the boundary.
__global__ __launch_bounds__(64) void fold_scatter_kernel(const MacroInfo* __restrict__ info,
                                                          const int64_t* __restrict__ toff,
                                                          const int32_t* __restrict__ fcolor,
                                                          int p, int c, int i,
                                                          const double* __restrict__ slots,
                                                          double* __restrict__ T) {
  const MacroInfo& mi = info[blockIdx.x];
  int L = 0, col = -1;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
    if (fcolor[mi.face[k]] == c && i < nF) col = L + i;
    L += nF;
  }
  if (col < 0) return;
  double* Tc = T + toff[blockIdx.x] + int64_t(col) * L;
  int r0 = 0;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
    for (int l = threadIdx.x; l < nF; l += 64) Tc[r0 + l] = slots[mi.slot_off[k] + l];
    r0 += nF;
  }
}

// Steps 1-3 with the folded operators: slots of macro K = T_K lambda_K, or
// T_K^T lambda_K for the transposed operator S^T (adjoint solves).  One
// wavefront per macro with lambda_K gathered into LDS.  Forward: T_K streamed
// column by column, coalesced across the lanes, lane l accumulating rows
// l + 64 t.  Transposed: lane l forms the dot product of column l + 64 t with
// lambda_K (each lane walks its own contiguous column; a macro's T_K is a
// few KB and stays in cache).
constexpr int kFoldRows = 3;   // rows per lane: L_K <= 192 (checked on the host)
__global__ __launch_bounds__(64) void fold_apply_kernel(const MacroInfo* __restrict__ info,
                                                        const int64_t* __restrict__ toff,
                                                        const double* __restrict__ T, int p,
                                                        const int32_t* __restrict__ skip,
                                                        int transpose,
                                                        const double* __restrict__ lam,
                                                        double* __restrict__ slots) {
  __shared__ double xl[64 * kFoldRows];
  const MacroInfo& mi = info[blockIdx.x];
  if (skip && skip[mi.inst]) return;
  const int lane = threadIdx.x;
  int L = 0;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
    for (int l = lane; l < nF; l += 64) xl[L + l] = lam[mi.tr_off[k] + l];
    L += nF;
  }
  if (L == 0) return;
  __syncthreads();
  const double* Tm = T + toff[blockIdx.x];
  double acc[kFoldRows];
#pragma unroll
  for (int t = 0; t < kFoldRows; ++t) acc[t] = 0.0;
  const int nt = (L + 63) >> 6;
  if (!transpose) {
#pragma unroll 4
    for (int c = 0; c < L; ++c) {
      const double x = xl[c];
      const double* col = Tm + int64_t(c) * L;
#pragma unroll
      for (int t = 0; t < kFoldRows; ++t) {
        const int r = lane + 64 * t;
        if (t < nt && r < L) acc[t] += col[r] * x;
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < kFoldRows; ++t) {
      const int c = lane + 64 * t;
      if (t < nt && c < L) {
        const double* col = Tm + int64_t(c) * L;
        double a = 0.0;
        for (int r = 0; r < L; ++r) a += col[r] * xl[r];
        acc[t] = a;
      }
    }
  }
  int r0 = 0;
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int nF = face_nodes(mi, k, p);
#pragma unroll
    for (int t = 0; t < kFoldRows; ++t) {
      const int r = lane + 64 * t;
      if (t < nt && r >= r0 && r < r0 + nF) slots[mi.slot_off[k] + (r - r0)] = acc[t];
    }
    r0 += nF;
  }
}

hipError_t launch_fold_indicator(const FaceInfo* fi, int64_t nf, const int32_t* icolor, int c,
                                 int i, double* lam, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(fold_indicator_kernel, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s,
                     fi, nf, icolor, c, i, lam);
  return hipGetLastError();
}

hipError_t launch_fold_scatter(const MacroInfo* info, int64_t n, const int64_t* toff,
                               const int32_t* fcolor, int p, int c, int i, const double* slots,
                               double* T, hipStream_t s) {
  hipLaunchKernelGGL(fold_scatter_kernel, dim3((unsigned)n), dim3(64), 0, s, info, toff, fcolor, p,
                     c, i, slots, T);
  return hipGetLastError();
}

hipError_t launch_fold_apply(const MacroInfo* info, int64_t n, const int64_t* toff, const double* T,
                             int p, const int32_t* skip, int transpose, const double* lam,
                             double* slots, hipStream_t s) {
  hipLaunchKernelGGL(fold_apply_kernel, dim3((unsigned)n), dim3(64), 0, s, info, toff, T, p, skip,
                     transpose, lam, slots);
  return hipGetLastError();
}

}  // namespace mhdg
