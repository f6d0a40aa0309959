// The matrix-based form of the trace operator (section 6.1's comparison of a
// globally assembled S with the matrix-free apply): S = D - sum_K C_K A_K^-1
// B_K (eq. global_problem) assembled over the interior trace unknowns from
// the folded macro operators T_K = C_K A_K^-1 B_K, stored block-sparse, and
// applied as one sparse matrix-vector product.
//
// Block (F, F') of S couples two interior faces of one macro (F = F' for the
// diagonal block, which both macros of F contribute to):
//   S_FF' = delta_FF' D_F - sum over the macros K holding F and F' of T_K[F, F'],
// with D_F = -2 tau |F| M_F (M_F the face's 1D trace mass), rows and columns in
// the faces' canonical trace order.  Each block is stored column-major
// (n_F rows, n_F' columns), so one column is contiguous across the lanes of
// the product kernel.  Beside S the left-preconditioned matrix D^-1 S is stored
// in the same layout (block (F, F') multiplied by D_F^-1 = -M_F^-1 / (2 tau
// |F|)), so that GMRES's preconditioned products are plain block-sparse
// products as well.
#include "internal.h"

namespace mhdg {

// One workgroup per block: its values from the (one or two) T_K sub-blocks
// and, on the diagonal, D_F.  T_K is column-major with leading dimension L_K.
__global__ __launch_bounds__(256) void trace_matrix_build_kernel(
    const TraceBlock* __restrict__ blk, const FaceInfo* __restrict__ faces,
    const double* __restrict__ tm, Templates Tp, double tau, const double* __restrict__ T,
    double* __restrict__ S) {
  const TraceBlock& b = blk[blockIdx.x];
  const int nF = b.nF, nC = b.nC;
  const FaceInfo& f = faces[b.row_face];
  const double* M1 = tm + Tp.lev[f.level].M1;
  double* out = S + b.voff;
  for (int x = threadIdx.x; x < nF * nC; x += blockDim.x) {
    const int j = x / nF, i = x % nF;
    double v = b.row_face == b.col_face ? -2.0 * tau * f.len * M1[size_t(i) * nF + j] : 0.0;
    for (int c = 0; c < b.ncontrib; ++c)
      v -= T[b.toff[c] + int64_t(b.c0[c] + j) * b.L[c] + (b.r0[c] + i)];
    out[x] = v;
  }
}

// The blocks of D^-1 S from those of S: one workgroup per block,
// P[i, j] = -1 / (2 tau |F|) sum_k (M_F^-1)[i, k] S[k, j], the sum in k order.
__global__ __launch_bounds__(256) void trace_matrix_precondition_kernel(
    const TraceBlock* __restrict__ blk, const FaceInfo* __restrict__ faces,
    const double* __restrict__ tm, Templates Tp, double tau, const double* __restrict__ S,
    double* __restrict__ Pm) {
  const TraceBlock& b = blk[blockIdx.x];
  const int nF = b.nF, nC = b.nC;
  const FaceInfo& f = faces[b.row_face];
  const double* Mi = tm + Tp.lev[f.level].M1inv;
  const double sc = -1.0 / (2.0 * tau * f.len);
  const double* Sb = S + b.voff;
  double* out = Pm + b.voff;
  for (int x = threadIdx.x; x < nF * nC; x += blockDim.x) {
    const int j = x / nF, i = x % nF;
    double d = 0.0;
    for (int k = 0; k < nF; ++k) d += Mi[size_t(i) * nF + k] * Sb[size_t(j) * nF + k];
    out[x] = sc * d;
  }
}

// y = S lam (or D^-1 S lam from the stored D^-1 S) for one face row per
// wavefront.  The row's blocks are stored one after another, so the row is
// one column-major n_F x K array (K = the sum of its blocks' column counts)
// whose columns k multiply the gathered trace values xs[k].  The wavefront
// splits into G groups of 64 / G lanes; group g takes the columns
// k = g mod G, lane i of a group rows i, i + 64 / G, ... (TR of them), and the
// G partial sums meet by lane exchanges, so every column is read once,
// coalesced.  U columns per group are loaded before any is used (a row of 125
// columns at n_F = 25 is read in four round trips), and the last partial
// batch is loaded the same way under a mask.  G and TR are chosen for the
// largest face of the mesh.  Faces of a masked coefficient instance write
// zeros (as the matrix-free apply does).
#ifndef MHDG_TM_COLS
#define MHDG_TM_COLS 16   // columns per lane group loaded before use (one face row per lane)
#endif
constexpr int kMaxTraceNF = (1 << kMaxLevel) * 4 + 1;
constexpr int kMaxRowCols = 5 * kMaxTraceNF;   // a face couples with at most 5 faces
template <int G, int TR>
__global__ __launch_bounds__(64) void trace_matrix_apply_kernel(
    const int32_t* __restrict__ row_ptr, const TraceBlock* __restrict__ blk,
    const FaceInfo* __restrict__ faces, const double* __restrict__ S,
    const int32_t* __restrict__ skip, const double* __restrict__ lam, double* __restrict__ out) {
  constexpr int W = 64 / G, U = TR == 1 ? MHDG_TM_COLS : (TR == 2 ? 8 : 4);
  __shared__ double xs[kMaxRowCols];
  const int fr = blockIdx.x, lane = threadIdx.x;
  // the row's (at most 5) blocks are looked up by one lane each (the table
  // holds each block's column trace offset), so the gather of the trace values
  // takes two memory round trips whatever the block count; these loads are
  // issued before the instance's mask is known
  const int b0 = row_ptr[fr], nblk = row_ptr[fr + 1] - b0;
  int my_nC = 0, my_off = 0;
  if (lane < nblk) {
    const TraceBlock& b = blk[b0 + lane];
    my_nC = b.nC;
    my_off = b.col_off;
  }
  const FaceInfo& f = faces[fr];
  const int nF = f.nF;
  if (skip && skip[f.inst]) {
    for (int i = lane; i < nF; i += 64) out[f.tr_off + i] = 0.0;
    return;
  }
  int incl = my_nC;   // inclusive prefix sum of the blocks' column counts
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  // wavefront-uniform (read from one lane into scalar registers): K, and the
  // end column and trace offset of each block
  const int K = __builtin_amdgcn_readlane(incl, nblk - 1);
  int bend[5], boff[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    bend[q] = __builtin_amdgcn_readlane(incl, q);
    boff[q] = __builtin_amdgcn_readlane(my_off, q) - (bend[q] - __builtin_amdgcn_readlane(my_nC, q));
  }
  for (int x = lane; x < K; x += 64) {
    int o = boff[0];
#pragma unroll
    for (int q = 1; q < 5; ++q)
      if (q < nblk && x >= bend[q - 1]) o = boff[q];
    xs[x] = lam[o + x];
  }
  __syncthreads();
  // the row's base is uniform across the wavefront and its blocks span far
  // less than 4 GiB, so each load takes a 32-bit byte offset from a scalar base
  // (one address register per load instead of two)
  const char* Sr = reinterpret_cast<const char*>(S + blk[b0].voff);
  const int g = lane / W, i0 = lane % W;
  double acc[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t) acc[t] = 0.0;
  for (int k = g; k < K; k += U * G) {
    double v[U][TR];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        const int i = i0 + W * t, kk = k + u * G;
        v[u][t] = (i < nF && kk < K)
                      ? *reinterpret_cast<const double*>(Sr + uint32_t(kk * nF + i) * 8u)
                      : 0.0;
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k + u * G;
      const double x = kk < K ? xs[kk] : 0.0;
#pragma unroll
      for (int t = 0; t < TR; ++t) acc[t] += v[u][t] * x;
    }
  }
  // the groups' partial sums: lane i0 of group 0 ends with the row sums
  for (int o = W; o < 64; o <<= 1)
#pragma unroll
    for (int t = 0; t < TR; ++t) acc[t] += __shfl_xor(acc[t], o, 64);
  if (g == 0)
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      const int i = i0 + W * t;
      if (i < nF) out[f.tr_off + i] = acc[t];
    }
}

hipError_t launch_trace_matrix_build(const TraceBlock* blk, int64_t n_blocks, const FaceInfo* faces,
                                     const double* tmpl, const Templates& T, double tau,
                                     const double* Tk, double* S, double* Pm, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(trace_matrix_build_kernel, dim3((unsigned)n_blocks), dim3(256), 0, s, blk,
                     faces, tmpl, T, tau, Tk, S);
  hipLaunchKernelGGL(trace_matrix_precondition_kernel, dim3((unsigned)n_blocks), dim3(256), 0, s,
                     blk, faces, tmpl, T, tau, S, Pm);
  return hipGetLastError();
}

hipError_t launch_trace_matrix_apply(const int32_t* row_ptr, const TraceBlock* blk,
                                     const FaceInfo* faces, int64_t n_faces, int max_nF,
                                     const double* S, const int32_t* skip, const double* lam,
                                     double* out, hipStream_t s) {
  if (n_faces == 0) return hipSuccess;
  const dim3 g((unsigned)n_faces), b(64);
#define MHDG_TM_APPLY(G_, TR_)                                                               \
  hipLaunchKernelGGL((trace_matrix_apply_kernel<G_, TR_>), g, b, 0, s, row_ptr, blk, faces, S, \
                     skip, lam, out)
  if (max_nF <= 16) MHDG_TM_APPLY(4, 1);
  else if (max_nF <= 32) MHDG_TM_APPLY(2, 1);
  else if (max_nF <= 64) MHDG_TM_APPLY(1, 1);
  else if (max_nF <= 128) MHDG_TM_APPLY(1, 2);
  else if (max_nF <= 192) MHDG_TM_APPLY(1, 3);
  else return hipErrorInvalidValue;
#undef MHDG_TM_APPLY
  return hipGetLastError();
}

}  // namespace mhdg
