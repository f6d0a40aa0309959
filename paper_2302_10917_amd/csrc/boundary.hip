// Boundary-condensed macro operators W_K = (A_K^-1)_bb.
//
// Steps 1-3 of the matrix-free method (section 3.3.2) apply C_K A_K^-1 B_K to
// lambda_K.  B_K is a sum of face integrals against the macro's basis, so it
// is nonzero only on the rows of nodes on the macro boundary; likewise C_K
// reads only those columns.  Hence C_K A_K^-1 B_K = C_b W_K B_b with W_K the
// boundary-to-boundary block of A_K^-1 over the three fields (q_x, q_y, u),
// 3 NBD = 9P rows and columns (NBD = 3P boundary nodes).  Where the interior
// block A_ii is invertible, W_K is the inverse of the boundary Schur
// complement A_bb - A_bi A_ii^-1 A_ib: the macro's interior unknowns are
// condensed out and only its boundary system is kept.  W_K is built here from
// the stored LU of the whole A_K, which needs no interior inverse and also
// serves a macro whose A_ii is singular (a lone cubic bubble).
//
// Storage: W_K column-major, NB x NB with NB = 9P, rows and columns in the
// compact boundary order of the per-macro solves (field f, boundary position
// b = kP + s, index f * 3P + b).  The apply lifts lambda_K with B_K into that
// order, multiplies by W_K and restricts with C_K; the transposed operator
// lifts with C_K^T, multiplies by W_K^T = (A_K^-T)_bb and restricts with B_K^T.
#include "lu_sweeps.h"

namespace mhdg {

// Build: one wavefront takes NR consecutive columns c0 .. c0+NR-1 of W_K.
// Column c is the solution of A_K y = e_c for the unit vector at compact
// boundary index c; the permuted unit right-hand sides are set up in
// registers (lane l holding rows l + 64 q), swept through the stored factors
// with NR right-hand sides at once, and the boundary rows of the NR solutions
// are staged in LDS and written as NR contiguous columns of W_K.  The
// ceil(NB / NR) wavefronts of a macro are consecutive in the dispatch of one
// XCD (block b runs on XCD b mod 8) and stream the same factor columns
// through that XCD's L2.
template <int NQ, int NR>
__global__ __launch_bounds__(64) void bc_build_kernel(
    const double* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, int64_t count, int nch,
    const int32_t* __restrict__ perm_all, const double* __restrict__ tm, Templates Tp,
    const int64_t* __restrict__ woff, double* __restrict__ W) {
  extern __shared__ double sm[];   // NR columns over the NB compact boundary rows
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int64_t m = int64_t(seq / nch) * 8 + xcd;
  const int chunk = seq % nch;
  if (m >= count) return;
  const int e = order[base + m];
  const MacroInfo& mi = info[e];
  const int N = mi.N, Q = mi.Q, NBD = 3 * mi.P, NB = 3 * NBD, lane = threadIdx.x;
  const int c0 = chunk * NR;
  if (c0 >= NB) return;
  const int32_t* bidx = ints_(tm, Tp.lev[mi.level].bnd_index);
  const int32_t* perm = perm_all + mi.loc_off;
  double y[NQ][NR];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    int c = -1;
    if (i < N) {
      const int rw = perm[i];
      const int f = rw / Q;
      const int b = bidx[rw - f * Q];
      if (b >= 0) c = f * NBD + b;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) y[q][r] = c == c0 + r ? 1.0 : 0.0;
  }
  lu_sweeps_nr<NQ, NR>(y, fac + mi.fac_off, N, mi.ld, lane);
  // every compact index is the image of exactly one local row, so the NR
  // staged columns are written whole
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    if (i < N) {
      const int f = i / Q;
      const int b = bidx[i - f * Q];
      if (b >= 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) sm[r * NB + f * NBD + b] = y[q][r];
      }
    }
  }
  __syncthreads();
  double* Wm = W + woff[e];
  for (int r = 0; r < NR && c0 + r < NB; ++r)
    for (int t = lane; t < NB; t += 64) Wm[int64_t(c0 + r) * NB + t] = sm[r * NB + t];
}

hipError_t launch_bc_build(const double* fac, const MacroInfo* info, const int32_t* order,
                           const SizeClass* classes, int n_classes, const int32_t* perm,
                           const double* tmpl, const Templates& T, const int64_t* woff,
                           double* W, hipStream_t s) {
  for (int c = 0; c < n_classes; ++c) {
    const SizeClass& sc = classes[c];
    if (sc.count == 0) continue;
    const int nq = (sc.N + 63) / 64;
    const int nr = nq <= 16 ? 4 : (nq <= 32 ? 2 : 1);
    const int NB = 9 * sc.P;
    const int nch = (NB + nr - 1) / nr;
    const int64_t nblk = (sc.count + 7) / 8 * 8 * int64_t(nch);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = size_t(nr) * NB * sizeof(double);
    const dim3 g((unsigned)nblk), b(64);
#define MHDG_BC_BUILD(NQ_, NR_)                                                            \
  hipLaunchKernelGGL((bc_build_kernel<NQ_, NR_>), g, b, lds, s, fac, info, order, sc.start, \
                     sc.count, nch, perm, tmpl, T, woff, W)
    if (nq <= 4) MHDG_BC_BUILD(4, 4);
    else if (nq <= 8) MHDG_BC_BUILD(8, 4);
    else if (nq <= 16) MHDG_BC_BUILD(16, 4);
    else if (nq <= 32) MHDG_BC_BUILD(32, 2);
    else if (nq <= 58) MHDG_BC_BUILD(58, 1);
    else return hipErrorInvalidValue;
#undef MHDG_BC_BUILD
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Apply: one wavefront per macro.  Lift (step 1) into the compact boundary
// vector xc in LDS, z = W_K xc (or W_K^T xc) with lane l owning rows
// l + 64 t (t < NT, NB <= 64 NT), restrict z with C_K (or B_K^T) into the
// macro's contribution slots (step 3).  W_K is read column by column,
// coalesced across the lanes, in batches of CB columns whose loads are all
// issued before any of them is used; the transposed product sums each
// column's dot product with xc across the wavefront.
template <int NT>
__global__ __launch_bounds__(64) void bc_apply_kernel(const MacroInfo* __restrict__ info,
                                                      const int64_t* __restrict__ woff,
                                                      const double* __restrict__ W,
                                                      const double* __restrict__ tm, Templates Tp,
                                                      double tau, const int32_t* __restrict__ skip,
                                                      int transpose,
                                                      const double* __restrict__ lam,
                                                      double* __restrict__ slots) {
  constexpr int CB = NT <= 2 ? 16 : (NT <= 4 ? 8 : 4);
  __shared__ double xc[64 * NT], zc[64 * NT];
  const MacroInfo& mi = info[blockIdx.x];
  if (skip && skip[mi.inst]) return;
  if (mi.tr_off[0] < 0 && mi.tr_off[1] < 0 && mi.tr_off[2] < 0) return;
  const int lane = threadIdx.x, NB = 9 * mi.P;
  for (int i = lane; i < NB; i += 64) xc[i] = 0.0;
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] >= 0)
      edge_scatter(mi, k, tm, Tp, lam + mi.tr_off[k], 1.0,
                   transpose ? coef_C(mi, k, tau) : coef_B(mi, k, tau), xc);
    __syncthreads();   // the next edge adds into the shared corner
  }
  const double* Wm = W + woff[blockIdx.x];
  double xr[NT], acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = lane + 64 * t;
    xr[t] = r < NB ? xc[r] : 0.0;
    acc[t] = 0.0;
  }
  for (int c0 = 0; c0 < NB; c0 += CB) {
    double a[CB][NT];
#pragma unroll
    for (int cc = 0; cc < CB; ++cc)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = c0 + cc, r = lane + 64 * t;
        a[cc][t] = (c < NB && r < NB) ? Wm[int64_t(c) * NB + r] : 0.0;
      }
    if (!transpose) {
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        const double x = c0 + cc < NB ? xc[c0 + cc] : 0.0;
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
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (c == lane + 64 * t) acc[t] = v;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = lane + 64 * t;
    if (r < NB) zc[r] = acc[t];
  }
  __syncthreads();
  for (int k = 0; k < 3; ++k)
    if (mi.tr_off[k] >= 0)
      edge_gather(mi, k, tm, Tp, zc, transpose ? coef_B(mi, k, tau) : coef_C(mi, k, tau),
                  slots + mi.slot_off[k]);
}

hipError_t launch_bc_apply(const MacroInfo* info, int64_t n, const int64_t* woff, const double* W,
                           int max_P, const double* tmpl, const Templates& T, double tau,
                           const int32_t* skip, int transpose, const double* lam, double* slots,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > 0x7fffffff) return hipErrorInvalidValue;
  const int nt = (9 * max_P + 63) / 64;
  const dim3 g((unsigned)n), b(64);
#define MHDG_BC_APPLY(NT_)                                                                      \
  hipLaunchKernelGGL((bc_apply_kernel<NT_>), g, b, 0, s, info, woff, W, tmpl, T, tau, skip,     \
                     transpose, lam, slots)
  switch (nt) {
    case 1: MHDG_BC_APPLY(1); break;
    case 2: MHDG_BC_APPLY(2); break;
    case 3: MHDG_BC_APPLY(3); break;
    case 4: MHDG_BC_APPLY(4); break;
    case 5: MHDG_BC_APPLY(5); break;
    case 6: MHDG_BC_APPLY(6); break;
    case 7: MHDG_BC_APPLY(7); break;
    case 8: MHDG_BC_APPLY(8); break;
    default: return hipErrorInvalidValue;
  }
#undef MHDG_BC_APPLY
  return hipGetLastError();
}

}  // namespace mhdg
