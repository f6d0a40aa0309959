// Steps 1-3 of the trace operator (section 3.3.2) for many trace vectors at
// once.  With one vector per launch every apply streams all stored factors
// from HBM; here a wavefront carries NR vectors through the forward and
// backward sweeps, so a factor column load serves NR products.
#include "lu_sweeps.h"

namespace mhdg {

// One wavefront per (macro, group of NR consecutive vectors).  Vector v of the
// launch reads lam + v * ld_lam and writes its contribution slots at
// slots + v * ld_slots (the slot numbering of the single-vector apply).  The
// ceil(n_rhs / NR) wavefronts of a macro are consecutive in the dispatch of one
// XCD (block b runs on XCD b mod 8), so they start together and stream the same
// factor columns through that XCD's L2.  (Workgroups of several such
// wavefronts on one CU, sharing columns through L1, were slower: their lifts
// and restrictions run one vector after the other behind workgroup barriers.)
template <int NQ, int NR>
__global__ __launch_bounds__(64) void apply_many_kernel(
    const double* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, int64_t count, int nch, int n_rhs,
    const int32_t* __restrict__ perm_all, const double* __restrict__ tm, Templates Tp,
    double tau, const double* __restrict__ lam, int64_t ld_lam, double* __restrict__ slots,
    int64_t ld_slots) {
  extern __shared__ double sm[];   // NR compact boundary vectors of 3 NBD entries
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int64_t m = int64_t(seq / nch) * 8 + xcd;
  const int chunk = seq % nch;
  if (m >= count) return;
  const MacroInfo& mi = info[order[base + m]];
  if (mi.tr_off[0] < 0 && mi.tr_off[1] < 0 && mi.tr_off[2] < 0) return;   // no slots
  const int N = mi.N, Q = mi.Q, P = mi.P, NBD = 3 * P, lane = threadIdx.x;
  const int v0 = chunk * NR;
  const int nv = min(NR, n_rhs - v0);
  // ---- step 1: x = B_K lam_K on the compact boundary rows, per vector
  for (int t = lane; t < NR * 3 * NBD; t += 64) sm[t] = 0.0;
  __syncthreads();
  for (int r = 0; r < nv; ++r) {
    const double* lv = lam + int64_t(v0 + r) * ld_lam;
    for (int k = 0; k < 3; ++k) {
      if (mi.tr_off[k] >= 0) edge_B(mi, k, tm, Tp, lv + mi.tr_off[k], 1.0, tau, sm + r * 3 * NBD);
      __syncthreads();
    }
  }
  const int32_t* bidx = ints_(tm, Tp.lev[mi.level].bnd_index);
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
  // ---- step 2: A_K^-1 x with the stored LU
  lu_sweeps_nr<NQ, NR>(y, fac + mi.fac_off, N, mi.ld, lane);
  // ---- step 3: C_K y into the contribution slots of each vector
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
  for (int r = 0; r < nv; ++r) {
    double* sv = slots + int64_t(v0 + r) * ld_slots;
    for (int k = 0; k < 3; ++k)
      if (mi.tr_off[k] >= 0) edge_C(mi, k, tm, Tp, sm + r * 3 * NBD, tau, sv + mi.slot_off[k]);
  }
}

// vectors per wavefront for local size N
static int apply_many_group(int N) {
  const int nq = (N + 63) / 64;
  return nq <= 8 ? 8 : (nq <= 16 ? 4 : (nq <= 32 ? 2 : 1));
}

hipError_t launch_apply_many(const double* fac, const MacroInfo* info, const int32_t* order,
                             const SizeClass* classes, int n_classes, const int32_t* perm,
                             const double* tmpl, const Templates& T, double tau, int n_rhs,
                             const double* lam, int64_t ld_lam, double* slots, int64_t ld_slots,
                             hipStream_t s) {
  for (int c = 0; c < n_classes; ++c) {
    const SizeClass& sc = classes[c];
    if (sc.count == 0) continue;
    const int nq = (sc.N + 63) / 64;
    const int nr = apply_many_group(sc.N);
    const int nch = (n_rhs + nr - 1) / nr;
    const int64_t nblk = (sc.count + 7) / 8 * 8 * int64_t(nch);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = size_t(nr) * 9 * sc.P * sizeof(double);
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 g((unsigned)nblk), b(64);
#define MHDG_APPLY_MANY(NQ_, NR_)                                                              \
  hipLaunchKernelGGL((apply_many_kernel<NQ_, NR_>), g, b, lds, s, fac, info, order, sc.start,  \
                     sc.count, nch, n_rhs, perm, tmpl, T, tau, lam, ld_lam, slots, ld_slots)
    if (nq <= 4) MHDG_APPLY_MANY(4, 8);
    else if (nq <= 8) MHDG_APPLY_MANY(8, 8);
    else if (nq <= 16) MHDG_APPLY_MANY(16, 4);
    else if (nq <= 32) MHDG_APPLY_MANY(32, 2);
    else if (nq <= 58) MHDG_APPLY_MANY(58, 1);
    else return hipErrorInvalidValue;
#undef MHDG_APPLY_MANY
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mhdg
