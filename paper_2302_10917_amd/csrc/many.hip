// Steps 1-3 of the trace operator (section 3.3.2) for many trace vectors at
// once.  With one vector per launch every apply streams all stored factors
// from HBM; here a wavefront carries NR vectors through the forward and
// backward sweeps, so a factor column load serves NR products.
#include "lu_sweeps.h"
#include "mrhs.h"

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

// The same product with the sweeps on MFMA (mrhs.h): one workgroup of NW
// wavefronts per (macro, group of 16 NH consecutive vectors), the factor read
// once per group.  Step 1 lifts all vectors of the group at once (work items
// (vector, boundary position) per edge), step 3 restricts them at once (work
// items (vector, trace node) per edge).
template <int NW, int TPW, int NH>
__global__ __launch_bounds__(64 * NW, 2) void apply_many_mfma_kernel(
    const double* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, int64_t count, int nch, int n_rhs,
    const int32_t* __restrict__ perm_all, const double* __restrict__ tm, Templates Tp,
    double tau, const double* __restrict__ lam, int64_t ld_lam, double* __restrict__ slots,
    int64_t ld_slots) {
  constexpr int NR = 16 * NH, NT = 64 * NW;
  extern __shared__ double sm[];
  double* vec = sm + mrhs_lds_doubles(NW, NH);   // NR compact boundary vectors of 3 NBD entries
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int64_t m = int64_t(seq / nch) * 8 + xcd;
  const int chunk = seq % nch;
  if (m >= count) return;
  const MacroInfo& mi = info[order[base + m]];
  if (mi.tr_off[0] < 0 && mi.tr_off[1] < 0 && mi.tr_off[2] < 0) return;   // no slots
  const int N = mi.N, Q = mi.Q, P = mi.P, NBD = 3 * P, tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int v0 = chunk * NR;
  const int nv = min(NR, n_rhs - v0);
  const LevelTemplates& LT = Tp.lev[mi.level];
  // ---- step 1: x = B_K lam_K on the compact boundary rows of every vector
  for (int t = tid; t < NR * 3 * NBD; t += NT) vec[t] = 0.0;
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] >= 0) {
      const int fl = mi.flevel[k], nF = (1 << fl) * Tp.p + 1;
      const double* T1 = tm + LT.T1[fl];
      const EdgeCoef c = coef_B(mi, k, tau);
      for (int w = tid; w < nv * (P + 1); w += NT) {
        const int r = w / (P + 1), s = w - r * (P + 1);
        const int sc = mi.orient[k] > 0 ? s : P - s;
        const double* lv = lam + int64_t(v0 + r) * ld_lam + mi.tr_off[k];
        double g = 0.0;
        for (int l = 0; l < nF; ++l) g += T1[size_t(sc) * nF + l] * lv[l];
        g *= mi.len[k];
        double* xc = vec + r * 3 * NBD;
        const int b = bpos(k, s, P);
        xc[b] += c.c0 * g;
        xc[NBD + b] += c.c1 * g;
        xc[2 * NBD + b] += c.c2 * g;
      }
    }
    __syncthreads();   // the next edge adds into the shared corner
  }
  // ---- the permuted right-hand sides into this wavefront's tiles
  const int32_t* bidx = ints_(tm, LT.bnd_index);
  const int32_t* perm = perm_all + mi.loc_off;
  d4 x[TPW][NH];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * (wid + NW * i) + lk + 4 * v;
      int cidx = -1;
      if (row < N) {
        const int rw = perm[row];
        const int f = rw / Q;
        const int b = bidx[rw - f * Q];
        if (b >= 0) cidx = f * NBD + b;
      }
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int j = 16 * h + li;
        x[i][h][v] = (cidx >= 0 && j < nv) ? vec[j * 3 * NBD + cidx] : 0.0;
      }
    }
  // ---- step 2: A_K^-1 x (ends with a workgroup barrier)
  mrhs_sweeps<NW, TPW, NH>(x, fac + mi.fac_off, N, mi.ld, sm, wid, lane);
  // ---- step 3: boundary rows of the solutions, then C_K into the slots
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * (wid + NW * i) + lk + 4 * v;
      if (row < N) {
        const int f = row / Q;
        const int b = bidx[row - f * Q];
        if (b >= 0) {
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            const int j = 16 * h + li;
            if (j < nv) vec[j * 3 * NBD + f * NBD + b] = x[i][h][v];
          }
        }
      }
    }
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    if (mi.tr_off[k] < 0) continue;
    const int fl = mi.flevel[k], nF = (1 << fl) * Tp.p + 1;
    const double* T1 = tm + LT.T1[fl];
    const EdgeCoef c = coef_C(mi, k, tau);
    for (int w = tid; w < nv * nF; w += NT) {
      const int r = w / nF, l = w - r * nF;
      const double* zc = vec + r * 3 * NBD;
      double acc = 0.0;
      for (int sc = 0; sc <= P; ++sc) {
        const int b = bpos(k, mi.orient[k] > 0 ? sc : P - sc, P);
        acc += T1[size_t(sc) * nF + l] * (c.c0 * zc[b] + c.c1 * zc[NBD + b] + c.c2 * zc[2 * NBD + b]);
      }
      slots[int64_t(v0 + r) * ld_slots + mi.slot_off[k] + l] = mi.len[k] * acc;
    }
  }
}

// vectors per wavefront for local size N
static int apply_many_group(int N) {
  const int nq = (N + 63) / 64;
  return nq <= 8 ? 8 : (nq <= 16 ? 4 : (nq <= 32 ? 2 : 1));
}

// The MFMA sweeps for groups of 16 vectors on macros of up to 1024 unknowns
// (8 tiles of 16 rows per wavefront at most), from 12 vectors per call: below
// that the per-wavefront sweeps (up to 4 or 8 vectors per factor pass) are as
// fast, since the workgroup sweeps are bound by one barrier per 16-column
// block (at 8192 macros with N_K = 975: 23.8 ms per group of 16 against
// 36 ms for four groups of 4).
static bool use_mfma_sweeps(int N, int n_rhs) { return n_rhs >= 12 && N <= 1024; }

hipError_t launch_apply_many(const double* fac, const MacroInfo* info, const int32_t* order,
                             const SizeClass* classes, int n_classes, const int32_t* perm,
                             const double* tmpl, const Templates& T, double tau, int n_rhs,
                             const double* lam, int64_t ld_lam, double* slots, int64_t ld_slots,
                             hipStream_t s) {
  for (int c = 0; c < n_classes; ++c) {
    const SizeClass& sc = classes[c];
    if (sc.count == 0) continue;
    if (use_mfma_sweeps(sc.N, n_rhs)) {
      // 16 vectors per workgroup, the factor read once per group
      const int ntile = (sc.N + 15) / 16;
      const int nw = ntile <= 16 ? 2 : (ntile <= 32 ? 4 : 8);
      const int nch = (n_rhs + 15) / 16;
      const int64_t nblk = (sc.count + 7) / 8 * 8 * int64_t(nch);
      if (nblk > 0x7fffffff) return hipErrorInvalidValue;
      const size_t lds = (size_t(mrhs_lds_doubles(nw, 1)) + size_t(16) * 9 * sc.P) * sizeof(double);
      const dim3 g((unsigned)nblk), b(64 * nw);
#define MHDG_APPLY_MANY_MFMA(NW_)                                                               \
  hipLaunchKernelGGL((apply_many_mfma_kernel<NW_, 8, 1>), g, b, lds, s, fac, info, order,       \
                     sc.start, sc.count, nch, n_rhs, perm, tmpl, T, tau, lam, ld_lam, slots,    \
                     ld_slots)
      if (nw == 2) MHDG_APPLY_MANY_MFMA(2);
      else if (nw == 4) MHDG_APPLY_MANY_MFMA(4);
      else MHDG_APPLY_MANY_MFMA(8);
#undef MHDG_APPLY_MANY_MFMA
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      continue;
    }
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
