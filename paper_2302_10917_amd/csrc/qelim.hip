// Per-macro solves with the flux eliminated exactly.
//
// A_K = [[M, 0, -E^x], [0, M, -E^y], [kappa H^x, kappa H^y, K]] (section 3.3.1
// blocks, H^d = (E^d)^T inside the continuous macro space).  On an affine macro
// M = |det J| Mhat and E^d = |det J| sum_a g_ad Ehat^a (g_0d = G[d],
// g_1d = G[2 + d]), so the first two block rows give q_d = M^-1 (x_d + E^d u)
// and the third one
//   S_u u = x_u - kappa sum_a P_a w_a,   w_a = sum_d g_ad x_d,
//   S_u = K + kappa |det J| sum_ab c_ab L_ab,   c_ab = sum_d g_ad g_bd,
// with the per-level templates P_a = (Ehat^a)^T Mhat^-1 and
// L_ab = P_a Ehat^b.  Then
//   q_d = |det J|^-1 Mhat^-1 x_d + sum_a g_ad P_a^T u.
// Only the LU of S_u (Q x Q, Q = N_K / 3) is stored per macro; the templates are
// shared by every macro of a level and are read from cache.
#include "macro_solve.h"
#include "mrhs.h"

namespace mhdg {

size_t qelim_lds_bytes(int Q, int P) { return size_t(6 * Q + 9 * P) * sizeof(double); }

// Column-streaming sweeps over a Q x Q factor block (column-major, leading
// dimension ld), lane l holding rows l + 64 g in y[g].  Software-pipelined:
// the loads of column j + D are issued before column j is used, so D columns
// are in flight per wavefront.  Every column issues exactly NQ loads (chunks
// that take no part re-read one address of the same column, a cache hit), so
// the number of loads in flight is the same at every step.
template <int NQ, int D>
__device__ __forceinline__ void qsweep_forward(double (&y)[NQ], const double* __restrict__ A,
                                               int ld, int Q, int lane) {
  double a[D][NQ];
  auto load = [&](int j, double (&buf)[NQ]) {
    const int jl = j < Q ? j : Q - 1;
    const int q = jl >> 6;
    const int idle = jl + 1 < Q ? jl + 1 : Q - 1;   // below the diagonal, in range
    const double* col = A + size_t(jl) * ld;
#pragma unroll
    for (int g = 0; g < NQ; ++g) {
      const int r = lane + 64 * g;
      int rr = (g < q || (g == q && r <= jl)) ? idle : r;
      rr = rr < Q ? rr : Q - 1;
      buf[g] = __builtin_nontemporal_load(col + rr);
    }
  };
#pragma unroll
  for (int d = 0; d < D; ++d) load(d, a[d]);
  for (int j0 = 0; j0 < Q; j0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int j = j0 + d;
      if (j < Q) {
        const int q = j >> 6;
        double yq = y[0];
#pragma unroll
        for (int g = 1; g < NQ; ++g)
          if (g == q) yq = y[g];
        const double yj = readlane_d(yq, j & 63);
#pragma unroll
        for (int g = 0; g < NQ; ++g) {
          const int r = lane + 64 * g;
          if (g >= q) y[g] -= ((r > j && r < Q) ? a[d][g] : 0.0) * yj;
        }
      }
      load(j + D, a[d]);
    }
  }
}

template <int NQ, int D>
__device__ __forceinline__ void qsweep_backward(double (&y)[NQ], const double* __restrict__ A,
                                                int ld, int Q, int lane) {
  double a[D][NQ];
  // column j (counted down), with the diagonal in lane j & 63 of chunk j >> 6
  auto load = [&](int j, double (&buf)[NQ]) {
    const int jl = j >= 0 ? j : 0;
    const int q = jl >> 6;
    const double* col = A + size_t(jl) * ld;
#pragma unroll
    for (int g = 0; g < NQ; ++g) {
      const int r = lane + 64 * g;
      const int rr = (g > q || (g == q && r > jl)) ? jl : r;
      buf[g] = __builtin_nontemporal_load(col + rr);
    }
  };
#pragma unroll
  for (int d = 0; d < D; ++d) load(Q - 1 - d, a[d]);
  for (int j0 = Q - 1; j0 >= 0; j0 -= D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int j = j0 - d;
      if (j >= 0) {
        const int q = j >> 6, jj = j & 63;
        double yq = y[0], dq = a[d][0];
#pragma unroll
        for (int g = 1; g < NQ; ++g)
          if (g == q) { yq = y[g]; dq = a[d][g]; }
        const double zj = readlane_d(yq, jj) / readlane_d(dq, jj);
#pragma unroll
        for (int g = 0; g < NQ; ++g) {
          const int r = lane + 64 * g;
          if (g == q && lane == jj) y[g] = zj;
          if (g <= q) y[g] -= (r < j ? a[d][g] : 0.0) * zj;
        }
      }
      load(j - D, a[d]);
    }
  }
}

// One wavefront per macro.  Modes as for the full-block solve: APPLY
// (x = B lam, slots = C y), RHS (x = xin, slots = C y), RECOVER (x = xin - B
// lam, y to yout and slots = C y), LOCAL (x = xin, y to yout).  The right-hand
// side and u live in LDS, the Schur-block solve in registers (lane l holding
// rows l + 64 q) with the column-streaming sweeps of the full-block solve.  NQ
// may exceed ceil(Q / 64): row indices are clamped to the block and rows past
// Q take no part.  FULL: the modes that return the whole solution (RECOVER,
// LOCAL); the others are compiled without that path.
template <int NQ, bool FULL>
__global__ __launch_bounds__(64) void qelim_solve_kernel(
    int mode, const double* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, const int32_t* __restrict__ perm_all,
    const double* __restrict__ tm, Templates Tp, const double* __restrict__ qt, QTemplates QT,
    const int32_t* __restrict__ skip, double tau, const double* __restrict__ lam,
    const double* xin, double* yout, double* __restrict__ slots) {
  extern __shared__ double sm[];
  const MacroInfo& mi = info[order[base + blockIdx.x]];
  if (skip && skip[mi.inst]) return;   // instance already converged: no work, outputs untouched
  const int Q = mi.Q, P = mi.P, NBD = 3 * P, lane = threadIdx.x;
  double* xs = sm;             // 3Q: right-hand side (q_x, q_y, u rows)
  double* w0 = xs + 3 * Q;     // Q: w_0, then nothing
  double* w1 = w0 + Q;         // Q: w_1
  double* us = w1 + Q;         // Q: z, then u
  double* xc = us + Q;         // 3 NBD: compact boundary rows (B lam, then C's input)
  const LevelTemplates& LT = Tp.lev[mi.level];
  const QLevel& QL = QT.lev[mi.level];
  const int32_t* enode = ints_(tm, LT.edge_node);
  const double* Minv = qt + QL.Minv;
  const double* P0 = qt + QL.P0;
  const double* P1 = qt + QL.P1;
  const double* PT0 = qt + QL.PT0;
  const double* PT1 = qt + QL.PT1;
  const double* Mbb = qt + QL.Mbb;
  const double G0 = mi.G[0], G1 = mi.G[1], G2 = mi.G[2], G3 = mi.G[3];
  const double idJ = 1.0 / mi.dJ, kap = mi.kappa;

  // ---- right-hand side x
  for (int t = lane; t < 3 * Q; t += 64) xs[t] = mode == MODE_APPLY ? 0.0 : xin[mi.loc_off + t];
  if (mode == MODE_APPLY || mode == MODE_RECOVER) {
    for (int t = lane; t < 3 * NBD; t += 64) xc[t] = 0.0;
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
      if (mi.tr_off[k] >= 0)
        edge_B(mi, k, tm, Tp, lam + mi.tr_off[k], mode == MODE_APPLY ? 1.0 : -1.0, tau, xc);
      __syncthreads();
    }
    for (int b = lane; b < NBD; b += 64) {   // boundary position b = kP + s, s < P
      const int k = b / P;
      const int node = enode[k * (P + 1) + (b - k * P)];
      xs[node] += xc[b];
      xs[Q + node] += xc[NBD + b];
      xs[2 * Q + node] += xc[2 * NBD + b];
    }
  }
  __syncthreads();
  // ---- w_a = sum_d g_ad x_d
  for (int j = lane; j < Q; j += 64) {
    const double a = xs[j], b = xs[Q + j];
    w0[j] = G0 * a + G1 * b;
    w1[j] = G2 * a + G3 * b;
  }
  __syncthreads();
  // ---- z = x_u - kappa sum_a P_a w_a (column j of P_a is row j of PT_a); for
  // APPLY only the boundary nodes carry w
  double y[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    y[q] = i < Q ? xs[2 * Q + i] : 0.0;
  }
  const int nj = mode == MODE_APPLY ? NBD : Q;
#pragma unroll 2
  for (int jj = 0; jj < nj; ++jj) {
    int j = jj;
    if (mode == MODE_APPLY) {
      const int k = jj / P;
      j = enode[k * (P + 1) + (jj - k * P)];
    }
    const double a0 = kap * w0[j], a1 = kap * w1[j];
    const double* r0 = PT0 + size_t(j) * Q;
    const double* r1 = PT1 + size_t(j) * Q;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      const int ii = i < Q ? i : Q - 1;
      const double v = r0[ii] * a0 + r1[ii] * a1;
      if (i < Q) y[q] -= v;
    }
  }
  // ---- permuted right-hand side of the Schur-block solve
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    if (i < Q) us[i] = y[q];
  }
  __syncthreads();
  const int32_t* perm = perm_all + mi.sperm_off;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    y[q] = i < Q ? us[perm[i]] : 0.0;
  }
  __syncthreads();
  // the factor block is streamed once per apply with non-temporal loads, so that
  // it does not displace the shared templates from L2
  const double* A = fac + mi.sfac_off;
  const int ld = mi.sld;
  constexpr int kDepth = NQ <= 6 ? 4 : (NQ <= 9 ? 3 : 2);
  qsweep_forward<NQ, kDepth>(y, A, ld, Q, lane);
  qsweep_backward<NQ, kDepth>(y, A, ld, Q, lane);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    if (i < Q) us[i] = y[q];
  }
  __syncthreads();
  // ---- full solution: q_d = Minv x_d / |det J| + sum_a g_ad P_a^T u (Minv symmetric)
  if (FULL) {
    double qx[NQ], qy[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) qx[q] = qy[q] = 0.0;
#pragma unroll 2
    for (int j = 0; j < Q; ++j) {
      const double x0 = xs[j] * idJ, x1 = xs[Q + j] * idJ, uj = us[j];
      const double* m = Minv + size_t(j) * Q;
      const double* p0 = P0 + size_t(j) * Q;
      const double* p1 = P1 + size_t(j) * Q;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        const int ii = i < Q ? i : Q - 1;
        const double mv = m[ii], a = p0[ii] * uj, c = p1[ii] * uj;
        qx[q] += mv * x0 + G0 * a + G2 * c;
        qy[q] += mv * x1 + G1 * a + G3 * c;
      }
    }
    double* out = yout + mi.loc_off;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      if (i < Q) {
        out[i] = qx[q];
        out[Q + i] = qy[q];
        out[2 * Q + i] = us[i];
      }
    }
  }
  // ---- boundary rows of the solution, then C_K (step 3).  Each field value is
  // one wavefront sum of per-lane partial combinations; for APPLY x_d lives on
  // the boundary only and its Minv product uses the boundary block Mbb.
  if (mode != MODE_LOCAL) {
    for (int b = 0; b < NBD; ++b) {
      const int k = b / P;
      const int nb = enode[k * (P + 1) + (b - k * P)];
      const double* r0 = PT0 + size_t(nb) * Q;
      const double* r1 = PT1 + size_t(nb) * Q;
      double v0 = 0.0, v1 = 0.0;
      for (int j = lane; j < Q; j += 64) {
        const double uj = us[j];
        const double s0 = r0[j] * uj, s1 = r1[j] * uj;
        v0 += G0 * s0 + G2 * s1;
        v1 += G1 * s0 + G3 * s1;
      }
      if (mode == MODE_APPLY) {
        const double* mb = Mbb + size_t(b) * NBD;
        for (int b2 = lane; b2 < NBD; b2 += 64) {
          const int k2 = b2 / P;
          const int n2 = enode[k2 * (P + 1) + (b2 - k2 * P)];
          const double mv = mb[b2] * idJ;
          v0 += mv * xs[n2];
          v1 += mv * xs[Q + n2];
        }
      } else {
        const double* m = Minv + size_t(nb) * Q;
        for (int j = lane; j < Q; j += 64) {
          const double mv = m[j] * idJ;
          v0 += mv * xs[j];
          v1 += mv * xs[Q + j];
        }
      }
      v0 = wave_sum_(v0);
      v1 = wave_sum_(v1);
      if (lane == 0) {
        xc[b] = v0;
        xc[NBD + b] = v1;
        xc[2 * NBD + b] = us[nb];
      }
    }
    __syncthreads();
    for (int k = 0; k < 3; ++k)
      if (mi.tr_off[k] >= 0) edge_C(mi, k, tm, Tp, xc, tau, slots + mi.slot_off[k]);
  }
}

// Folded operators T_K = C_K A_K^-1 B_K from the Schur-block factors.  As the
// full-block build: one wavefront per (macro, NR consecutive columns of B_K);
// a column is the boundary-row lift of a unit trace value, so x_q and x_u live
// on the boundary and w_a = sum_d g_ad x_d too.  z = x_u - kappa sum_a P_a w_a
// uses the boundary columns of P_a (rows of PT_a), each row read once for the
// NR columns; the NR Schur-block solves run together in registers; the
// boundary values q_d = Mbb x_d / |det J| + sum_a g_ad P_a^T u (each lane
// summing its own boundary position over the rows of the transposed boundary
// rows of PT_a, u read from LDS) and u are restricted with C_K into NR columns
// of T_K.  The wavefronts of a macro are consecutive in one XCD's dispatch
// (block b runs on XCD b mod 8).
// BC: the boundary-condensed blocks W_K = (A_K^-1)_bb instead.  Column c of
// W_K (c < 9P, compact boundary order) is the solution for the unit vector at
// compact index c, which is a boundary vector like a lift of B_K, so the
// same steps apply; its boundary values (q_x, q_y, u at the 3P boundary
// positions) are written as column c of W_K (toff / T: W_K's offsets and
// storage) instead of being restricted with C_K.
template <int NQ, int NR, bool BC>
__global__ __launch_bounds__(64) void qelim_fold_build_kernel(
    const double* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, int64_t count, int nch,
    const int32_t* __restrict__ perm_all, const double* __restrict__ tm, Templates Tp,
    const double* __restrict__ qt, QTemplates QT, double tau, const int64_t* __restrict__ toff,
    double* __restrict__ T) {
  extern __shared__ double sm[];
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int64_t m = int64_t(seq / nch) * 8 + xcd;
  const int chunk = seq % nch;
  if (m >= count) return;
  const int e = order[base + m];
  const MacroInfo& mi = info[e];
  const int Q = mi.Q, P = mi.P, NBD = 3 * P, lane = threadIdx.x, p = Tp.p;
  int lo[3], nk[3], L = 0;
  for (int k = 0; k < 3; ++k) {
    lo[k] = L;
    nk[k] = mi.tr_off[k] >= 0 ? (1 << mi.flevel[k]) * p + 1 : 0;
    L += nk[k];
  }
  const int ncols = BC ? 3 * NBD : L;
  const int col0 = chunk * NR;
  if (col0 >= ncols) return;
  // LDS: the columns of B_K (later the boundary values of the solutions),
  // then the unpermuted right-hand sides (later the solutions)
  double* xc = sm;                    // NR x 3 NBD: columns of B_K (boundary rows)
  double* us = xc + NR * 3 * NBD;     // NR x Q: z before the permuted gather; then u
  double* zc = xc;                    // NR x 3 NBD: boundary values of the solutions
  const LevelTemplates& LT = Tp.lev[mi.level];
  const QLevel& QL = QT.lev[mi.level];
  const int32_t* enode = ints_(tm, LT.edge_node);
  const int32_t* bidx = ints_(tm, LT.bnd_index);
  const double* PT0 = qt + QL.PT0;
  const double* PT1 = qt + QL.PT1;
  const double* Mbb = qt + QL.Mbb;
  const double G0 = mi.G[0], G1 = mi.G[1], G2 = mi.G[2], G3 = mi.G[3];
  const double idJ = 1.0 / mi.dJ, kap = mi.kappa;
  for (int t = lane; t < NR * 3 * NBD; t += 64) xc[t] = 0.0;
  __syncthreads();
  if (BC) {
    if (lane < NR && col0 + lane < ncols) xc[lane * 3 * NBD + col0 + lane] = 1.0;
  } else for (int r = 0; r < NR && col0 + r < L; ++r) {
    const int col = col0 + r;
    const int k = col < lo[1] ? 0 : (col < lo[2] ? 1 : 2);
    const int i = col - lo[k], nF = nk[k];
    const double* T1 = tm + LT.T1[mi.flevel[k]];
    const EdgeCoef c = coef_B(mi, k, tau);
    double* x = xc + r * 3 * NBD;
    for (int s = lane; s <= P; s += 64) {
      const int sc = mi.orient[k] > 0 ? s : P - s;
      const double g = T1[size_t(sc) * nF + i] * mi.len[k];
      const int b = bpos(k, s, P);
      x[b] = c.c0 * g;
      x[NBD + b] = c.c1 * g;
      x[2 * NBD + b] = c.c2 * g;
    }
  }
  __syncthreads();
  // ---- z = x_u - kappa sum_a P_a w_a
  double y[NQ][NR];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    const int b = i < Q ? bidx[i] : -1;
#pragma unroll
    for (int r = 0; r < NR; ++r) y[q][r] = b >= 0 ? xc[r * 3 * NBD + 2 * NBD + b] : 0.0;
  }
  for (int b = 0; b < NBD; ++b) {
    const int k = b / P;
    const int nb = enode[k * (P + 1) + (b - k * P)];
    double a0[NR], a1[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double x0 = xc[r * 3 * NBD + b], x1 = xc[r * 3 * NBD + NBD + b];
      a0[r] = kap * (G0 * x0 + G1 * x1);
      a1[r] = kap * (G2 * x0 + G3 * x1);
    }
    const double* r0 = PT0 + size_t(nb) * Q;
    const double* r1 = PT1 + size_t(nb) * Q;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      const int ii = i < Q ? i : Q - 1;
      const double p0 = i < Q ? r0[ii] : 0.0, p1 = i < Q ? r1[ii] : 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) y[q][r] -= p0 * a0[r] + p1 * a1[r];
    }
  }
  // ---- permuted right-hand sides, Schur-block solves
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    if (i < Q)
#pragma unroll
      for (int r = 0; r < NR; ++r) us[r * Q + i] = y[q][r];
  }
  __syncthreads();
  const int32_t* perm = perm_all + mi.sperm_off;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    const int pi = i < Q ? perm[i] : 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) y[q][r] = i < Q ? us[r * Q + pi] : 0.0;
  }
  __syncthreads();
  const double* A = fac + mi.sfac_off;
  const int ld = mi.sld;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jend = min(64, Q - 64 * q);
    for (int jj = 0; jj < jend; ++jj) {
      const int j = 64 * q + jj;
      double yj[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) yj[r] = readlane_d(y[q][r], jj);
      const double* col = A + size_t(j) * ld;
#pragma unroll
      for (int g = q; g < NQ; g += kLoadGroup) {
        double a[kLoadGroup];
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
          const int rw = lane + 64 * (g + t);
          int rr = (g + t == q && rw <= j) ? j + 1 : rw;
          rr = rr < Q ? rr : Q - 1;
          a[t] = (g + t < NQ) ? col[rr] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
          const int rw = lane + 64 * (g + t);
          if (g + t < NQ) {
            const double av = (rw > j && rw < Q) ? a[t] : 0.0;
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
    const int jend = min(64, Q - 64 * q);
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
      for (int g = 0; g <= q; g += kLoadGroup) {
        double a[kLoadGroup];
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
          const int rw = lane + 64 * (g + t);
          const int rr = (g + t == q && rw >= j) ? (j > 0 ? j - 1 : 0) : rw;
          a[t] = (g + t <= q) ? col[rr] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kLoadGroup; ++t) {
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
  // ---- boundary values of the solutions: u to LDS, then each lane sums q_d
  // at its own boundary position over all rows (no cross-lane sums): one
  // lane per position, or, for the last fewer than 64 positions, T lanes per
  // row group and 64 / T groups whose partial sums meet by lane exchanges
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int j = lane + 64 * q;
    if (j < Q)
#pragma unroll
      for (int r = 0; r < NR; ++r) us[r * Q + j] = y[q][r];
  }
  __syncthreads();
  const double* PB0 = qt + QL.PB0;
  const double* PB1 = qt + QL.PB1;
  constexpr int kPass = 3;   // boundary positions up to 192 (P <= 64)
  double v0[kPass][NR], v1[kPass][NR], ub[kPass][NR];
#pragma unroll
  for (int h = 0; h < kPass; ++h) {
#pragma unroll
    for (int r = 0; r < NR; ++r) v0[h][r] = v1[h][r] = ub[h][r] = 0.0;
    const int cnt = min(64, NBD - 64 * h);
    if (cnt <= 0) continue;
    int Tl = 1;
    while (Tl < cnt) Tl <<= 1;
    const int Gn = 64 / Tl, bi = lane & (Tl - 1), g = lane / Tl;
    const int b = 64 * h + bi;
    const bool bok = bi < cnt;
    const int bb = bok ? b : 64 * h;
    double s0[NR], s1[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s0[r] = s1[r] = 0.0;
#pragma unroll 4
    for (int j = g; j < Q; j += Gn) {
      const double p0 = PB0[size_t(j) * NBD + bb], p1 = PB1[size_t(j) * NBD + bb];
      const double c0 = G0 * p0 + G2 * p1, c1 = G1 * p0 + G3 * p1;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double u = us[r * Q + j];
        s0[r] += c0 * u;
        s1[r] += c1 * u;
      }
    }
#pragma unroll 4
    for (int b2 = g; b2 < NBD; b2 += Gn) {   // Mbb x_d / |det J| (Mbb is symmetric)
      const double mv = Mbb[size_t(b2) * NBD + bb] * idJ;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        s0[r] += mv * xc[r * 3 * NBD + b2];
        s1[r] += mv * xc[r * 3 * NBD + NBD + b2];
      }
    }
    for (int o = Tl; o < 64; o <<= 1)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        s0[r] += __shfl_xor(s0[r], o, 64);
        s1[r] += __shfl_xor(s1[r], o, 64);
      }
    const int kb = bb / P;
    const int nb = enode[kb * (P + 1) + (bb - kb * P)];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      v0[h][r] = s0[r];
      v1[h][r] = s1[r];
      ub[h][r] = us[r * Q + nb];
    }
  }
  __syncthreads();   // xc is read by every lane above; zc takes its place
#pragma unroll
  for (int h = 0; h < kPass; ++h) {
    const int cnt = min(64, NBD - 64 * h);
    int Tl = 1;
    while (Tl < cnt) Tl <<= 1;
    const int bi = lane & (Tl - 1);
    if (cnt > 0 && lane < Tl && bi < cnt)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int b = 64 * h + bi;
        zc[r * 3 * NBD + b] = v0[h][r];
        zc[r * 3 * NBD + NBD + b] = v1[h][r];
        zc[r * 3 * NBD + 2 * NBD + b] = ub[h][r];
      }
  }
  __syncthreads();
  double* Tm = T + toff[e];
  if (BC) {
    for (int r = 0; r < NR && col0 + r < ncols; ++r)
      for (int t = lane; t < 3 * NBD; t += 64)
        Tm[int64_t(col0 + r) * (3 * NBD) + t] = zc[r * 3 * NBD + t];
    return;
  }
  for (int r = 0; r < NR && col0 + r < L; ++r) {
    double* Tc = Tm + int64_t(col0 + r) * L;
    for (int k = 0; k < 3; ++k)
      if (nk[k] > 0) edge_C(mi, k, tm, Tp, zc + r * 3 * NBD, tau, Tc + lo[k]);
  }
}

// The same build for large Schur blocks with 16 columns of B_K per workgroup
// of NW wavefronts, the factor read once per 16 columns: the right-hand
// sides are formed in the MFMA tile layout of mrhs.h (lane (li, lk) of
// wavefront w: column col0 + li, rows 16 (w + NW i) + lk + 4 v of the permuted
// order), z = x_u - kappa sum_a P_a w_a summed over the P + 1 boundary
// positions of the column's own edge (the only nonzero entries of its lift);
// the sweeps run on MFMA; the boundary values
//   q_d(b) = sum_j c_d(j, b) u_j + Mbb x_d / |det J|,  c_0 = G0 PB0 + G2 PB1,
//   c_1 = G1 PB0 + G3 PB1,
// are formed per wavefront as MFMA products of the PB tiles with its own
// solution tiles, summed across the wavefronts by LDS atomics; u on the
// boundary nodes comes from the wavefront that holds it.  The restriction
// with C_K then writes the 16 columns of T_K.
template <int NW, int TPW>
__global__ __launch_bounds__(64 * NW, 2) void qelim_fold_build_mfma_kernel(
    const double* __restrict__ fac, const MacroInfo* __restrict__ info,
    const int32_t* __restrict__ order, int64_t base, int64_t count, int nch,
    const int32_t* __restrict__ perm_all, const double* __restrict__ tm, Templates Tp,
    const double* __restrict__ qt, QTemplates QT, double tau, const int64_t* __restrict__ toff,
    double* __restrict__ T) {
  extern __shared__ double sm[];   // the sweeps' LDS, later the 16 boundary vectors zc
  const int xcd = blockIdx.x & 7, seq = blockIdx.x >> 3;
  const int64_t m = int64_t(seq / nch) * 8 + xcd;
  const int chunk = seq % nch;
  if (m >= count) return;
  const int e = order[base + m];
  const MacroInfo& mi = info[e];
  const int Q = mi.Q, P = mi.P, NBD = 3 * P, p = Tp.p, tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: branches around MFMAs
  int lo[3], nk[3], L = 0;
  for (int k = 0; k < 3; ++k) {
    lo[k] = L;
    nk[k] = mi.tr_off[k] >= 0 ? (1 << mi.flevel[k]) * p + 1 : 0;
    L += nk[k];
  }
  const int col0 = chunk * 16;
  if (col0 >= L) return;
  const int ncol = min(16, L - col0);
  const LevelTemplates& LT = Tp.lev[mi.level];
  const QLevel& QL = QT.lev[mi.level];
  const int32_t* enode = ints_(tm, LT.edge_node);
  const int32_t* bidx = ints_(tm, LT.bnd_index);
  const double* PT0 = qt + QL.PT0;
  const double* PT1 = qt + QL.PT1;
  const double G0 = mi.G[0], G1 = mi.G[1], G2 = mi.G[2], G3 = mi.G[3];
  const double idJ = 1.0 / mi.dJ, kap = mi.kappa;
  // this lane's column: its edge kr, trace node ir, coefficients of B_K
  const int col = col0 + min(li, ncol - 1);
  const bool live = li < ncol;
  const int kr = col < lo[1] ? 0 : (col < lo[2] ? 1 : 2);
  const int ir = col - lo[kr], nFr = nk[kr];
  const double* T1r = tm + LT.T1[mi.flevel[kr]];
  const EdgeCoef cr = coef_B(mi, kr, tau);
  const int orr = mi.orient[kr];
  const double lenr = mi.len[kr];
  // lift value of this column at position s of its edge
  auto gval = [&](int s) -> double {
    const int sc = orr > 0 ? s : P - s;
    return live ? T1r[size_t(sc) * nFr + ir] * lenr : 0.0;
  };
  // ---- permuted right-hand sides z[perm[row]] in the tile layout
  const int32_t* perm = perm_all + mi.sperm_off;
  d4 x[TPW][1];
  int rp[TPW][4];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * (wid + NW * i) + lk + 4 * v;
      const int r2 = row < Q ? perm[row] : -1;
      rp[i][v] = r2;
      double z = 0.0;
      if (r2 >= 0) {
        const int b = bidx[r2];   // x_u on the column's own edge
        int sp = -1;
        if (b >= 0) {
          if (b >= kr * P && b < kr * P + P) sp = b - kr * P;
          else if (b == ((kr + 1) % 3) * P) sp = P;
        }
        if (sp >= 0) z = cr.c2 * gval(sp);
      }
      x[i][0][v] = z;
    }
  for (int sp = 0; sp <= P; ++sp) {
    const double g = gval(sp);
    const double x0 = cr.c0 * g, x1 = cr.c1 * g;
    const double a0 = kap * (G0 * x0 + G1 * x1), a1 = kap * (G2 * x0 + G3 * x1);
    const int nb = enode[kr * (P + 1) + sp];
    const double* r0 = PT0 + size_t(nb) * Q;
    const double* r1 = PT1 + size_t(nb) * Q;
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r2 = rp[i][v];
        const int rr = r2 >= 0 ? r2 : 0;
        const double pv = r0[rr] * a0 + r1[rr] * a1;
        if (r2 >= 0) x[i][0][v] -= pv;
      }
  }
  // ---- Schur-block solves (end with a workgroup barrier)
  mrhs_sweeps<NW, TPW, 1, 2>(x, fac + mi.sfac_off, Q, mi.sld, sm, wid, lane);
  // ---- boundary values: zc[r][b] = Mbb terms, then += the PB products, and u
  double* zc = sm;   // 16 x 3 NBD
  const double* Mbb = qt + QL.Mbb;
  for (int w = tid; w < 16 * NBD; w += 64 * NW) {
    const int r = w / NBD, b = w - r * NBD;
    double s0 = 0.0, s1 = 0.0;
    if (r < ncol) {
      const int cc = col0 + r;
      const int k = cc < lo[1] ? 0 : (cc < lo[2] ? 1 : 2);
      const int i = cc - lo[k], nF = nk[k];
      const double* T1 = tm + LT.T1[mi.flevel[k]];
      const EdgeCoef c = coef_B(mi, k, tau);
      for (int sp = 0; sp <= P; ++sp) {
        const int sc = mi.orient[k] > 0 ? sp : P - sp;
        const double g = T1[size_t(sc) * nF + i] * mi.len[k];
        const double mv = Mbb[size_t(bpos(k, sp, P)) * NBD + b] * idJ;   // Mbb is symmetric
        s0 += mv * c.c0 * g;
        s1 += mv * c.c1 * g;
      }
    }
    zc[r * 3 * NBD + b] = s0;
    zc[r * 3 * NBD + NBD + b] = s1;
    zc[r * 3 * NBD + 2 * NBD + b] = 0.0;
  }
  __syncthreads();
  const double* PB0 = qt + QL.PB0;
  const double* PB1 = qt + QL.PB1;
  const int nbc = (NBD + 15) / 16;
  for (int bc = 0; bc < nbc; ++bc) {
    d4 q0 = {0.0, 0.0, 0.0, 0.0}, q1 = {0.0, 0.0, 0.0, 0.0};
    const int bA = min(16 * bc + li, NBD - 1);   // A row: boundary position
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wid + NW * i;
      if (16 * t >= Q) continue;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int j = 16 * t + 4 * s + lk;   // A column: solution row
        const int jj = min(j, Q - 1);
        const double p0 = PB0[size_t(jj) * NBD + bA], p1 = PB1[size_t(jj) * NBD + bA];
        const double c0 = j < Q ? G0 * p0 + G2 * p1 : 0.0;
        const double c1 = j < Q ? G1 * p0 + G3 * p1 : 0.0;
        q0 = Mfma<double>::run(c0, x[i][0][s], q0);
        q1 = Mfma<double>::run(c1, x[i][0][s], q1);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = 16 * bc + lk + 4 * v;
      if (b < NBD) {
        atomicAdd(&zc[li * 3 * NBD + b], q0[v]);
        atomicAdd(&zc[li * 3 * NBD + NBD + b], q1[v]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * (wid + NW * i) + lk + 4 * v;
      if (row < Q) {
        const int b = bidx[row];
        if (b >= 0) zc[li * 3 * NBD + 2 * NBD + b] = x[i][0][v];
      }
    }
  __syncthreads();
  // ---- restriction with C_K into the 16 columns of T_K
  double* Tm = T + toff[e];
  for (int k = 0; k < 3; ++k) {
    if (nk[k] == 0) continue;
    const int fl = mi.flevel[k], nF = nk[k];
    const double* T1 = tm + LT.T1[fl];
    const EdgeCoef c = coef_C(mi, k, tau);
    for (int w = tid; w < ncol * nF; w += 64 * NW) {
      const int r = w / nF, l = w - r * nF;
      const double* z = zc + r * 3 * NBD;
      double acc = 0.0;
      for (int sc = 0; sc <= P; ++sc) {
        const int b = bpos(k, mi.orient[k] > 0 ? sc : P - sc, P);
        acc += T1[size_t(sc) * nF + l] * (c.c0 * z[b] + c.c1 * z[NBD + b] + c.c2 * z[2 * NBD + b]);
      }
      Tm[int64_t(col0 + r) * L + lo[k] + l] = mi.len[k] * acc;
    }
  }
}

// T_K (bc = false, max_L the largest L_K) or W_K (bc = true) for every macro
static hipError_t qelim_build(bool bc, const double* fac, const MacroInfo* info,
                              const int32_t* order, const SizeClass* classes, int n_classes,
                              const int32_t* perm, const double* tmpl, const Templates& T,
                              const double* qtm, const QTemplates& QT, double tau, int max_L,
                              const int64_t* toff, double* out, hipStream_t s) {
  for (int c = 0; c < n_classes; ++c) {
    const SizeClass& sc = classes[c];
    if (sc.count == 0) continue;
    const int Q = sc.N / 3;
    const int nq = (Q + 63) / 64;
    if (!bc && Q > 1024 && Q <= 1280) {
      // 16 columns per workgroup of 8 wavefronts, the Schur factor read once per 16
      const int nch = (max_L + 15) / 16;
      const int64_t nblk = (sc.count + 7) / 8 * 8 * int64_t(nch);
      if (nblk > 0x7fffffff) return hipErrorInvalidValue;
      const size_t lds = size_t(std::max(mrhs_lds_doubles(8, 1), 16 * 9 * sc.P)) * sizeof(double);
      if (lds > 65536) return hipErrorInvalidValue;
      hipLaunchKernelGGL((qelim_fold_build_mfma_kernel<8, 10>), dim3((unsigned)nblk), dim3(512),
                         lds, s, fac, info, order, sc.start, sc.count, nch, perm, tmpl, T, qtm,
                         QT, tau, toff, out);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      continue;
    }
    const int nr = nq <= 4 ? 4 : (nq <= 14 ? 2 : 1);
    const int cols = bc ? 9 * sc.P : max_L;
    const int nch = (cols + nr - 1) / nr;
    const int64_t nblk = (sc.count + 7) / 8 * 8 * int64_t(nch);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = (size_t(nr) * (9 * sc.P + Q)) * sizeof(double);
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 g((unsigned)nblk), b(64);
#define MHDG_QFOLD(NQ_, NR_)                                                                   \
  if (bc)                                                                                      \
    hipLaunchKernelGGL((qelim_fold_build_kernel<NQ_, NR_, true>), g, b, lds, s, fac, info,     \
                       order, sc.start, sc.count, nch, perm, tmpl, T, qtm, QT, tau, toff, out); \
  else                                                                                         \
    hipLaunchKernelGGL((qelim_fold_build_kernel<NQ_, NR_, false>), g, b, lds, s, fac, info,    \
                       order, sc.start, sc.count, nch, perm, tmpl, T, qtm, QT, tau, toff, out)
    if (nq <= 2) { MHDG_QFOLD(2, 4); }
    else if (nq <= 4) { MHDG_QFOLD(4, 4); }
    else if (nq <= 6) { MHDG_QFOLD(6, 2); }
    else if (nq <= 9) { MHDG_QFOLD(9, 2); }
    else if (nq <= 14) { MHDG_QFOLD(14, 2); }
    else if (nq <= 20) { MHDG_QFOLD(20, 1); }
    else return hipErrorInvalidValue;
#undef MHDG_QFOLD
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_qelim_fold_build(const double* fac, const MacroInfo* info, const int32_t* order,
                                   const SizeClass* classes, int n_classes, const int32_t* perm,
                                   const double* tmpl, const Templates& T, const double* qtm,
                                   const QTemplates& QT, double tau, int max_L,
                                   const int64_t* toff, double* out, hipStream_t s) {
  return qelim_build(false, fac, info, order, classes, n_classes, perm, tmpl, T, qtm, QT, tau,
                     max_L, toff, out, s);
}

hipError_t launch_qelim_bc_build(const double* fac, const MacroInfo* info, const int32_t* order,
                                 const SizeClass* classes, int n_classes, const int32_t* perm,
                                 const double* tmpl, const Templates& T, const double* qtm,
                                 const QTemplates& QT, double tau, const int64_t* woff, double* W,
                                 hipStream_t s) {
  return qelim_build(true, fac, info, order, classes, n_classes, perm, tmpl, T, qtm, QT, tau, 0,
                     woff, W, s);
}

hipError_t launch_qelim_solve(int mode, const double* fac, const MacroInfo* info,
                              const int32_t* order, const SizeClass* classes, int n_classes,
                              const int32_t* perm, const double* tmpl, const Templates& T,
                              const double* qtm, const QTemplates& QT, const int32_t* skip,
                              double tau, const double* lam, const double* xin, double* yout,
                              double* slots, hipStream_t s) {
  for (int c = 0; c < n_classes; ++c) {
    const SizeClass& sc = classes[c];
    if (sc.count == 0) continue;
    const int Q = sc.N / 3;
    const int nq = (Q + 63) / 64;
    const size_t lds = qelim_lds_bytes(Q, sc.P);
    const dim3 g((unsigned)sc.count), b(64);
    const bool full = mode == MODE_RECOVER || mode == MODE_LOCAL;
#define MHDG_QELIM_SOLVE(NQ_)                                                                  \
  if (full)                                                                                    \
    hipLaunchKernelGGL((qelim_solve_kernel<NQ_, true>), g, b, lds, s, mode, fac, info, order,  \
                       sc.start, perm, tmpl, T, qtm, QT, skip, tau, lam, xin, yout, slots);    \
  else                                                                                         \
    hipLaunchKernelGGL((qelim_solve_kernel<NQ_, false>), g, b, lds, s, mode, fac, info, order, \
                       sc.start, perm, tmpl, T, qtm, QT, skip, tau, lam, xin, yout, slots)
    if (nq <= 2) { MHDG_QELIM_SOLVE(2); }
    else if (nq <= 4) { MHDG_QELIM_SOLVE(4); }
    else if (nq <= 6) { MHDG_QELIM_SOLVE(6); }
    else if (nq <= 9) { MHDG_QELIM_SOLVE(9); }
    else if (nq <= 14) { MHDG_QELIM_SOLVE(14); }
    else if (nq <= 20) { MHDG_QELIM_SOLVE(20); }
    else return hipErrorInvalidValue;
#undef MHDG_QELIM_SOLVE
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mhdg
