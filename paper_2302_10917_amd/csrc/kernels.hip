// HIP kernels (gfx950) of the macro-element HDG local-problem path.
//
//   assemble      A_K from the exact reference templates, scaled by the macro's
//                 affine map, kappa_K, a and tau (forms of paper section 3.2)
//   lu            in-place LU with partial row pivoting, one workgroup per macro;
//                 register-resident pivoted panels, MFMA trailing updates
//                 (the in-place factorisation of the remark in section 3.3.2)
//   macro_solve   steps 1-3 of the matrix-free algorithm for one macro per
//                 wavefront: gather lambda_K, x = B_K lambda_K, y = A_K^-1 x,
//                 v^ = C_K y into a per-(macro, edge) slot; also the local
//                 right-hand side solve and the local recovery (eq. local_problem)
//   face_combine  step 4 per interior face: D_F lambda - v^_1 - v^_2, or with
//                 the D^-1 preconditioner lambda - D_F^-1 (v^_1 + v^_2)
//   dirichlet     L2 projection of g_D onto the boundary trace spaces
//   vector ops    deterministic two-pass dot products and Krylov updates
#include "internal.h"
#include "macro_solve.h"
#include "mfma.h"

namespace mhdg {


__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ const int32_t* ints(const double* base, int64_t off) {
  return reinterpret_cast<const int32_t*>(base + off);
}

// ------------------------------------------------------------------ assembly
// SUPG parameter of section 3.4 for a macro's sub-triangles (all congruent,
// diameter h): Pe = |a| h / (2 kappa), tau = h / (2|a|) (coth Pe - 1/Pe), with
// the series Pe/3 - Pe^3/45 + 2 Pe^5/945 of the bracket for small Pe; zero when
// the forms are not stabilised or there is no advection.
__device__ __forceinline__ double supg_tau(const MacroInfo& mi) {
  const double h = mi.hsupg, an = sqrt(mi.bx * mi.bx + mi.by * mi.by);
  if (!(h > 0.0) || an == 0.0) return 0.0;
  const double pe = an * h / (2.0 * mi.kappa);
  const double xi = pe < 1e-2 ? pe * (1.0 / 3.0 - pe * pe * (1.0 / 45.0 - pe * pe * (2.0 / 945.0)))
                              : 1.0 / tanh(pe) - 1.0 / pe;
  return h / (2.0 * an) * xi;
}

struct EntryCtx {
  const double* Mh;
  const double* E0;
  const double* E1;
  const double* M1;
  const int32_t* epos;
  const double* Sp;   // SUPG templates (null when not stabilised)
  double G[4], dJ, len[3], kappa, bx, by, tau;
  // SUPG: tau_supg, a.grad = al0 d_xi + al1 d_eta, lap = sum g_bc d_b d_c
  double ts, al0, al1, g00, g01, g11;
  int Q, P;
};

__device__ __forceinline__ EntryCtx make_ctx(const MacroInfo& mi, const double* tm,
                                             const Templates& T, double tau) {
  EntryCtx c;
  const LevelTemplates& L = T.lev[mi.level];
  c.Mh = tm + L.Mhat;
  c.E0 = tm + L.E0;
  c.E1 = tm + L.E1;
  c.M1 = tm + L.M1;
  c.epos = ints(tm, L.node_epos);
  for (int k = 0; k < 4; ++k) c.G[k] = mi.G[k];
  c.dJ = mi.dJ;
  for (int k = 0; k < 3; ++k) c.len[k] = mi.len[k];
  c.kappa = mi.kappa;
  c.bx = mi.bx;
  c.by = mi.by;
  c.tau = tau;
  c.Q = mi.Q;
  c.P = mi.P;
  c.ts = supg_tau(mi);
  c.Sp = c.ts != 0.0 ? tm + L.supg : nullptr;
  c.al0 = mi.G[0] * mi.bx + mi.G[1] * mi.by;
  c.al1 = mi.G[2] * mi.bx + mi.G[3] * mi.by;
  c.g00 = mi.G[0] * mi.G[0] + mi.G[1] * mi.G[1];
  c.g01 = mi.G[0] * mi.G[2] + mi.G[1] * mi.G[3];
  c.g11 = mi.G[2] * mi.G[2] + mi.G[3] * mi.G[3];
  return c;
}

// SUPG block entry tau sum_e (a.grad phi_i, a.grad phi_j - kappa lap phi_j)_e
// = tau |det J| (sum_kl al_k al_l S_kl - kappa sum_k al_k sum_c g_c T_kc)_ij
__device__ __forceinline__ double supg_entry(const EntryCtx& c, int i, int j) {
  const size_t QQ = size_t(c.Q) * c.Q, o = size_t(i) * c.Q + j;
  const double* S = c.Sp;
  const double s = c.al0 * c.al0 * S[o] + c.al1 * c.al1 * S[QQ + o] + c.al0 * c.al1 * S[2 * QQ + o];
  const double t0 = c.g00 * S[3 * QQ + o] + 2.0 * c.g01 * S[4 * QQ + o] + c.g11 * S[5 * QQ + o];
  const double t1 = c.g00 * S[6 * QQ + o] + 2.0 * c.g01 * S[7 * QQ + o] + c.g11 * S[8 * QQ + o];
  return c.ts * c.dJ * (s - c.kappa * (c.al0 * t0 + c.al1 * t1));
}

// E^d_ij = (phi_j, d_d phi_i)_K = |det J| sum_k G[k][d] Ehat^k_ij
__device__ __forceinline__ double Ed(const EntryCtx& c, int d, int i, int j) {
  const size_t o = size_t(i) * c.Q + j;
  return c.dJ * (c.G[d] * c.E0[o] + c.G[2 + d] * c.E1[o]);
}

// boundary mass <phi_j, phi_i>_dK from the 1D trace mass on each edge
__device__ __forceinline__ double Mb(const EntryCtx& c, int i, int j) {
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int si = c.epos[3 * i + k], sj = c.epos[3 * j + k];
    if (si >= 0 && sj >= 0) v += c.len[k] * c.M1[size_t(si) * (c.P + 1) + sj];
  }
  return v;
}

// Entry (r, c) of A_K = [[M, 0, -E^x], [0, M, -E^y], [kappa H^x, kappa H^y, K]]
// with H^d = (E^d)^T (integration by parts inside the continuous macro space)
// and K = -(a_x E^x + a_y E^y) + tau Mb (+ the SUPG block when stabilised).
__device__ double a_entry(const EntryCtx& c, int r, int col) {
  const int Q = c.Q;
  const int rb = r / Q, i = r - rb * Q, cb = col / Q, j = col - cb * Q;
  switch (rb * 3 + cb) {
    case 0: case 4: return c.dJ * c.Mh[size_t(i) * Q + j];
    case 1: case 3: return 0.0;
    case 2: return -Ed(c, 0, i, j);
    case 5: return -Ed(c, 1, i, j);
    case 6: return c.kappa * Ed(c, 0, j, i);
    case 7: return c.kappa * Ed(c, 1, j, i);
    default:
      return -(c.bx * Ed(c, 0, i, j) + c.by * Ed(c, 1, i, j)) + c.tau * Mb(c, i, j) +
             (c.Sp ? supg_entry(c, i, j) : 0.0);
  }
}

__global__ void set_kappa_kernel(MacroInfo* info, const double* kappa, int64_t n, int32_t* bad) {
  int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e < n) {
    const double k = kappa[e];
    info[e].kappa = k;
    bad[e] = (k > 0.0 && k < __builtin_huge_val()) ? 0 : 1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(T* fac, const MacroInfo* __restrict__ info,
                                                       const double* __restrict__ tm, Templates Tp,
                                                       double tau) {
  const MacroInfo& mi = info[blockIdx.x];
  const int N = mi.N, ld = mi.ld;
  const int rows_per = 8;
  const int r0 = blockIdx.y * rows_per;
  if (r0 >= N) return;
  EntryCtx c = make_ctx(mi, tm, Tp, tau);
  T* A = fac + mi.fac_off;
  const int r1 = min(N, r0 + rows_per);
  for (int r = r0; r < r1; ++r)
    for (int col = threadIdx.x; col < N; col += blockDim.x)
      A[size_t(r) * ld + col] = (T)a_entry(c, r, col);
}

// Schur block of the flux-eliminated form, row-major into the block at sfac_off:
// S_u = K + kappa |det J| (c_00 L_00 + c_01 (L_01 + L_01^T) + c_11 L_11) with
// c_ab = sum_d g_ad g_bd, g_0d = G[d], g_1d = G[2 + d] (E^d = |det J| sum_a
// g_ad Ehat^a) and K the u-u block of A_K.
__global__ __launch_bounds__(256) void qelim_assemble_kernel(double* fac,
                                                             const MacroInfo* __restrict__ info,
                                                             const double* __restrict__ tm,
                                                             Templates Tp,
                                                             const double* __restrict__ qt,
                                                             QTemplates QT, double tau) {
  const MacroInfo& mi = info[blockIdx.x];
  const int Q = mi.Q, ld = mi.sld;
  const int rows_per = 8;
  const int r0 = blockIdx.y * rows_per;
  if (r0 >= Q) return;
  EntryCtx c = make_ctx(mi, tm, Tp, tau);
  const QLevel& QL = QT.lev[mi.level];
  const double* L00 = qt + QL.L00;
  const double* L01 = qt + QL.L01;
  const double* L11 = qt + QL.L11;
  const double G0 = mi.G[0], G1 = mi.G[1], G2 = mi.G[2], G3 = mi.G[3];
  const double c00 = G0 * G0 + G1 * G1, c01 = G0 * G2 + G1 * G3, c11 = G2 * G2 + G3 * G3;
  const double sc = mi.kappa * mi.dJ;
  double* A = fac + mi.sfac_off;
  const int r1 = min(Q, r0 + rows_per);
  for (int r = r0; r < r1; ++r)
    for (int col = threadIdx.x; col < Q; col += blockDim.x) {
      const size_t o = size_t(r) * Q + col;
      const double lap = c00 * L00[o] + c01 * (L01[o] + L01[size_t(col) * Q + r]) + c11 * L11[o];
      A[size_t(r) * ld + col] = a_entry(c, 2 * Q + r, 2 * Q + col) + sc * lap;
    }
}

hipError_t launch_qelim_assemble(double* fac, const MacroInfo* info, int64_t n, int maxQ,
                                 const double* tmpl, const Templates& T, const double* qtm,
                                 const QTemplates& QT, double tau, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)n, (unsigned)((maxQ + 7) / 8));
  hipLaunchKernelGGL(qelim_assemble_kernel, grid, dim3(256), 0, s, fac, info, tmpl, T, qtm, QT,
                     tau);
  return hipGetLastError();
}

__global__ void extract_kernel(const MacroInfo* info, int64_t e, const double* tm, Templates Tp,
                               double tau, double* dst) {
  const MacroInfo& mi = info[e];
  EntryCtx c = make_ctx(mi, tm, Tp, tau);
  const int N = mi.N;
  const int r = blockIdx.x;
  if (r >= N) return;
  for (int col = threadIdx.x; col < N; col += blockDim.x) dst[size_t(r) * N + col] = a_entry(c, r, col);
}

// ------------------------------------------------------------------ LU
// One workgroup of NT threads factors one macro's N x N row-major block in
// place: PA = LU with partial pivoting (largest |a|, ties to the smallest
// row).  Panels of NB columns are held in registers (thread t owns rows
// k0 + t + q NT); the pivot search is a wavefront max-reduction followed by a
// cross-wave reduction in LDS; the trailing update runs on MFMA 16x16x4 tiles.
// perm[i] receives the original row of factor row i; status = first zero
// pivot column + 1, or 0.  On exit L (unit lower) and U are stored
// column-major in the block: element (i, j) at j * ld + i, ld = N rounded up
// to 16 (FP64 columns start on 128-byte lines).
template <typename T, int NT, int RPT, int NB>
__global__ __launch_bounds__(NT) void lu_kernel(T* fac, const MacroInfo* __restrict__ info,
                                                const int32_t* __restrict__ order, int64_t base,
                                                int32_t* perm_all, int32_t* status) {
  constexpr int NW = NT / 64;
  const int e = order[base + blockIdx.x];
  const MacroInfo& mi = info[e];
  const int N = mi.N, ld = mi.ld;   // rows of the stored block are ld apart
  T* A = fac + mi.fac_off;
  int32_t* perm = perm_all + mi.loc_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  __shared__ double s_red_v[NW];
  __shared__ int s_red_i[NW];
  __shared__ T s_row[NB];
  __shared__ T s_swap[2][NB];
  __shared__ T s_L11[NB * NB];
  __shared__ int s_piv[NB];
  __shared__ int s_status;

  for (int i = tid; i < N; i += NT) perm[i] = i;
  if (tid == 0) s_status = 0;
  __syncthreads();

  T pr[RPT][NB];
  for (int k0 = 0; k0 < N; k0 += NB) {
    const int nb = min(NB, N - k0);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = k0 + tid + q * NT;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        pr[q][c] = (row < N && c < nb) ? A[size_t(row) * ld + k0 + c] : T(0);
    }
    // ---- panel factorisation
    for (int j = 0; j < nb; ++j) {
      const int col = k0 + j;
      // candidates are rows col..N-1; a NaN counts as +inf so that it is
      // chosen and reported, and the chosen row always lies in [col, N)
      double best = -1.0;
      int bidx = col;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = k0 + tid + q * NT;
        double v = -1.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c == j) v = pivot_mag((double)pr[q][c]);
        if (row >= col && row < N && v > best) { best = v; bidx = row; }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        double ov = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bidx, o, 64);
        if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
      }
      if (lane == 0) { s_red_v[wid] = best; s_red_i[wid] = bidx; }
      __syncthreads();
      best = s_red_v[0];
      bidx = s_red_i[0];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        double ov = s_red_v[w];
        int oi = s_red_i[w];
        if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
      }
      const int prow = min(max(bidx, col), N - 1);
      const int own_c = (col - k0) % NT, slot_c = (col - k0) / NT;
      const int own_p = (prow - k0) % NT, slot_p = (prow - k0) / NT;
      if (prow != col) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (tid == own_p && q == slot_p)
            for (int c = 0; c < NB; ++c) s_swap[0][c] = pr[q][c];
          if (tid == own_c && q == slot_c)
            for (int c = 0; c < NB; ++c) s_swap[1][c] = pr[q][c];
        }
      }
      __syncthreads();
      if (prow != col) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (tid == own_c && q == slot_c)
            for (int c = 0; c < NB; ++c) pr[q][c] = s_swap[0][c];
          if (tid == own_p && q == slot_p)
            for (int c = 0; c < NB; ++c) pr[q][c] = s_swap[1][c];
        }
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (tid == own_c && q == slot_c)
          for (int c = 0; c < NB; ++c) s_row[c] = pr[q][c];
      if (tid == 0) {
        s_piv[j] = prow;
        if (s_status == 0) s_status = pivot_status(best, col);
      }
      __syncthreads();
      if (best != 0.0) {
        const T piv = s_row[j];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int row = k0 + tid + q * NT;
          if (row > col && row < N) {
            T l = T(0);
#pragma unroll
            for (int c = 0; c < NB; ++c)
              if (c == j) { l = pr[q][c] / piv; pr[q][c] = l; }
#pragma unroll
            for (int c = 0; c < NB; ++c)
              if (c > j) pr[q][c] -= l * s_row[c];
          }
        }
      }
    }
    // ---- write the panel back; keep L11 in LDS
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = k0 + tid + q * NT;
      if (row < N) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nb) A[size_t(row) * ld + k0 + c] = pr[q][c];
        if (row < k0 + nb)
          for (int c = 0; c < NB; ++c) s_L11[(row - k0) * NB + c] = pr[q][c];
      }
    }
    __syncthreads();
    // ---- row interchanges outside the panel, in pivot order
    for (int c = tid; c < N; c += NT) {
      if (c >= k0 && c < k0 + nb) continue;
      for (int j = 0; j < nb; ++j) {
        const int prow = s_piv[j], col = k0 + j;
        if (prow != col) {
          T a = A[size_t(col) * ld + c], b = A[size_t(prow) * ld + c];
          A[size_t(col) * ld + c] = b;
          A[size_t(prow) * ld + c] = a;
        }
      }
    }
    if (tid == 0)
      for (int j = 0; j < nb; ++j) {
        const int prow = s_piv[j], col = k0 + j;
        if (prow != col) { int t = perm[col]; perm[col] = perm[prow]; perm[prow] = t; }
      }
    __syncthreads();
    if (k0 + nb >= N) break;
    // ---- U12 = L11^-1 A12
    for (int c = k0 + nb + tid; c < N; c += NT) {
      T v[NB];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) v[jj] = jj < nb ? A[size_t(k0 + jj) * ld + c] : T(0);
#pragma unroll
      for (int jj = 1; jj < NB; ++jj)
#pragma unroll
        for (int ii = 0; ii < jj; ++ii) v[jj] -= s_L11[jj * NB + ii] * v[ii];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        if (jj < nb) A[size_t(k0 + jj) * ld + c] = v[jj];
    }
    __syncthreads();
    // ---- A22 -= L21 U12 on MFMA 16x16x4 tiles
    {
      const int base = k0 + nb;
      const int nt = (N - base + 15) / 16;
      const int li = lane & 15, lk = lane >> 4;
      for (int rt = wid; rt < nt; rt += NW) {
        const int r0 = base + 16 * rt;
        T a[NB / 4];
#pragma unroll
        for (int s = 0; s < NB / 4; ++s) {
          const int k = 4 * s + lk, row = r0 + li;
          a[s] = (row < N && k < nb) ? -A[size_t(row) * ld + k0 + k] : T(0);
        }
        for (int ct = 0; ct < nt; ++ct) {
          const int c0 = base + 16 * ct;
          const int colc = c0 + li;
          T b[NB / 4];
#pragma unroll
          for (int s = 0; s < NB / 4; ++s) {
            const int k = 4 * s + lk;
            b[s] = (k < nb && colc < N) ? A[size_t(k0 + k) * ld + colc] : T(0);
          }
          typename Mfma<T>::acc acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = r0 + Mfma<T>::drow(lk, v);
            acc[v] = (row < N && colc < N) ? A[size_t(row) * ld + colc] : T(0);
          }
#pragma unroll
          for (int s = 0; s < NB / 4; ++s) acc = Mfma<T>::run(a[s], b[s], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = r0 + Mfma<T>::drow(lk, v);
            if (row < N && colc < N) A[size_t(row) * ld + colc] = acc[v];
          }
        }
      }
    }
    __syncthreads();
  }
  // ---- store the factors column-major (in-place transpose by 32 x 32 tile pairs):
  // the triangular solves then read one contiguous column per step.
  __syncthreads();
  {
    __shared__ T t0[32][33];
    __shared__ T t1[32][33];
    const int nt = (N + 31) / 32;
    for (int I = 0; I < nt; ++I)
      for (int J = I; J < nt; ++J) {
        for (int e = tid; e < 1024; e += NT) {
          const int a = e >> 5, b = e & 31;
          const int r = 32 * I + a, c = 32 * J + b;
          t0[a][b] = (r < N && c < N) ? A[size_t(r) * ld + c] : T(0);
          const int r2 = 32 * J + a, c2 = 32 * I + b;
          t1[a][b] = (r2 < N && c2 < N) ? A[size_t(r2) * ld + c2] : T(0);
        }
        __syncthreads();
        for (int e = tid; e < 1024; e += NT) {
          const int a = e >> 5, b = e & 31;
          const int r = 32 * I + a, c = 32 * J + b;
          if (r < N && c < N) A[size_t(r) * ld + c] = t1[b][a];
          const int r2 = 32 * J + a, c2 = 32 * I + b;
          if (r2 < N && c2 < N) A[size_t(r2) * ld + c2] = t0[b][a];
        }
        __syncthreads();
      }
  }
  if (tid == 0) status[e] = s_status;
}

// ------------------------------------------------------------------ step 4
__global__ __launch_bounds__(64) void face_combine_kernel(int mode, const FaceInfo* __restrict__ fi,
                                                          const double* __restrict__ tm, Templates Tp,
                                                          double tau, const double* __restrict__ lam,
                                                          const double* __restrict__ slots,
                                                          double* __restrict__ out,
                                                          const int32_t* __restrict__ skip) {
  __shared__ double v[(1 << kMaxLevel) * 4 + 1];
  __shared__ double lf[(1 << kMaxLevel) * 4 + 1];
  const FaceInfo& f = fi[blockIdx.x];
  const int nF = f.nF;
  if (skip && skip[f.inst]) {   // converged instance: its slots are stale
    for (int l = threadIdx.x; l < nF; l += 64) out[f.tr_off + l] = 0.0;
    return;
  }
  const LevelTemplates& L = Tp.lev[f.level];
  for (int l = threadIdx.x; l < nF; l += 64) {
    v[l] = mode == FACE_DINV ? 0.0 : slots[f.slot[0] + l] + slots[f.slot[1] + l];
    lf[l] = lam ? lam[f.tr_off + l] : 0.0;
  }
  __syncthreads();
  const double* M1 = tm + L.M1;
  const double* Mi = tm + L.M1inv;
  for (int l = threadIdx.x; l < nF; l += 64) {
    double r;
    if (mode == FACE_S || mode == FACE_RESID) {
      double d = 0.0;  // D_F lam = -2 tau |F| M1 lam
      for (int k = 0; k < nF; ++k) d += M1[size_t(l) * nF + k] * lf[k];
      d *= -2.0 * tau * f.len;
      r = mode == FACE_S ? d - v[l] : d + v[l];
    } else if (mode == FACE_RHS) {
      r = -v[l];
    } else if (mode == FACE_DINV) {
      double d = 0.0;  // D_F^-1 lam = -M1^-1 lam / (2 tau |F|)
      for (int k = 0; k < nF; ++k) d += Mi[size_t(l) * nF + k] * lf[k];
      r = -d / (2.0 * tau * f.len);
    } else {
      double d = 0.0;  // -D_F^-1 v = M1^-1 v / (2 tau |F|)
      for (int k = 0; k < nF; ++k) d += Mi[size_t(l) * nF + k] * v[k];
      d /= 2.0 * tau * f.len;
      r = mode == FACE_PREC_S ? lf[l] + d : d;
    }
    out[f.tr_off + l] = r;
  }
}

// Step 4 for n_rhs vectors in one launch (workgroup (face, vector)): vector v
// reads lam + v * ld_lam and slots + v * ld_slots and writes out + v * ld_lam.
// out = D lam - v^ (precondition = 0) or lam - D^-1 v^ (precondition = 1).
__global__ __launch_bounds__(64) void face_combine_many_kernel(
    int precondition, const FaceInfo* __restrict__ fi, const double* __restrict__ tm,
    Templates Tp, double tau, const double* __restrict__ lam, int64_t ld_lam,
    const double* __restrict__ slots, int64_t ld_slots, double* __restrict__ out) {
  __shared__ double v[(1 << kMaxLevel) * 4 + 1];
  __shared__ double lf[(1 << kMaxLevel) * 4 + 1];
  const FaceInfo& f = fi[blockIdx.x];
  const int nF = f.nF;
  const double* lv = lam + int64_t(blockIdx.y) * ld_lam + f.tr_off;
  const double* sv = slots + int64_t(blockIdx.y) * ld_slots;
  double* ov = out + int64_t(blockIdx.y) * ld_lam + f.tr_off;
  for (int l = threadIdx.x; l < nF; l += 64) {
    v[l] = sv[f.slot[0] + l] + sv[f.slot[1] + l];
    lf[l] = lv[l];
  }
  __syncthreads();
  const LevelTemplates& L = Tp.lev[f.level];
  const double* M = tm + (precondition ? L.M1inv : L.M1);
  for (int l = threadIdx.x; l < nF; l += 64) {
    double d = 0.0;
    if (precondition) {   // lam - D_F^-1 v = lam + M1^-1 v / (2 tau |F|)
      for (int k = 0; k < nF; ++k) d += M[size_t(l) * nF + k] * v[k];
      ov[l] = lf[l] + d / (2.0 * tau * f.len);
    } else {              // D_F lam - v = -2 tau |F| M1 lam - v
      for (int k = 0; k < nF; ++k) d += M[size_t(l) * nF + k] * lf[k];
      ov[l] = d * (-2.0 * tau * f.len) - v[l];
    }
  }
}

// ------------------------------------------------------------------ data
// lam_D = M1^-1 b, b_l = sum over segments and sampling points of
// (w_q / npc) g_q mu_l(t_q): the L2 projection of g_D onto M(F).
__global__ __launch_bounds__(64) void dirichlet_kernel(const BndFaceInfo* __restrict__ bf,
                                                       const double* __restrict__ tm, Templates Tp,
                                                       const double* __restrict__ g,
                                                       double* __restrict__ lamD) {
  __shared__ double b[(1 << kMaxLevel) * 4 + 1];
  const BndFaceInfo& f = bf[blockIdx.x];
  const int p = Tp.p, kb = Tp.kb, nF = f.nF, npc = 1 << f.level;
  const double* phi = tm + Tp.dir_basis;
  const double* w = tm + Tp.dir_w;
  for (int l = threadIdx.x; l < nF; l += 64) {
    double acc = 0.0;
    // node l belongs to segment l/p (local a = l%p) and, if l%p == 0, to segment l/p - 1 (a = p)
    const int c1 = l / p, a1 = l % p;
    if (c1 < npc)
      for (int q = 0; q < kb; ++q) acc += w[q] * g[f.g_off + c1 * kb + q] * phi[a1 * kb + q];
    if (a1 == 0 && c1 > 0)
      for (int q = 0; q < kb; ++q) acc += w[q] * g[f.g_off + (c1 - 1) * kb + q] * phi[p * kb + q];
    b[l] = acc / npc;
  }
  __syncthreads();
  const double* Mi = tm + Tp.lev[f.level].M1inv;
  for (int l = threadIdx.x; l < nF; l += 64) {
    double acc = 0.0;
    for (int k = 0; k < nF; ++k) acc += Mi[size_t(l) * nF + k] * b[k];
    lamD[f.lam_off + l] = acc;
  }
}

// R_K = [0; 0; |det J| Mhat f_K] - sum over Dirichlet edges of B_k lam_D
__global__ __launch_bounds__(64) void local_rhs_kernel(const MacroInfo* __restrict__ info,
                                                       const BndFaceInfo* __restrict__ bf,
                                                       const double* __restrict__ tm, Templates Tp,
                                                       const double* __restrict__ f,
                                                       const double* __restrict__ lamD, double tau,
                                                       double* __restrict__ R) {
  extern __shared__ double x[];
  const MacroInfo& mi = info[blockIdx.x];
  const int N = mi.N, Q = mi.Q;
  const double* Mh = tm + Tp.lev[mi.level].Mhat;
  const double* fK = f + mi.node_off;
  // SUPG source tau (a.grad w, f_h)_K = tau |det J| (al0 Ehat^0 + al1 Ehat^1) f_K
  const double ts = supg_tau(mi);
  const double* E0 = tm + Tp.lev[mi.level].E0;
  const double* E1 = tm + Tp.lev[mi.level].E1;
  const double al0 = ts * (mi.G[0] * mi.bx + mi.G[1] * mi.by);
  const double al1 = ts * (mi.G[2] * mi.bx + mi.G[3] * mi.by);
  for (int i = threadIdx.x; i < N; i += 64) {
    double v = 0.0;
    if (i >= 2 * Q) {
      const int ii = i - 2 * Q;
      for (int j = 0; j < Q; ++j) v += Mh[size_t(ii) * Q + j] * fK[j];
      if (ts != 0.0)
        for (int j = 0; j < Q; ++j)
          v += (al0 * E0[size_t(ii) * Q + j] + al1 * E1[size_t(ii) * Q + j]) * fK[j];
      v *= mi.dJ;
    }
    x[i] = v;
  }
  __syncthreads();
  // Dirichlet columns of B_K, accumulated in compact boundary form then added
  const int P = mi.P, NBD = 3 * P;
  double* xc = x + N;
  for (int i = threadIdx.x; i < 3 * NBD; i += 64) xc[i] = 0.0;
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    if (mi.bnd_face[k] >= 0)
      edge_B(mi, k, tm, Tp, lamD + bf[mi.bnd_face[k]].lam_off, -1.0, tau, xc);
    __syncthreads();
  }
  const int32_t* en = ints(tm, Tp.lev[mi.level].edge_node);
  for (int b = threadIdx.x; b < NBD; b += 64) {
    const int node = en[(b / P) * (P + 1) + b % P];
    for (int f = 0; f < 3; ++f) x[f * Q + node] += xc[f * NBD + b];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += 64) R[mi.loc_off + i] = x[i];
}

// ------------------------------------------------------------------ macro conservation
// out_K = <flux^.n, 1>_dK - (f_h, 1)_K with the LDG-H flux
// flux^.n = a.n lam + kappa q.n + tau (u - lam) (section 3.1): the local
// problem tested with w = 1, which lies in the macro's space, so the value
// vanishes (to rounding) for every U_K that solves its local problem.  Per
// edge k, with G[i][l] = |F| T1[s][l] and sum_l mu_l = 1 on the face:
//   <lam, 1>_F = |F| sum_s sum_l T1[s][l] lam_l,
//   <v, 1>_F   = |F| sum_s (sum_l T1[s][l]) v(node s)   (v = q_x, q_y, u),
// lam being the interior trace or the Dirichlet trace of a boundary face;
// (f_h, 1)_K = |det J| 1^T Mhat f_K.  One wavefront per macro.
__global__ __launch_bounds__(64) void flux_balance_kernel(
    const MacroInfo* __restrict__ info, const BndFaceInfo* __restrict__ bf,
    const double* __restrict__ tm, Templates Tp, double tau, const double* __restrict__ lam,
    const double* __restrict__ lamD, const double* __restrict__ U,
    const double* __restrict__ f, double* __restrict__ out) {
  const MacroInfo& mi = info[blockIdx.x];
  const int Q = mi.Q, P = mi.P, lane = threadIdx.x, p = Tp.p;
  const LevelTemplates& LT = Tp.lev[mi.level];
  const double* Mh = tm + LT.Mhat;
  const double* fK = f + mi.node_off;
  const double* qx = U + mi.loc_off;
  const double* qy = qx + Q;
  const double* u = qx + 2 * Q;
  double acc = 0.0;
  for (int i = lane; i < Q; i += 64) {
    double v = 0.0;
    for (int j = 0; j < Q; ++j) v += Mh[size_t(i) * Q + j] * fK[j];
    acc -= mi.dJ * v;
  }
  const int32_t* en = ints(tm, LT.edge_node);
  for (int k = 0; k < 3; ++k) {
    const double* lF = mi.tr_off[k] >= 0 ? lam + mi.tr_off[k]
                                         : lamD + bf[mi.bnd_face[k]].lam_off;
    const int nF = (1 << mi.flevel[k]) * p + 1;
    const double* T1 = tm + LT.T1[mi.flevel[k]];
    const double nx = mi.nrm[2 * k], ny = mi.nrm[2 * k + 1];
    const double an = mi.bx * nx + mi.by * ny;
    double e = 0.0;
    for (int s = lane; s <= P; s += 64) {
      const int sc = mi.orient[k] > 0 ? s : P - s;
      double w = 0.0, gl = 0.0;
      for (int l = 0; l < nF; ++l) {
        const double t = T1[size_t(sc) * nF + l];
        w += t;
        gl += t * lF[l];
      }
      const int node = en[k * (P + 1) + s];
      e += (an - tau) * gl + (mi.kappa * (nx * qx[node] + ny * qy[node]) + tau * u[node]) * w;
    }
    acc += mi.len[k] * e;
  }
  acc = wave_sum(acc);
  if (lane == 0) out[blockIdx.x] = acc;
}

hipError_t launch_flux_balance(const MacroInfo* info, int64_t n, const BndFaceInfo* bf,
                               const double* tmpl, const Templates& T, double tau,
                               const double* lam, const double* lamD, const double* U,
                               const double* f, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(flux_balance_kernel, dim3((unsigned)n), dim3(64), 0, s, info, bf, tmpl, T,
                     tau, lam, lamD, U, f, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ FP64 residual of the local rows
// out_K = R_K - A_K U_K - B_K lam_K in FP64, matrix-free: with the reference
// templates (Mhat symmetric, E^k and their transposes) the three block rows are
//   v_x: |J| Mhat q_x - E^x u,   v_y: |J| Mhat q_y - E^y u,
//   w:   kappa (E^x^T q_x + E^y^T q_y) - (a_x E^x + a_y E^y) u + tau Mb u,
// E^d = |J| sum_k G[k][d] Ehat^k.  lam may be NULL (no trace term).
__global__ __launch_bounds__(256) void local_residual_kernel(
    const MacroInfo* __restrict__ info, const double* __restrict__ tm, Templates Tp,
    double tau, const double* __restrict__ R, const double* __restrict__ U,
    const double* __restrict__ lam, double* __restrict__ out) {
  extern __shared__ double sh[];
  const MacroInfo& mi = info[blockIdx.x];
  const int N = mi.N, Q = mi.Q, P = mi.P, NBD = 3 * P;
  const LevelTemplates& L = Tp.lev[mi.level];
  double* u = sh;
  double* xc = sh + N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) u[i] = U[mi.loc_off + i];
  for (int i = threadIdx.x; i < 3 * NBD; i += blockDim.x) xc[i] = 0.0;
  __syncthreads();
  if (lam)
    for (int k = 0; k < 3; ++k) {
      if (mi.tr_off[k] >= 0) edge_B(mi, k, tm, Tp, lam + mi.tr_off[k], 1.0, tau, xc);
      __syncthreads();
    }
  const double* Mh = tm + L.Mhat;
  const double* E0 = tm + L.E0;
  const double* E1 = tm + L.E1;
  const double* E0T = tm + L.E0T;
  const double* E1T = tm + L.E1T;
  const double* M1 = tm + L.M1;
  const int32_t* ep = ints(tm, L.node_epos);
  const int32_t* en = ints(tm, L.edge_node);
  const int32_t* bidx = ints(tm, L.bnd_index);
  const double dJ = mi.dJ, g0 = mi.G[0], g1 = mi.G[1], g2 = mi.G[2], g3 = mi.G[3];
  const EntryCtx sc = make_ctx(mi, tm, Tp, tau);
  for (int i = threadIdx.x; i < Q; i += blockDim.x) {
    double mqx = 0, mqy = 0, e0u = 0, e1u = 0, e0x = 0, e1x = 0, e0y = 0, e1y = 0;
    for (int j = 0; j < Q; ++j) {
      const size_t o = size_t(j) * Q + i;
      const double qx = u[j], qy = u[Q + j], uu = u[2 * Q + j];
      const double m = Mh[o], a0 = E0T[o], a1 = E1T[o], b0 = E0[o], b1 = E1[o];
      mqx += m * qx;
      mqy += m * qy;
      e0u += a0 * uu;     // (Ehat^0 u)_i
      e1u += a1 * uu;
      e0x += b0 * qx;     // (Ehat^0^T q_x)_i
      e1x += b1 * qx;
      e0y += b0 * qy;
      e1y += b1 * qy;
    }
    const double Exu = dJ * (g0 * e0u + g2 * e1u), Eyu = dJ * (g1 * e0u + g3 * e1u);
    const double ExTqx = dJ * (g0 * e0x + g2 * e1x), EyTqy = dJ * (g1 * e0y + g3 * e1y);
    double mbu = 0.0;
    for (int k = 0; k < 3; ++k) {
      const int si = ep[3 * i + k];
      if (si < 0) continue;
      const int lo = si - Tp.p > 0 ? si - Tp.p : 0, hi = si + Tp.p < P ? si + Tp.p : P;
      double acc = 0.0;
      for (int s2 = lo; s2 <= hi; ++s2) acc += M1[size_t(si) * (P + 1) + s2] * u[2 * Q + en[k * (P + 1) + s2]];
      mbu += mi.len[k] * acc;
    }
    double av[3];
    av[0] = dJ * mqx - Exu;
    av[1] = dJ * mqy - Eyu;
    av[2] = mi.kappa * (ExTqx + EyTqy) - (mi.bx * Exu + mi.by * Eyu) + tau * mbu;
    if (sc.Sp) {   // SUPG block row i (row-major templates)
      double su = 0.0;
      for (int j = 0; j < Q; ++j) su += supg_entry(sc, i, j) * u[2 * Q + j];
      av[2] += su;
    }
    const int b = bidx[i];
    for (int f = 0; f < 3; ++f) {
      double r = R[mi.loc_off + f * Q + i] - av[f];
      if (b >= 0) r -= xc[f * NBD + b];
      out[mi.loc_off + f * Q + i] = r;
    }
  }
}

// slots of macro K <- C_K U_K (step 3 applied to a given local vector)
__global__ __launch_bounds__(64) void boundary_C_kernel(const MacroInfo* __restrict__ info,
                                                        const double* __restrict__ tm, Templates Tp,
                                                        double tau, const double* __restrict__ U,
                                                        double* __restrict__ slots) {
  extern __shared__ double zc[];
  const MacroInfo& mi = info[blockIdx.x];
  const int Q = mi.Q, P = mi.P, NBD = 3 * P;
  const int32_t* en = ints(tm, Tp.lev[mi.level].edge_node);
  for (int b = threadIdx.x; b < NBD; b += 64) {
    const int node = en[(b / P) * (P + 1) + b % P];
    for (int f = 0; f < 3; ++f) zc[f * NBD + b] = U[mi.loc_off + f * Q + node];
  }
  __syncthreads();
  for (int k = 0; k < 3; ++k)
    if (mi.tr_off[k] >= 0) edge_C(mi, k, tm, Tp, zc, tau, slots + mi.slot_off[k]);
}

// ------------------------------------------------------------------ adjoint contractions
// For macro K with forward solution U = (q_x, q_y, u), local adjoint
// Psi = (psi_x, psi_y, psi_w), trace adjoint psi_lam and traces lam_k on its
// edges (interior: global trace, Dirichlet: projected data):
//   dJ/dkappa_K = -[psi_w^T (E^x^T q_x + E^y^T q_y) + sum_{interior k} psi_lam,k^T G_k^T (n_x q_x + n_y q_y)]
//   dJ/da_d (macro part) = psi_w^T E^d u - n_d sum_k lam_k^T G_k^T psi_w
// (A_K and C_K are affine in kappa_K; A_K through -(a.E) u and B_K through
// (a.n - tau) are affine in a; D_F does not depend on a, f and tau are fixed).
__global__ __launch_bounds__(256) void adjoint_contract_kernel(
    const MacroInfo* __restrict__ info, const BndFaceInfo* __restrict__ bf,
    const double* __restrict__ tm, Templates Tp, const double* __restrict__ U,
    const double* __restrict__ Psi, const double* __restrict__ lam,
    const double* __restrict__ psi_lam, const double* __restrict__ lamD,
    double* __restrict__ dkappa, double* __restrict__ dbeta_part) {
  extern __shared__ double sh[];
  __shared__ double red[3][256];
  const MacroInfo& mi = info[blockIdx.x];
  const int N = mi.N, Q = mi.Q, P = mi.P;
  const LevelTemplates& L = Tp.lev[mi.level];
  double* u = sh;
  double* ps = sh + N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    u[i] = U[mi.loc_off + i];
    ps[i] = Psi[mi.loc_off + i];
  }
  __syncthreads();
  const double* E0 = tm + L.E0;
  const double* E1 = tm + L.E1;
  const double* E0T = tm + L.E0T;
  const double* E1T = tm + L.E1T;
  const double dJ = mi.dJ, g0 = mi.G[0], g1 = mi.G[1], g2 = mi.G[2], g3 = mi.G[3];
  double ak = 0.0, abx = 0.0, aby = 0.0;
  for (int i = threadIdx.x; i < Q; i += blockDim.x) {
    double e0x = 0, e1x = 0, e0y = 0, e1y = 0, e0u = 0, e1u = 0;
    for (int j = 0; j < Q; ++j) {
      const size_t o = size_t(j) * Q + i;
      const double b0 = E0[o], b1 = E1[o], a0 = E0T[o], a1 = E1T[o];
      e0x += b0 * u[j];
      e1x += b1 * u[j];
      e0y += b0 * u[Q + j];
      e1y += b1 * u[Q + j];
      e0u += a0 * u[2 * Q + j];
      e1u += a1 * u[2 * Q + j];
    }
    const double pw = ps[2 * Q + i];
    ak += pw * dJ * ((g0 * e0x + g2 * e1x) + (g1 * e0y + g3 * e1y));
    abx += pw * dJ * (g0 * e0u + g2 * e1u);
    aby += pw * dJ * (g1 * e0u + g3 * e1u);
  }
  // edge terms
  const int32_t* en = ints(tm, L.edge_node);
  for (int k = 0; k < 3; ++k) {
    const int fl = mi.flevel[k];
    const int nF = (1 << fl) * Tp.p + 1;
    const double* T1 = tm + L.T1[fl];
    const double nx = mi.nrm[2 * k], ny = mi.nrm[2 * k + 1];
    const bool interior = mi.tr_off[k] >= 0;
    const double* lk = interior ? lam + mi.tr_off[k] : lamD + bf[mi.bnd_face[k]].lam_off;
    for (int l = threadIdx.x; l < nF; l += blockDim.x) {
      double gq = 0.0, gw = 0.0;
      for (int sc = 0; sc <= P; ++sc) {
        const int s = mi.orient[k] > 0 ? sc : P - sc;
        const int node = en[k * (P + 1) + s];
        const double t = T1[size_t(sc) * nF + l];
        gq += t * (nx * u[node] + ny * u[Q + node]);
        gw += t * ps[2 * Q + node];
      }
      gq *= mi.len[k];
      gw *= mi.len[k];
      if (interior) ak += psi_lam[mi.tr_off[k] + l] * gq;
      abx -= nx * lk[l] * gw;
      aby -= ny * lk[l] * gw;
    }
  }
  red[0][threadIdx.x] = ak;
  red[1][threadIdx.x] = abx;
  red[2][threadIdx.x] = aby;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dkappa[blockIdx.x] = -red[0][0];
    dbeta_part[2 * blockIdx.x] = red[1][0];
    dbeta_part[2 * blockIdx.x + 1] = red[2][0];
  }
}

// out[c] = sum_K part[stride K + c] in a fixed order (c < stride)
__global__ __launch_bounds__(256) void strided_sum_kernel(const double* __restrict__ part, int64_t n,
                                                          int stride, double* __restrict__ out) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int64_t K = threadIdx.x; K < n; K += 256) acc += part[K * stride + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// out_K,f = M_K v_K,f for the three fields (M_K = |det J| Mhat, the macro mass matrix)
__global__ __launch_bounds__(256) void mass_kernel(const MacroInfo* __restrict__ info,
                                                   const double* __restrict__ tm, Templates Tp,
                                                   const double* __restrict__ v, double* __restrict__ out) {
  extern __shared__ double sh[];
  const MacroInfo& mi = info[blockIdx.x];
  const int N = mi.N, Q = mi.Q;
  const double* Mh = tm + Tp.lev[mi.level].Mhat;
  for (int i = threadIdx.x; i < N; i += blockDim.x) sh[i] = v[mi.loc_off + i];
  __syncthreads();
  for (int i = threadIdx.x; i < Q; i += blockDim.x) {
    double a0 = 0, a1 = 0, a2 = 0;
    for (int j = 0; j < Q; ++j) {
      const double m = Mh[size_t(j) * Q + i];
      a0 += m * sh[j];
      a1 += m * sh[Q + j];
      a2 += m * sh[2 * Q + j];
    }
    out[mi.loc_off + i] = mi.dJ * a0;
    out[mi.loc_off + Q + i] = mi.dJ * a1;
    out[mi.loc_off + 2 * Q + i] = mi.dJ * a2;
  }
}

// ------------------------------------------------------------------ vector ops
// Row chunks of the Krylov vectors handled by one partial dot product.
constexpr int kDotChunk = 2048;   // rows per partial sum: enough workgroups for a few columns

int dots_nblk(int64_t n) {
  int64_t b = (n + kDotChunk - 1) / kDotChunk;
  return (int)(b < 1 ? 1 : b);
}

// partial[c * nblk + blk] = sum over row chunk blk of V[c][i] w[i]: one
// wavefront per (column, chunk), coalesced loads, a fixed-order reduction.
// The vectors hold nseg independent segments of length n (one per coefficient
// instance); block x handles chunk (x % nblk) of segment (x / nblk).
__global__ __launch_bounds__(256) void dots_partial_kernel(const double* __restrict__ V, int64_t ld,
                                                           int ncols, const double* __restrict__ w,
                                                           int64_t n, double* __restrict__ partial,
                                                           const int32_t* __restrict__ skip) {
  const int nblk_all = gridDim.x;
  const int nblk = n > kDotChunk ? (int)((n + kDotChunk - 1) / kDotChunk) : 1;   // = dots_nblk(n)
  const int seg = blockIdx.x / nblk, blk = blockIdx.x % nblk;
  const int nseg = nblk_all / nblk;
  const int c = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= ncols || (skip && skip[seg])) return;
  const double* v = V + c * ld + int64_t(seg) * n;
  w += int64_t(seg) * n;
  const int64_t i0 = int64_t(blk) * kDotChunk;
  const int64_t i1 = i0 + kDotChunk < n ? i0 + kDotChunk : n;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t i = i0 + lane;
  for (; i + 192 < i1; i += 256) {
    a0 += v[i] * w[i];
    a1 += v[i + 64] * w[i + 64];
    a2 += v[i + 128] * w[i + 128];
    a3 += v[i + 192] * w[i + 192];
  }
  for (; i < i1; i += 64) a0 += v[i] * w[i];
  const double acc = wave_sum((a0 + a1) + (a2 + a3));
  if (lane == 0) partial[(int64_t(c) * nseg + seg) * nblk + blk] = acc;
}

// Two inner products per column in one read of V: for column c and segment
// seg, partial[((2c + 0) nseg + seg) nblk + blk] = <V_c, x> and
// partial[((2c + 1) nseg + seg) nblk + blk] = <V_c, y> over one chunk.  A
// workgroup takes eight columns over one chunk; its 256 threads stride the
// chunk together, each loading x and y once for all eight columns (ten
// independent loads per element), and the four wavefronts' sums meet in LDS.
__global__ __launch_bounds__(256) void dots2_partial_kernel(const double* __restrict__ V, int64_t ld,
                                                            int ncols, const double* __restrict__ x,
                                                            const double* __restrict__ y, int64_t n,
                                                            double* __restrict__ partial,
                                                            const int32_t* __restrict__ skip) {
  __shared__ double red[4][16];
  const int nblk = n > kDotChunk ? (int)((n + kDotChunk - 1) / kDotChunk) : 1;
  const int seg = blockIdx.x / nblk, blk = blockIdx.x % nblk;
  const int nseg = gridDim.x / nblk;
  const int cb = blockIdx.y * 8;
  const int nc = min(8, ncols - cb);
  if (skip && skip[seg]) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double* Vb = V + int64_t(cb) * ld + int64_t(seg) * n;
  x += int64_t(seg) * n;
  y += int64_t(seg) * n;
  const int64_t i0 = int64_t(blk) * kDotChunk;
  const int64_t i1 = i0 + kDotChunk < n ? i0 + kDotChunk : n;
  double ax[8], ay[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) ax[c] = ay[c] = 0.0;
  for (int64_t i = i0 + tid; i < i1; i += 256) {
    const double xv = x[i], yv = y[i];
    double v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = Vb[int64_t(c < nc ? c : 0) * ld + i];   // every load issued
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      ax[c] += v[c] * xv;
      ay[c] += v[c] * yv;
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const double sx = wave_sum(ax[c]), sy = wave_sum(ay[c]);
    if (lane == 0) {
      red[wid][2 * c] = sx;
      red[wid][2 * c + 1] = sy;
    }
  }
  __syncthreads();
  if (tid < 2 * nc) {
    const double v = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    const int c = cb + (tid >> 1), w = tid & 1;
    partial[(int64_t(2 * c + w) * nseg + seg) * nblk + blk] = v;
  }
}

// The same products for few columns (short Krylov bases): each wavefront takes
// two columns (c and c + 4 of its block's eight) over the whole chunk, so
// every load of x and y serves two columns and no LDS reduction is needed.
__global__ __launch_bounds__(256) void dots2_partial_narrow_kernel(const double* __restrict__ V, int64_t ld,
                                                            int ncols, const double* __restrict__ x,
                                                            const double* __restrict__ y, int64_t n,
                                                            double* __restrict__ partial,
                                                            const int32_t* __restrict__ skip) {
  const int nblk = n > kDotChunk ? (int)((n + kDotChunk - 1) / kDotChunk) : 1;
  const int seg = blockIdx.x / nblk, blk = blockIdx.x % nblk;
  const int nseg = gridDim.x / nblk;
  const int c0 = blockIdx.y * 8 + (threadIdx.x >> 6), c1 = c0 + 4;
  const int lane = threadIdx.x & 63;
  if (c0 >= ncols || (skip && skip[seg])) return;
  const bool two = c1 < ncols;
  const double* v0p = V + c0 * ld + int64_t(seg) * n;
  const double* v1p = V + (two ? c1 : c0) * ld + int64_t(seg) * n;
  x += int64_t(seg) * n;
  y += int64_t(seg) * n;
  const int64_t i0 = int64_t(blk) * kDotChunk;
  const int64_t i1 = i0 + kDotChunk < n ? i0 + kDotChunk : n;
  double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0, e0 = 0.0, e1 = 0.0, f0 = 0.0, f1 = 0.0;
  int64_t i = i0 + lane;
  for (; i + 64 < i1; i += 128) {
    const double x0 = x[i], x1 = x[i + 64], y0 = y[i], y1 = y[i + 64];
    const double p0 = v0p[i], p1 = v0p[i + 64], q0 = v1p[i], q1 = v1p[i + 64];
    a0 += p0 * x0;
    a1 += p1 * x1;
    b0 += p0 * y0;
    b1 += p1 * y1;
    e0 += q0 * x0;
    e1 += q1 * x1;
    f0 += q0 * y0;
    f1 += q1 * y1;
  }
  for (; i < i1; i += 64) {
    const double x0 = x[i], y0 = y[i], p0 = v0p[i], q0 = v1p[i];
    a0 += p0 * x0;
    b0 += p0 * y0;
    e0 += q0 * x0;
    f0 += q0 * y0;
  }
  const double sa = wave_sum(a0 + a1), sb = wave_sum(b0 + b1);
  const double se = wave_sum(e0 + e1), sf = wave_sum(f0 + f1);
  if (lane == 0) {
    partial[(int64_t(2 * c0) * nseg + seg) * nblk + blk] = sa;
    partial[(int64_t(2 * c0 + 1) * nseg + seg) * nblk + blk] = sb;
    if (two) {
      partial[(int64_t(2 * c1) * nseg + seg) * nblk + blk] = se;
      partial[(int64_t(2 * c1 + 1) * nseg + seg) * nblk + blk] = sf;
    }
  }
}

// Hessenberg correction of the delayed reorthogonalisation:
// out[i nseg + seg] = sum_{k < kmax, k >= i - 1} a_k Hb[(k ld + i) nseg + seg],
// with a_k = pq[(2k) nseg + seg] (the first products of dots2) and Hb the
// finished (unrotated) Hessenberg columns, column k holding rows 0..k+1.
// Block of 64 (row, segment) pairs x 8 groups of k; the 8 partial sums meet in LDS.
__global__ __launch_bounds__(512) void hbar_gemv_kernel(const double* __restrict__ Hb, int64_t ld,
                                                        int nseg, int kmax, int rows,
                                                        const double* __restrict__ pq,
                                                        double* __restrict__ out) {
  __shared__ double red[8][64];
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t t = blockIdx.x * int64_t(64) + lane;
  double acc = 0.0;
  if (t < int64_t(rows) * nseg) {
    const int i = (int)(t / nseg), seg = (int)(t % nseg);
    const int k0 = i > 0 ? i - 1 : 0;
#pragma unroll 4
    for (int kk = k0 + grp; kk < kmax; kk += 8)
      acc += pq[int64_t(2 * kk) * nseg + seg] * Hb[(int64_t(kk) * ld + i) * nseg + seg];
  }
  red[grp][lane] = acc;
  __syncthreads();
  if (grp == 0 && t < int64_t(rows) * nseg) {
    double s = 0.0;
#pragma unroll
    for (int g2 = 0; g2 < 8; ++g2) s += red[g2][lane];
    out[t] = s;
  }
}

// Fused update of the delayed reorthogonalisation, one read of V_0..V_{j-1}:
//   V_j     <- s1 u - sum_k ca_k V_k          (u = V_j on entry: q_j)
//   V_{j+1} <- s2 z + s3 u - sum_k cd_k V_k   (the next once-orthogonalised vector)
// coefficients per segment: ca, cd [k nseg + seg], s [3 nseg] = (s1, s2, s3).
// One element per lane; when a wavefront lies in one segment (all but the
// few straddling a segment boundary) its coefficients are wave-uniform and
// read with scalar loads, leaving one vector load per column.
__global__ __launch_bounds__(256) void dual_update_kernel(double* __restrict__ V, int64_t ld, int j,
                                                          int64_t n, int nseg,
                                                          const double* __restrict__ ca,
                                                          const double* __restrict__ cd,
                                                          const double* __restrict__ sc,
                                                          const double* __restrict__ z,
                                                          double* __restrict__ u2,
                                                          const int32_t* __restrict__ skip) {
  const int64_t total = n * nseg;
  const int64_t idx0 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const bool ok = idx0 < total;
  const int64_t idx = ok ? idx0 : total - 1;   // in-bounds address; result discarded
  const int seg = (int)(idx / n);
  if (skip && skip[seg]) return;   // segment out of this cycle: V left as it is
  const int seg0 = __builtin_amdgcn_readfirstlane(seg);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  if (__all(seg == seg0)) {
    const double* cas = ca + seg0;
    const double* cds = cd + seg0;
    int k = 0;
    for (; k + 3 < j; k += 4) {
      const double v0 = V[k * ld + idx], v1 = V[(k + 1) * ld + idx];
      const double v2 = V[(k + 2) * ld + idx], v3 = V[(k + 3) * ld + idx];
      a0 += cas[int64_t(k) * nseg] * v0;
      d0 += cds[int64_t(k) * nseg] * v0;
      a1 += cas[int64_t(k + 1) * nseg] * v1;
      d1 += cds[int64_t(k + 1) * nseg] * v1;
      a2 += cas[int64_t(k + 2) * nseg] * v2;
      d2 += cds[int64_t(k + 2) * nseg] * v2;
      a3 += cas[int64_t(k + 3) * nseg] * v3;
      d3 += cds[int64_t(k + 3) * nseg] * v3;
    }
    for (; k < j; ++k) {
      const double v0 = V[k * ld + idx];
      a0 += cas[int64_t(k) * nseg] * v0;
      d0 += cds[int64_t(k) * nseg] * v0;
    }
  } else {
    for (int k = 0; k < j; ++k) {
      const double v0 = V[k * ld + idx];
      a0 += ca[int64_t(k) * nseg + seg] * v0;
      d0 += cd[int64_t(k) * nseg + seg] * v0;
    }
  }
  if (!ok) return;
  const double u = V[j * ld + idx];
  const double s1 = sc[seg], s2 = sc[nseg + seg], s3 = sc[2 * nseg + seg];
  // masked segments (all coefficients zero) become exact zeros
  V[j * ld + idx] = s1 == 0.0 ? 0.0 : s1 * u - ((a0 + a1) + (a2 + a3));
  const double un = s2 == 0.0 ? 0.0 : s2 * z[idx] + s3 * u - ((d0 + d1) + (d2 + d3));
  V[(j + 1) * ld + idx] = un;
  if (u2) u2[idx] = un;   // second copy of u_{j+1} (the captured apply's input vector)
}

// out[c * nseg + seg] = sum over the chunks of (column c, segment seg)
__global__ __launch_bounds__(64) void dots_final_kernel(const double* __restrict__ partial, int nblk,
                                                        double* __restrict__ out, int nseg,
                                                        const int32_t* __restrict__ skip) {
  const int c = blockIdx.x;
  if (skip && skip[c % nseg]) return;   // segment out of this cycle: no partial sums to add
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) acc += partial[int64_t(c) * nblk + b];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) out[c] = acc;
}

// w += sign * V h with one coefficient vector per segment: h[c * nseg + seg]
__global__ void gemv_sub_kernel(const double* __restrict__ V, int64_t ld, int ncols_all,
                                const double* __restrict__ hh, double* __restrict__ w, int64_t n,
                                int nseg, double sign, const int32_t* __restrict__ ncol_seg) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n * nseg) return;
  const int seg = (int)(i / n);
  const int ncols = ncol_seg ? min(ncols_all, ncol_seg[seg]) : ncols_all;
  if (ncols <= 0) return;
  const double* h = hh + seg;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int c = 0;
  for (; c + 3 < ncols; c += 4) {
    a0 += V[c * ld + i] * h[int64_t(c) * nseg];
    a1 += V[(c + 1) * ld + i] * h[int64_t(c + 1) * nseg];
    a2 += V[(c + 2) * ld + i] * h[int64_t(c + 2) * nseg];
    a3 += V[(c + 3) * ld + i] * h[int64_t(c + 3) * nseg];
  }
  for (; c < ncols; ++c) a0 += V[c * ld + i] * h[int64_t(c) * nseg];
  w[i] += sign * ((a0 + a1) + (a2 + a3));
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y,
                             int64_t n) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

__global__ void scale_copy_kernel(double a, const double* __restrict__ x, double* __restrict__ y,
                                  int64_t n) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// y = alpha[seg] x per segment of length n
__global__ void seg_scale_copy_kernel(const double* __restrict__ alpha, const double* __restrict__ x,
                                      double* __restrict__ y, int64_t n, int nseg) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n * nseg) {
    const double a = alpha[i / n];
    y[i] = a == 0.0 ? 0.0 : a * x[i];   // masked segments become exact zeros
  }
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_set_kappa(MacroInfo* info, const double* kappa, int64_t n, int32_t* bad,
                            hipStream_t s) {
  hipLaunchKernelGGL(set_kappa_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, info, kappa, n,
                     bad);
  return hipGetLastError();
}

hipError_t launch_assemble(void* fac, int precision, const MacroInfo* info, const int32_t*,
                           int64_t n, const double* tmpl, const Templates& T, double tau,
                           hipStream_t s) {
  int maxN = 0;
  for (int r = 0; r <= kMaxLevel; ++r)
    if (T.lev[r].present) maxN = maxN > T.lev[r].N ? maxN : T.lev[r].N;
  dim3 grid((unsigned)n, (unsigned)((maxN + 7) / 8));
  if (precision == 1)
    hipLaunchKernelGGL(assemble_kernel<float>, grid, dim3(256), 0, s, (float*)fac, info, tmpl, T,
                       tau);
  else
    hipLaunchKernelGGL(assemble_kernel<double>, grid, dim3(256), 0, s, (double*)fac, info, tmpl, T,
                       tau);
  return hipGetLastError();
}

template <typename T>
static hipError_t lu_class(T* fac, const MacroInfo* info, const int32_t* order, const SizeClass& c,
                           int32_t* perm, int32_t* status, char* scratch, size_t scratch_bytes,
                           hipStream_t s) {
  const int v = c.lu_var ? c.lu_var : default_lu_variant(c.N);
  if (v == LU_SPLIT)
    return lu_split_class(fac, info, order, c, perm, status, scratch, scratch_bytes, s);
  if (v >= LU_BLOCKED) return lu_blocked_class(v, fac, info, order, c, perm, status, s);
  const dim3 g((unsigned)c.count);
  if (c.N <= 256)
    hipLaunchKernelGGL((lu_kernel<T, 256, 1, 16>), g, dim3(256), 0, s, fac, info, order, c.start, perm, status);
  else if (c.N <= 1024)
    hipLaunchKernelGGL((lu_kernel<T, 256, 4, 16>), g, dim3(256), 0, s, fac, info, order, c.start, perm, status);
  else if (c.N <= 4096)
    hipLaunchKernelGGL((lu_kernel<T, 1024, 4, 8>), g, dim3(1024), 0, s, fac, info, order, c.start, perm, status);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_lu(void* fac, int precision, const MacroInfo* info, const int32_t* order,
                     const SizeClass* classes, int n_classes, int32_t* perm, int32_t* status,
                     char* scratch, size_t scratch_bytes, hipStream_t s) {
  for (int c = 0; c < n_classes; ++c) {
    hipError_t e = precision == 1
                       ? lu_class((float*)fac, info, order, classes[c], perm, status, scratch,
                                  scratch_bytes, s)
                       : lu_class((double*)fac, info, order, classes[c], perm, status, scratch,
                                  scratch_bytes, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_dirichlet(const BndFaceInfo* bf, int64_t nbf, const double* tmpl,
                            const Templates& T, const double* g, double* lamD, hipStream_t s) {
  hipLaunchKernelGGL(dirichlet_kernel, dim3((unsigned)nbf), dim3(64), 0, s, bf, tmpl, T, g, lamD);
  return hipGetLastError();
}

static int max_present_N(const Templates& T) {
  int maxN = 0;
  for (int r = 0; r <= kMaxLevel; ++r)
    if (T.lev[r].present && T.lev[r].N > maxN) maxN = T.lev[r].N;
  return maxN;
}

hipError_t launch_local_rhs(const MacroInfo* info, int64_t n, const BndFaceInfo* bf,
                            const double* tmpl, const Templates& T, const double* f,
                            const double* lamD, double tau, double* R,
                            hipStream_t s) {
  int maxP = 0;
  for (int r = 0; r <= kMaxLevel; ++r)
    if (T.lev[r].present && T.lev[r].P > maxP) maxP = T.lev[r].P;
  size_t lds = size_t(max_present_N(T) + 9 * maxP) * sizeof(double);
  hipLaunchKernelGGL(local_rhs_kernel, dim3((unsigned)n), dim3(64), lds, s, info, bf, tmpl, T, f,
                     lamD, tau, R);
  return hipGetLastError();
}

// instantiated in solve_nq_*.hip
#define MS_DECL(T_, Q_)                                                                        \
  extern template void macro_solve_launch<T_, Q_>(int, const void*, const MacroInfo*,          \
                                                  const int32_t*, int64_t, int64_t,             \
                                                  size_t, const int32_t*, const double*,        \
                                                  const Templates&, const int32_t*, double,      \
                                                  const double*, const double*, double*,        \
                                                  double*, hipStream_t);
MS_DECL(bf16_t, 1) MS_DECL(bf16_t, 2) MS_DECL(bf16_t, 3) MS_DECL(bf16_t, 5) MS_DECL(bf16_t, 8)
MS_DECL(bf16_t, 16)
#define MS_DECL2(Q_) MS_DECL(double, Q_) MS_DECL(float, Q_)
MS_DECL2(1) MS_DECL2(2) MS_DECL2(3) MS_DECL2(5) MS_DECL2(8) MS_DECL2(16) MS_DECL2(27)
MS_DECL2(58)
#undef MS_DECL2
#undef MS_DECL
#define MST_DECL(Q_)                                                                           \
  extern template void macro_solve_t_launch<Q_>(int, const void*, const MacroInfo*,            \
                                                const int32_t*, int64_t, int64_t,               \
                                                size_t, const int32_t*, const double*,          \
                                                const Templates&, const int32_t*, double,        \
                                                const double*, const double*, double*, double*, \
                                                hipStream_t);
MST_DECL(1) MST_DECL(2) MST_DECL(3) MST_DECL(5) MST_DECL(8) MST_DECL(16) MST_DECL(27) MST_DECL(58)
#undef MST_DECL

static hipError_t macro_solve_t_dispatch(int nq, int mode, const void* fac, const MacroInfo* info,
                                         const int32_t* order, int64_t base, int64_t n, size_t lds,
                                         const int32_t* perm, const double* tmpl,
                                         const Templates& Tp, const int32_t* skip, double tau,
                                         const double* mu, const double* xin, double* yout,
                                         double* slots, hipStream_t s) {
#define MST_CASE(Q_)                                                                          \
  if (nq <= Q_) {                                                                             \
    macro_solve_t_launch<Q_>(mode, fac, info, order, base, n, lds, perm, tmpl, Tp, skip,      \
                             tau, mu, xin, yout, slots, s);                                   \
    return hipGetLastError();                                                                 \
  }
  MST_CASE(1) MST_CASE(2) MST_CASE(3) MST_CASE(5) MST_CASE(8) MST_CASE(16) MST_CASE(27) MST_CASE(58)
#undef MST_CASE
  return hipErrorInvalidValue;
}

#define MSO_DECL(T_, W_, LG_)                                                                 \
  extern template void macro_solve_launch<T_, 16, W_, LG_>(int, const void*, const MacroInfo*,   \
                                                           const int32_t*, int64_t, int64_t,     \
                                                           size_t, const int32_t*, const double*,\
                                                           const Templates&, const int32_t*,     \
                                                           double, const double*, const double*, \
                                                           double*, double*, hipStream_t);
MSO_DECL(double, 6, 8) MSO_DECL(double, 5, 8) MSO_DECL(double, 5, 12) MSO_DECL(double, 4, 16)
MSO_DECL(float, 6, 8) MSO_DECL(float, 5, 8) MSO_DECL(float, 5, 12) MSO_DECL(float, 4, 16)
#undef MSO_DECL

#define MSW_DECL(T_, Q_, W_)                                                                  \
  extern template void macro_solve_mw_launch<T_, Q_, W_>(int, const void*, const MacroInfo*,  \
                                                     const int32_t*, int64_t, int64_t, size_t,\
                                                     const int32_t*, const double*,           \
                                                     const Templates&, const int32_t*, double, \
                                                     const double*, const double*, double*,   \
                                                     double*, hipStream_t);
MSW_DECL(double, 27, 4) MSW_DECL(float, 27, 4) MSW_DECL(double, 58, 4) MSW_DECL(float, 58, 4)
MSW_DECL(double, 27, 8) MSW_DECL(float, 27, 8) MSW_DECL(double, 58, 8) MSW_DECL(float, 58, 8)
MSW_DECL(double, 16, 4) MSW_DECL(float, 16, 4)
#undef MSW_DECL

template <typename T>
static hipError_t macro_solve_dispatch(int variant, int nq, int mode, const void* fac,
                                       const MacroInfo* info, const int32_t* order, int64_t base,
                                       int64_t n, size_t lds, const int32_t* perm,
                                       const double* tmpl, const Templates& Tp,
                                       const int32_t* skip, double tau, const double* lam,
                                       const double* xin, double* yout, double* slots,
                                       hipStream_t s) {
  if (variant == SOLVE_WAVE) {
#define MS_CASE(Q_)                                                                           \
  if (nq <= Q_) {                                                                             \
    macro_solve_launch<T, Q_>(mode, fac, info, order, base, n, lds, perm, tmpl, Tp, skip,     \
                              tau, lam, xin, yout, slots, s);                                 \
    return hipGetLastError();                                                                 \
  }
    MS_CASE(1) MS_CASE(2) MS_CASE(3) MS_CASE(5) MS_CASE(8) MS_CASE(16) MS_CASE(27) MS_CASE(58)
#undef MS_CASE
    return hipErrorInvalidValue;
  }
  if (variant >= SOLVE_WAVE6 && variant <= SOLVE_WAVE4_LG16 && nq > 8 && nq <= 16) {
#define MO_CASE(V_, W_, LG_)                                                                  \
  if (variant == V_) {                                                                        \
    macro_solve_launch<T, 16, W_, LG_>(mode, fac, info, order, base, n, lds, perm, tmpl, Tp,  \
                                       skip, tau, lam, xin, yout, slots, s);                  \
    return hipGetLastError();                                                                 \
  }
    MO_CASE(SOLVE_WAVE6, 6, 8) MO_CASE(SOLVE_WAVE5, 5, 8) MO_CASE(SOLVE_WAVE5_LG12, 5, 12)
    MO_CASE(SOLVE_WAVE4_LG16, 4, 16)
#undef MO_CASE
  }
#define MW_CASE(Q_, W_)                                                                       \
  if (nq <= Q_) {                                                                             \
    macro_solve_mw_launch<T, Q_, W_>(mode, fac, info, order, base, n, lds, perm, tmpl, Tp,    \
                                     skip, tau, lam, xin, yout, slots, s);                    \
    return hipGetLastError();                                                                 \
  }
  if (variant == SOLVE_MW4) { MW_CASE(16, 4) MW_CASE(27, 4) MW_CASE(58, 4) }
  if (variant == SOLVE_MW8) { MW_CASE(27, 8) MW_CASE(58, 8) }
#undef MW_CASE
  return hipErrorInvalidValue;
}

// BF16 factors: one wavefront per macro, N_K <= 1024
static hipError_t macro_solve_dispatch_bf16(int variant, int nq, int mode, const void* fac,
                                            const MacroInfo* info, const int32_t* order,
                                            int64_t base, int64_t n, size_t lds,
                                            const int32_t* perm, const double* tmpl,
                                            const Templates& Tp, const int32_t* skip, double tau,
                                            const double* lam, const double* xin, double* yout,
                                            double* slots, hipStream_t s) {
  if (variant != SOLVE_WAVE) return hipErrorInvalidValue;
#define MB_CASE(Q_)                                                                           \
  if (nq <= Q_) {                                                                             \
    macro_solve_launch<bf16_t, Q_>(mode, fac, info, order, base, n, lds, perm, tmpl, Tp, skip,\
                                   tau, lam, xin, yout, slots, s);                            \
    return hipGetLastError();                                                                 \
  }
  MB_CASE(1) MB_CASE(2) MB_CASE(3) MB_CASE(5) MB_CASE(8) MB_CASE(16)
#undef MB_CASE
  return hipErrorInvalidValue;
}

// FP32 factors -> BF16 storage, rounding to nearest (ties to even).  A
// grid-stride loop: the factor arrays exceed the 2^32 work-items one
// dispatch can address.
__global__ void to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += stride) {
    const uint32_t b = __float_as_uint(src[i]);
    dst[i] = (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
  }
}

hipError_t launch_to_bf16(const float* src, void* dst, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, (uint16_t*)dst,
                     n);
  return hipGetLastError();
}

int default_solve_variant(int N) {
  if (N > 16 * 64) return SOLVE_MW4;
  return N > 8 * 64 ? SOLVE_WAVE4_LG16 : SOLVE_WAVE;
}
bool solve_variant_ok(int v, int N) {
  if (N > 58 * 64) return false;
  if (v == SOLVE_WAVE || v == SOLVE_MW4) return true;
  if (v >= SOLVE_WAVE6 && v <= SOLVE_WAVE4_LG16) return N > 8 * 64 && N <= 16 * 64;
  return v == SOLVE_MW8 && N > 16 * 64;
}
int default_lu_variant(int N) { return N <= 256 ? LU_PANEL : LU_SPLIT; }
bool lu_variant_ok(int v, int N) { return N <= 4096 && v >= LU_PANEL && v <= LU_SPLIT; }

// One launch per size class, each with the register-block count of its
// local size (NQ = ceil(N/64)) and LDS for its boundary vectors.
hipError_t launch_macro_solve(int mode, int transpose, const void* fac, int precision,
                              const MacroInfo* info, const int32_t* order,
                              const SizeClass* classes, int n_classes, const int32_t* perm,
                              const double* tmpl, const Templates& T, const int32_t* skip,
                              double tau, const double* lam, const double* xin, double* yout,
                              double* slots, hipStream_t s) {
  if (transpose && precision != 0) return hipErrorInvalidValue;
  for (int c = 0; c < n_classes; ++c) {
    const SizeClass& sc = classes[c];
    const size_t lds = size_t(18) * sc.P * sizeof(double);
    const int nq = (sc.N + 63) / 64;
    hipError_t e;
    // BF16 factors have the one-wavefront kernel only
    const int v = sc.solve_var ? sc.solve_var
                               : (precision == 2 ? SOLVE_WAVE : default_solve_variant(sc.N));
    if (transpose)
      e = macro_solve_t_dispatch(nq, mode, fac, info, order, sc.start, sc.count, lds, perm, tmpl, T,
                                 skip, tau, lam, xin, yout, slots, s);
    else if (precision == 2)
      e = macro_solve_dispatch_bf16(v, nq, mode, fac, info, order, sc.start, sc.count, lds, perm,
                                    tmpl, T, skip, tau, lam, xin, yout, slots, s);
    else if (precision == 1)
      e = macro_solve_dispatch<float>(v, nq, mode, fac, info, order, sc.start, sc.count, lds, perm,
                                      tmpl, T, skip, tau, lam, xin, yout, slots, s);
    else
      e = macro_solve_dispatch<double>(v, nq, mode, fac, info, order, sc.start, sc.count, lds,
                                       perm, tmpl, T, skip, tau, lam, xin, yout, slots, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_face_combine(int mode, const FaceInfo* fi, int64_t nf, const double* tmpl,
                               const Templates& T, double tau, const double* lam,
                               const double* slots, double* out, hipStream_t s,
                               const int32_t* skip) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(face_combine_kernel, dim3((unsigned)nf), dim3(64), 0, s, mode, fi, tmpl, T,
                     tau, lam, slots, out, skip);
  return hipGetLastError();
}

hipError_t launch_face_combine_many(int precondition, const FaceInfo* fi, int64_t nf,
                                    const double* tmpl, const Templates& T, double tau,
                                    int n_rhs, const double* lam, int64_t ld_lam,
                                    const double* slots, int64_t ld_slots, double* out,
                                    hipStream_t s) {
  if (nf == 0 || n_rhs == 0) return hipSuccess;
  if (n_rhs > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(face_combine_many_kernel, dim3((unsigned)nf, (unsigned)n_rhs), dim3(64), 0,
                     s, precondition, fi, tmpl, T, tau, lam, ld_lam, slots, ld_slots, out);
  return hipGetLastError();
}

hipError_t launch_extract_matrix(const MacroInfo* info, int64_t e, const double* tmpl,
                                 const Templates& T, double tau, double* dst, hipStream_t s) {
  // the row count is the macro's N; launch max_N rows and let extra rows exit
  int maxN = max_present_N(T);
  hipLaunchKernelGGL(extract_kernel, dim3((unsigned)maxN), dim3(256), 0, s, info, e, tmpl, T,
                     tau, dst);
  return hipGetLastError();
}

static int max_present_P(const Templates& T) {
  int maxP = 0;
  for (int r = 0; r <= kMaxLevel; ++r)
    if (T.lev[r].present && T.lev[r].P > maxP) maxP = T.lev[r].P;
  return maxP;
}

hipError_t launch_local_residual(const MacroInfo* info, int64_t n, const double* tmpl,
                                 const Templates& T, double tau, const double* R, const double* U, const double* lam,
                                 double* out, hipStream_t s) {
  size_t lds = size_t(max_present_N(T) + 9 * max_present_P(T)) * sizeof(double);
  hipLaunchKernelGGL(local_residual_kernel, dim3((unsigned)n), dim3(256), lds, s, info, tmpl, T,
                     tau, R, U, lam, out);
  return hipGetLastError();
}

hipError_t launch_boundary_C(const MacroInfo* info, int64_t n, const double* tmpl,
                             const Templates& T, double tau, const double* U, double* slots,
                             hipStream_t s) {
  size_t lds = size_t(9 * max_present_P(T)) * sizeof(double);
  hipLaunchKernelGGL(boundary_C_kernel, dim3((unsigned)n), dim3(64), lds, s, info, tmpl, T, tau, U,
                     slots);
  return hipGetLastError();
}

hipError_t launch_adjoint_contract(const MacroInfo* info, int64_t n, const BndFaceInfo* bf,
                                   const double* tmpl, const Templates& T, const double* U,
                                   const double* Psi, const double* lam, const double* psi_lam,
                                   const double* lamD, double* dkappa, double* dbeta_part,
                                   double* dbeta, hipStream_t s) {
  size_t lds = size_t(2 * max_present_N(T)) * sizeof(double);
  hipLaunchKernelGGL(adjoint_contract_kernel, dim3((unsigned)n), dim3(256), lds, s, info, bf, tmpl,
                     T, U, Psi, lam, psi_lam, lamD, dkappa, dbeta_part);
  hipLaunchKernelGGL(strided_sum_kernel, dim3(2), dim3(256), 0, s, dbeta_part, n, 2, dbeta);
  return hipGetLastError();
}

hipError_t launch_mass(const MacroInfo* info, int64_t n, const double* tmpl, const Templates& T,
                       const double* v, double* out, hipStream_t s) {
  size_t lds = size_t(max_present_N(T)) * sizeof(double);
  hipLaunchKernelGGL(mass_kernel, dim3((unsigned)n), dim3(256), lds, s, info, tmpl, T, v, out);
  return hipGetLastError();
}

hipError_t launch_dots(const double* V, int64_t ld, int ncols, const double* w, int64_t n,
                       double* partial, int nblk, double* out, hipStream_t s, int nseg,
                       const int32_t* skip) {
  hipLaunchKernelGGL(dots_partial_kernel, dim3(nblk * nseg, (ncols + 3) / 4), dim3(256), 0, s, V,
                     ld, ncols, w, n, partial, skip);
  hipLaunchKernelGGL(dots_final_kernel, dim3(ncols * nseg), dim3(64), 0, s, partial, nblk, out,
                     nseg, skip);
  return hipGetLastError();
}

hipError_t launch_gemv_sub(const double* V, int64_t ld, int ncols, const double* h, double* w,
                           int64_t n, double sign, hipStream_t s, int nseg,
                           const int32_t* ncol_seg) {
  if (ncols == 0) return hipSuccess;
  hipLaunchKernelGGL(gemv_sub_kernel, dim3(blocks_for(n * nseg, 256)), dim3(256), 0, s, V, ld,
                     ncols, h, w, n, nseg, sign, ncol_seg);
  return hipGetLastError();
}

hipError_t launch_dots2_partial(const double* V, int64_t ld, int ncols, const double* x,
                                const double* y, int64_t n, double* partial, int nblk,
                                hipStream_t s, int nseg, const int32_t* skip) {
  // eight columns per workgroup either way; past 48 columns the workgroup
  // shares x and y across its eight (measured: 18.2 against 15.9 us per call
  // at 20 columns on 304,000 rows, faster on the long bases of GMRES(1000))
  if (ncols > 48)
    hipLaunchKernelGGL(dots2_partial_kernel, dim3(nblk * nseg, (ncols + 7) / 8), dim3(256), 0, s,
                       V, ld, ncols, x, y, n, partial, skip);
  else
    hipLaunchKernelGGL(dots2_partial_narrow_kernel, dim3(nblk * nseg, (ncols + 7) / 8), dim3(256),
                       0, s, V, ld, ncols, x, y, n, partial, skip);
  return hipGetLastError();
}

hipError_t launch_dots2(const double* V, int64_t ld, int ncols, const double* x, const double* y,
                        int64_t n, double* partial, int nblk, double* out, hipStream_t s,
                        int nseg, const int32_t* skip) {
  const hipError_t e = launch_dots2_partial(V, ld, ncols, x, y, n, partial, nblk, s, nseg, skip);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dots_final_kernel, dim3(2 * ncols * nseg), dim3(64), 0, s, partial, nblk, out,
                     nseg, skip);
  return hipGetLastError();
}

hipError_t launch_hbar_gemv(const double* Hb, int64_t ld, int nseg, int kmax, int rows,
                            const double* pq, double* out, hipStream_t s) {
  const int64_t tot = int64_t(rows) * nseg;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(hbar_gemv_kernel, dim3(blocks_for(tot, 64)), dim3(512), 0, s, Hb, ld, nseg,
                     kmax, rows, pq, out);
  return hipGetLastError();
}

hipError_t launch_dual_update(double* V, int64_t ld, int j, int64_t n, int nseg, const double* ca,
                              const double* cd, const double* sc, const double* z, double* u2,
                              hipStream_t s, const int32_t* skip) {
  hipLaunchKernelGGL(dual_update_kernel, dim3(blocks_for(n * nseg, 256)), dim3(256), 0, s, V, ld,
                     j, n, nseg, ca, cd, sc, z, u2, skip);
  return hipGetLastError();
}

hipError_t launch_seg_scale_copy(const double* alpha, const double* x, double* y, int64_t n, int nseg,
                                 hipStream_t s) {
  hipLaunchKernelGGL(seg_scale_copy_kernel, dim3(blocks_for(n * nseg, 256)), dim3(256), 0, s, alpha,
                     x, y, n, nseg);
  return hipGetLastError();
}

hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t launch_scale_copy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, x, y, n);
  return hipGetLastError();
}

}  // namespace mhdg
