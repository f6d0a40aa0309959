// Device side of the restarted GMRES on D^-1 S lam = D^-1 f^ (section 6.1:
// GMRES on the condensed trace system, preconditioned with the inverse of the
// face blocks D_F).  The host driver in host.cpp launches, per restart cycle,
//   apply -> dual products -> Hessenberg correction -> gm_step -> dual update
// for every Arnoldi column, then gm_step in its closing mode, gm_lsq, the
// update x += V y and the residual of the next cycle with gm_start.  The
// scalar recurrences that a host loop would otherwise run between kernels
// (second projection and norm of the new direction, finishing the Hessenberg
// column, Givens rotations, the residual estimate, the coefficients of the
// next update, the triangular solve) run here, one wavefront per segment
// (coefficient instance), so a cycle needs no host round trip and can be
// captured in hipGraphs.
//
// The Arnoldi process is Gram-Schmidt with delayed reorthogonalisation: the
// direction u_j of column j is once orthogonalised when its apply is taken;
// its second projection and norm come from the same pass of inner products
// that also gives the first projection of z = D^-1 S u_j.  With
//   p_c = <q_c, u_j> (c < j), p_j = <u_j, u_j>, c_c = <q_c, z>, c_j = <u_j, z>,
//   a = p[0..j), beta = sqrt(p_j - a.a)
// column j-1 of the Hessenberg matrix is [h_{j-1} + a; beta], q_j =
// (u_j - Q a) / beta, and the next direction is
//   u_{j+1} = (z - Q_j [c; (c_j - a.c) / beta]) / beta
// (one fused pass over V, dual_update_kernel), with h_j = ([c_0..c_{j-1},
// (c_j - a.c) / beta] - Hbar a) / beta stored for the next column.
#include "internal.h"

namespace mhdg {

__device__ __forceinline__ double gm_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Residual of a cycle start.  nrm[q] = ||D^-1 r||^2 (the preconditioned
// residual), nrm_true[q] = ||r||^2 and fref[q] = ||f^|| when the stopping
// test is on the unpreconditioned residual (else null).  Sets per segment
// done / active / skip, the first Krylov coefficient g_0 = beta, alpha (1 to
// take the residual as u_0, 0 to zero it) and the target of the in-cycle
// residual estimate; any[0] = 1 if some segment iterates in this cycle.
__global__ __launch_bounds__(256) void gm_start_kernel(GmDev d, int R) {
  const double rtol = d.prm[0];
  const int max_iter = (int)d.prm[1];
  const int hld = R + 1;
  int act_any = 0;
  for (int q = threadIdx.x; q < d.ns; q += blockDim.x) {
    double* gq = d.g + int64_t(q) * hld;
    d.jc[q] = 0;
    if (d.done[q]) {
      d.active[q] = 0;
      d.skip[q] = 1;
      d.alpha[q] = 0.0;
      gq[0] = 0.0;
      continue;
    }
    const double beta = sqrt(d.nrm[q]);
    const double br = d.bref[q];
    if (!(fabs(beta) < __builtin_huge_val()) || !(fabs(br) < __builtin_huge_val())) {
      d.flag[q] = 1;   // non-finite residual: the host reports the segment as failed
      d.done[q] = 1;
      d.active[q] = 0;
      d.skip[q] = 1;
      d.alpha[q] = 0.0;
      gq[0] = 0.0;
      continue;
    }
    const double rel = beta / br;
    d.rel[q] = rel;
    bool conv;
    double tgt = rtol;
    if (d.nrm_true) {
      const double rt = sqrt(d.nrm_true[q]), fr = d.fref[q];
      d.rel_true[q] = fr > 0.0 ? rt / fr : 0.0;
      conv = fr == 0.0 || rt <= rtol * fr || beta == 0.0;
      // the estimate tracks the preconditioned residual: scale the target by
      // the ratio of the two norms at the cycle start
      if (rt > 0.0) tgt = rtol * fr * beta / (rt * br);
    } else {
      conv = rel <= rtol || beta == 0.0;
    }
    if (conv) d.done[q] = 1;
    const int act = !conv && d.iters[q] < max_iter;
    d.active[q] = act;
    d.skip[q] = !act;
    d.alpha[q] = act ? 1.0 : 0.0;
    d.tgt[q] = tgt;
    gq[0] = act ? beta : 0.0;
    act_any |= act;
  }
  act_any = __syncthreads_or(act_any);
  if (threadIdx.x == 0) d.any[0] = act_any;
}

// Step j of the cycle, one wavefront per segment.  Reads the dual products
// p, c of dots2 (pq[(2c) ns + q], pq[(2c + 1) ns + q]) and Hbar a (pq[2 (j +
// 1) ns + i ns + q], columns < j - 1, for j >= 2).  In the closing mode
// (last) only the single products p of the projection pass are present, in
// hy[c ns + q], and no next direction is prepared.  LDS: the finished column
// and the rotations, 3 (R + 2) doubles.  The step runs on one wavefront
// (lanes 0..63 of its workgroup), so its LDS hand-offs need only a
// wavefront-scope fence.
__device__ __forceinline__ void gm_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ void gm_step_wave(const GmDev& d, int R, int j, int last, double* lds, int* act_sp) {
  int& act_s = *act_sp;
  double* col = lds;                 // unrotated column j-1, rows 0..j
  double* csl = lds + (R + 2);       // rotations 0..j-2
  double* snl = csl + (R + 2);
  const int q = blockIdx.x, lane = threadIdx.x & 63, ns = d.ns;
  const int hld = R + 1;
  const int max_iter = (int)d.prm[1];
  double* ca = d.coef;
  double* cd = d.coef + int64_t(j) * ns;
  double* sc = d.coef + 2 * int64_t(j) * ns;
  if (!d.active[q]) {
    if (j >= 1)
      for (int i = lane; i <= j; i += 64) d.Hb[(int64_t(j - 1) * hld + i) * ns + q] = 0.0;
    if (!last) {
      for (int c = lane; c < j; c += 64) {
        ca[int64_t(c) * ns + q] = 0.0;
        cd[int64_t(c) * ns + q] = 0.0;
      }
      if (lane < 3) sc[int64_t(lane) * ns + q] = 0.0;
    }
    return;
  }
  if (!last && lane == 0) d.napp[q] += 1;   // the apply of u_j ran for this segment
  auto P = [&](int c) -> double {
    return last ? d.hy[int64_t(c) * ns + q] : d.pq[int64_t(2 * c) * ns + q];
  };
  auto C = [&](int c) -> double { return d.pq[int64_t(2 * c + 1) * ns + q]; };
  // second projection of u_j and its norm
  double aa = 0.0;
  for (int c = lane; c < j; c += 64) {
    const double a = P(c);
    aa += a * a;
  }
  aa = gm_wave_sum(aa);
  const double om = P(j);
  const double bt = sqrt(fmax(om - aa, 0.0));
  double* hp = d.hprev + int64_t(q) * hld;
  bool act = true;
  if (j >= 1) {
    const int jj = j - 1;
    for (int i = lane; i < j; i += 64) col[i] = hp[i] + P(i);
    for (int i = lane; i < jj; i += 64) {
      csl[i] = d.cs[int64_t(q) * R + i];
      snl[i] = d.sn[int64_t(q) * R + i];
    }
    if (lane == 0) col[j] = bt;
    gm_wave_sync();
    for (int i = lane; i <= j; i += 64) d.Hb[(int64_t(jj) * hld + i) * ns + q] = col[i];
    double* Hc = d.H + (int64_t(q) * R + jj) * hld;   // rotated column jj
    if (lane == 0) {
      // earlier rotations on the new column, then the one that zeroes row jj + 1
      double a = col[0];
      for (int i = 0; i < jj; ++i) {
        const double b = col[i + 1], c_ = csl[i], s_ = snl[i];
        Hc[i] = c_ * a + s_ * b;
        a = -s_ * a + c_ * b;
      }
      const double b = col[jj + 1];
      const double rr = hypot(a, b);
      const double c_ = rr == 0.0 ? 1.0 : a / rr;
      const double s_ = rr == 0.0 ? 0.0 : b / rr;
      Hc[jj] = rr;
      Hc[jj + 1] = 0.0;
      d.cs[int64_t(q) * R + jj] = c_;
      d.sn[int64_t(q) * R + jj] = s_;
      double* gq = d.g + int64_t(q) * hld;
      const double gj = gq[jj];
      gq[jj + 1] = -s_ * gj;
      gq[jj] = c_ * gj;
      const double est = fabs(gq[jj + 1]) / d.bref[q];
      d.est[q] = est;
      d.jc[q] = j;
      const int it = d.iters[q] + 1;
      d.iters[q] = it;
      if (est <= d.tgt[q] || bt == 0.0 || it >= max_iter) {
        d.active[q] = 0;
        d.skip[q] = 1;
      }
    }
    if (lane == 0) act_s = d.active[q];
    gm_wave_sync();
    act = act_s != 0;
  } else if (bt == 0.0) {
    if (lane == 0) {
      d.active[q] = 0;
      d.skip[q] = 1;
    }
    act = false;
  }
  if (last) return;
  if (!act) {
    for (int c = lane; c < j; c += 64) {
      ca[int64_t(c) * ns + q] = 0.0;
      cd[int64_t(c) * ns + q] = 0.0;
    }
    if (lane < 3) sc[int64_t(lane) * ns + q] = 0.0;
    return;
  }
  // coefficients of q_j and u_{j+1}, and h_j for the next column
  double ab = 0.0;
  for (int c = lane; c < j; c += 64) ab += P(c) * C(c);
  ab = gm_wave_sum(ab);
  const double cj = (C(j) - ab) / bt;
  const double aj1 = j >= 1 ? P(j - 1) : 0.0;
  const double* hyv = d.pq + 2 * int64_t(j + 1) * ns;
  for (int i = lane; i <= j; i += 64) {
    double hba = (j >= 2 && i < j) ? hyv[int64_t(i) * ns + q] : 0.0;
    if (j >= 1) hba += aj1 * col[i];
    const double ci = i < j ? C(i) : cj;
    hp[i] = (ci - hba) / bt;
  }
  for (int c = lane; c < j; c += 64) {
    const double ac = P(c);
    ca[int64_t(c) * ns + q] = ac / bt;
    cd[int64_t(c) * ns + q] = (C(c) - (cj / bt) * ac) / bt;
  }
  if (lane == 0) {
    sc[q] = 1.0 / bt;
    sc[ns + q] = 1.0 / bt;
    sc[2 * int64_t(ns) + q] = -cj / (bt * bt);
  }
}


__global__ __launch_bounds__(64) void gm_step_kernel(GmDev d, int R, int j, int last) {
  extern __shared__ double lds[];
  __shared__ int act_s;
  gm_step_wave(d, R, j, last, lds, &act_s);
}

// Column j's scalar work in one launch per segment, for j + 1 <= kGmColumnMax:
// the sums of the chunk partials of dots2 (the 2 (j + 1) dual products), the
// Hbar correction (j >= 2), then the step on wavefront 0.  Every sum keeps the
// order of the separate kernels (dots_final: chunks strided over the 64 lanes,
// then the wavefront sum; hbar_gemv: k strided by 8 in eight groups, the groups
// added in order), so the results equal the three-launch sequence bit for bit.
// 16 wavefronts: four products per wavefront in flight, 128 rows x 8 groups of
// the correction.  LDS: the step's 3 (R + 2) doubles plus the group sums.
constexpr int kGmColWaves = 16;
__global__ __launch_bounds__(64 * kGmColWaves) void gm_column_kernel(GmDev d,
                                                                    const double* __restrict__ partial,
                                                                    int nblk, int R, int j) {
  extern __shared__ double lds[];
  __shared__ int act_s;
  __shared__ double red[8][128];
  const int q = blockIdx.x, ns = d.ns, tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int np = 2 * (j + 1);
  if (!d.skip[q]) {   // a skipped segment has no partial sums (as in dots_final)
    for (int c0 = 4 * wid; c0 < np; c0 += 4 * kGmColWaves) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int b = lane; b < nblk; b += 64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u < np ? c0 + u : np - 1;
          acc[u] += partial[(int64_t(c) * ns + q) * nblk + b];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double v = gm_wave_sum(acc[u]);
        if (lane == 0 && c0 + u < np) d.pq[int64_t(c0 + u) * ns + q] = v;
      }
    }
  }
  __syncthreads();
  if (j >= 2) {   // Hbar a over the finished columns k < j - 1, rows i < j
    const int hld = R + 1, kmax = j - 1;
    const int g = tid & 7, r = tid >> 3;
    double* out = d.pq + 2 * int64_t(j + 1) * ns;
    for (int i0 = 0; i0 < j; i0 += 128) {
      const int i = i0 + r;
      double acc = 0.0;
      if (i < j) {
        const int k0 = i > 0 ? i - 1 : 0;
        for (int kk = k0 + g; kk < kmax; kk += 8)
          acc += d.pq[int64_t(2 * kk) * ns + q] * d.Hb[(int64_t(kk) * hld + i) * ns + q];
      }
      red[g][r] = acc;
      __syncthreads();
      if (g == 0 && i < j) {
        double sum = 0.0;
#pragma unroll
        for (int g2 = 0; g2 < 8; ++g2) sum += red[g2][r];
        out[int64_t(i) * ns + q] = sum;
      }
      __syncthreads();
    }
  }
  if (wid != 0) return;
  gm_step_wave(d, R, j, 0, lds, &act_s);
}

// y = R^-1 g over the jc[q] finished columns of segment q (upper triangular,
// column-oriented back substitution; g is consumed), then skip[q] = done[q]
// for the residual apply of the next cycle start.
__global__ __launch_bounds__(64) void gm_lsq_kernel(GmDev d, int R) {
  __shared__ double yi_s;
  const int q = blockIdx.x, lane = threadIdx.x, ns = d.ns;
  const int hld = R + 1;
  const int jq = d.jc[q];
  double* gq = d.g + int64_t(q) * hld;
  const double* Hq = d.H + int64_t(q) * R * hld;
  for (int i = jq - 1; i >= 0; --i) {
    if (lane == 0) {
      const double yi = gq[i] / Hq[int64_t(i) * hld + i];
      d.y[int64_t(i) * ns + q] = yi;
      yi_s = yi;
    }
    __syncthreads();
    const double yi = yi_s;
    for (int k = lane; k < i; k += 64) gq[k] -= Hq[int64_t(i) * hld + k] * yi;
    __syncthreads();
  }
  if (lane == 0) d.skip[q] = d.done[q];
}

hipError_t launch_gm_start(const GmDev& d, int R, hipStream_t s) {
  hipLaunchKernelGGL(gm_start_kernel, dim3(1), dim3(256), 0, s, d, R);
  return hipGetLastError();
}

hipError_t launch_gm_step(const GmDev& d, int R, int j, int last, hipStream_t s) {
  const size_t lds = 3 * size_t(R + 2) * sizeof(double);
  hipLaunchKernelGGL(gm_step_kernel, dim3(d.ns), dim3(64), lds, s, d, R, j, last);
  return hipGetLastError();
}

hipError_t launch_gm_column(const GmDev& d, const double* partial, int nblk, int R, int j,
                            hipStream_t s) {
  if (j + 1 > kGmColumnMax) return hipErrorInvalidValue;
  const size_t lds = 3 * size_t(R + 2) * sizeof(double);
  hipLaunchKernelGGL(gm_column_kernel, dim3(d.ns), dim3(64 * kGmColWaves), lds, s, d, partial,
                     nblk, R, j);
  return hipGetLastError();
}

hipError_t launch_gm_lsq(const GmDev& d, int R, hipStream_t s) {
  hipLaunchKernelGGL(gm_lsq_kernel, dim3(d.ns), dim3(64), 0, s, d, R);
  return hipGetLastError();
}

}  // namespace mhdg
