// Host side of the macro-element HDG library: mesh setup (faces, levels,
// orientation, numbering), exact reference templates, workspace layout, the
// GMRES driver and the C ABI declared in include/mhdg.h.
#include "../../include/mhdg.h"
#include "internal.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace mhdg;

struct TracePlan;

struct mhdg_mesh {
  int32_t p = 1;
  int64_t n_vertices = 0, n_macro = 0;
  std::vector<double> xy;
  std::vector<int32_t> tri, level;
  // faces
  int64_t n_faces = 0, n_int = 0, n_bnd = 0;
  std::vector<MacroInfo> macros;
  std::vector<FaceInfo> faces;
  std::vector<BndFaceInfo> bfaces;
  std::vector<int32_t> order;     // macro processing order (largest local size first)
  std::vector<SizeClass> classes; // contiguous runs of equal local size in that order
  int64_t n_trace = 0, n_nodes = 0, n_local = 0, n_bnd_points = 0, n_slots = 0, n_lamD = 0;
  int32_t max_level = 0, max_N = 0;
  // Coefficient instances: the tables above describe n_inst disjoint copies
  // of one mesh (instance-major); `one` keeps the single-copy tables.
  struct One {
    int64_t n_macro, n_faces, n_int, n_bnd, n_trace, n_nodes, n_local, n_bnd_points, n_slots,
        n_lamD, fac_total;
    std::vector<MacroInfo> macros;
    std::vector<FaceInfo> faces;
    std::vector<BndFaceInfo> bfaces;
    std::vector<int32_t> order;
    std::vector<SizeClass> classes;
  } one;
  int32_t n_inst = 1;
  // templates
  Templates T{};
  std::vector<double> tmpl;       // blob (int tables stored bit-wise in doubles' space)
  QTemplates QT{};                // flux-eliminated form: offsets into qtmpl
  std::vector<double> qtmpl;      // built on first use of MHDG_QELIM
  // factor state
  bool factored = false, have_rhs = false;
  bool supg = false;               // SUPG inside the macros (mhdg_set_supg)
  // folded operators T_K (mhdg_fold_operator): valid until the next factor_local
  bool folded = false;
  int64_t* fold_toff = nullptr;   // device: element offset of T_K
  double* fold_T = nullptr;       // device: T_K column-major, L_K x L_K
  int fold_maxL = 0;              // largest L_K
  // assembled trace matrix (mhdg_assemble_trace_matrix): valid until the next
  // factor_local or fold
  bool assembled = false;
  const int32_t* tm_row_ptr = nullptr;    // device: block rows per interior face
  const TraceBlock* tm_blocks = nullptr;  // device: block table
  const double* tm_values = nullptr;      // device: block values of S
  const double* tm_pvalues = nullptr;     // device: block values of D^-1 S
  int64_t tm_n_blocks = 0, tm_n_values = 0;
  int tm_max_nF = 0;                      // largest interior face trace
  // host block plan of the assembled matrix: fixed by the mesh topology and the
  // instance count, so built once (cleared by set_instances)
  mutable std::shared_ptr<const TracePlan> tm_plan;
  // boundary-condensed blocks W_K (mhdg_condense_boundary): valid until the
  // next factor_local
  bool bcond = false;
  const int64_t* bc_off = nullptr;   // device: element offset of W_K
  const double* bc_W = nullptr;      // device: W_K column-major, 9P x 9P
  int bc_maxP = 0;
  int precision = MHDG_FP64;
  double tau = 1;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  FactorLayout L{};
  std::string err;
  // kernel timing (mhdg_profile)
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[6];
  // captured applies (every size class and instance, then the face combine)
  // keyed by their vector pointers and flags; valid until the next
  // factor_local / set_instances
  struct ApplyGraph {
    const double* lam;
    double* out;
    int32_t flags;
    const int32_t* skip;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<ApplyGraph> graphs;
  // captured GMRES cycles (gmres_device): the chunks of a cycle and the first
  // cycle start, keyed by the solve's vectors, restart, segments and flags
  struct GmKey {
    const double* V;
    const double* x;
    const double* b;
    const double* fh;
    int R, ns;
    int32_t flags;
    bool operator==(const GmKey& o) const {
      return V == o.V && x == o.x && b == o.b && fh == o.fh && R == o.R && ns == o.ns &&
             flags == o.flags;
    }
  };
  struct GmGraphs {
    GmKey key;
    std::vector<hipGraphExec_t> x;
  };
  std::vector<GmGraphs> gm_graphs;
  hipStream_t cap = nullptr;   // private stream the graphs are captured on
  // two events for the look-ahead of directly launched GMRES cycles
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  hipEvent_t* chunk_events() {
    for (auto& e : chunk_ev)
      if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return chunk_ev;
  }
  // page-locked host buffer for the small per-iteration GMRES transfers (kept
  // until the handle is destroyed; host memory only)
  double* pinned = nullptr;
  size_t pinned_n = 0;
  double* host_buffer(size_t n) {
    if (n > pinned_n) {
      if (pinned) (void)hipHostFree(pinned);
      pinned = nullptr;
      pinned_n = 0;
      if (hipHostMalloc((void**)&pinned, n * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return nullptr;
      pinned_n = n;
    }
    return pinned;
  }
  void drop_graphs() {
    for (auto& a : graphs) { (void)hipGraphExecDestroy(a.x); (void)hipGraphDestroy(a.g); }
    graphs.clear();
    for (auto& c : gm_graphs)
      for (auto x : c.x) (void)hipGraphExecDestroy(x);
    gm_graphs.clear();
  }
  ~mhdg_mesh() {
    for (auto& v : ev)
      for (auto& p : v) { hipEventDestroy(p.first); hipEventDestroy(p.second); }
    drop_graphs();
    for (auto e : chunk_ev)
      if (e) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    if (pinned) (void)hipHostFree(pinned);
  }
};

namespace {
// Brackets one launch with events when profiling is on.
struct ProfScope {
  mhdg_mesh* m;
  int k;
  hipStream_t s;
  hipEvent_t b = nullptr, e = nullptr;
  ProfScope(mhdg_mesh* m_, int k_, hipStream_t s_) : m(m_), k(k_), s(s_) {
    if (!m->prof) return;
    if (hipEventCreate(&b) != hipSuccess || hipEventCreate(&e) != hipSuccess) { b = e = nullptr; return; }
    (void)hipEventRecord(b, s);
  }
  ~ProfScope() {
    if (!b) return;
    (void)hipEventRecord(e, s);
    m->ev[k].push_back({b, e});
  }
};
}  // namespace

namespace {

mhdg_status fail(mhdg_mesh* m, mhdg_status s, const std::string& msg) {
  if (m) m->err = msg;
  return s;
}

#define HIP_TRY(m, call)                                                         \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(m, MHDG_ERR_HIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- small dense LA
// In-place inverse of an n x n row-major matrix by Gauss-Jordan with partial
// pivoting.  Used only for tiny Vandermonde and 1D mass matrices.
bool invert(std::vector<double>& a, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    if (a[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[c * n + k], a[piv * n + k]);
        std::swap(inv[c * n + k], inv[piv * n + k]);
      }
    double d = 1.0 / a[c * n + c];
    for (int k = 0; k < n; ++k) { a[c * n + k] *= d; inv[c * n + k] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { a[r * n + k] -= f * a[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
    }
  }
  a.swap(inv);
  return true;
}

// Gauss-Legendre nodes and weights on [0, 1] by Newton iteration on the
// Legendre polynomial from its three-term recurrence.
void gauss_legendre01(int k, std::vector<double>& t, std::vector<double>& w) {
  t.assign(k, 0.0);
  w.assign(k, 0.0);
  for (int i = 0; i < k; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (k + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int n = 2; n <= k; ++n) {
        double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
      }
      if (k == 1) { p1 = x; p0 = 1.0; }
      dp = k * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int n = 2; n <= k; ++n) {
      double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
      p0 = p1;
      p1 = p2;
    }
    if (k == 1) { p1 = x; p0 = 1.0; }
    dp = k * (x * p1 - p0) / (x * x - 1.0);
    // ascending order in t
    t[k - 1 - i] = 0.5 * (x + 1.0);
    w[k - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);  // = 2/((1-x^2)P'^2) scaled by 1/2
  }
}

// 1D Lagrange basis on nodes a/p, a = 0..p, evaluated at tau.
void lagrange1d(int p, double tau, double* out) {
  for (int a = 0; a <= p; ++a) {
    double v = 1.0;
    for (int b = 0; b <= p; ++b)
      if (b != a) v *= (tau - double(b) / p) / (double(a - b) / p);
    out[a] = v;
  }
}

// Silvester's product form of the equispaced Lagrange basis: the node with
// barycentric multi-index (i, j, k), i + j + k = p, has basis
// R_i(l1) R_j(l2) R_k(l3), R_n(z) = prod_{a<n} (p z - a)/(a + 1).
static void silvester(int p, int n, double z, double& val, double& der) {
  val = 1.0;
  der = 0.0;
  for (int a = 0; a < n; ++a) {
    double f = (p * z - a) / (a + 1);
    der = der * f + val * p / (a + 1);
    val *= f;
  }
}

// R_n with its first and second derivatives.
static void silvester2(int p, int n, double z, double& val, double& der, double& dd) {
  val = 1.0;
  der = 0.0;
  dd = 0.0;
  for (int a = 0; a < n; ++a) {
    const double f = (p * z - a) / (a + 1), fp = double(p) / (a + 1);
    dd = dd * f + 2.0 * der * fp;
    der = der * f + val * fp;
    val *= f;
  }
}

// Reference P_p triangle matrices of the SUPG forms (same nodes and rule as
// reference_triangle; the integrands have degree <= 2p - 2):
// St[2k + l][i][j] = (d_k psi_i, d_l psi_j) and Tt[3k + c][i][j] =
// (d_k psi_i, D_c psi_j) with D_0 = d_xi^2, D_1 = d_xi d_eta, D_2 = d_eta^2.
void reference_triangle_supg(int p, std::vector<double> St[4], std::vector<double> Tt[6]) {
  std::vector<std::pair<int, int>> loc;
  for (int t = 0; t <= p; ++t)
    for (int s = 0; s <= p - t; ++s) loc.push_back({s, t});
  const int n = (int)loc.size();
  std::vector<double> t01, w01;
  gauss_legendre01(p + 2, t01, w01);
  for (int k = 0; k < 4; ++k) St[k].assign(n * n, 0.0);
  for (int k = 0; k < 6; ++k) Tt[k].assign(n * n, 0.0);
  std::vector<double> d[2], dd[3];
  for (auto& v : d) v.resize(n);
  for (auto& v : dd) v.resize(n);
  for (size_t qa = 0; qa < t01.size(); ++qa)
    for (size_t qb = 0; qb < t01.size(); ++qb) {
      const double a = 2 * t01[qa] - 1, b = 2 * t01[qb] - 1;
      const double xi = (1 + a) * (1 - b) / 4, eta = (1 + b) / 2;
      const double w = 4 * w01[qa] * w01[qb] * (1 - b) / 8;
      const double l1 = 1 - xi - eta;
      for (int m = 0; m < n; ++m) {
        const int j = loc[m].first, k = loc[m].second, i = p - j - k;
        double r1, d1, e1, r2, d2, e2, r3, d3, e3;
        silvester2(p, i, l1, r1, d1, e1);
        silvester2(p, j, xi, r2, d2, e2);
        silvester2(p, k, eta, r3, d3, e3);
        // d/dxi = d/dl2 - d/dl1, d/deta = d/dl3 - d/dl1
        d[0][m] = r1 * d2 * r3 - d1 * r2 * r3;
        d[1][m] = r1 * r2 * d3 - d1 * r2 * r3;
        dd[0][m] = r1 * e2 * r3 - 2 * d1 * d2 * r3 + e1 * r2 * r3;
        dd[1][m] = r1 * d2 * d3 - d1 * d2 * r3 - d1 * r2 * d3 + e1 * r2 * r3;
        dd[2][m] = r1 * r2 * e3 - 2 * d1 * r2 * d3 + e1 * r2 * r3;
      }
      for (int ii = 0; ii < n; ++ii)
        for (int jj = 0; jj < n; ++jj) {
          for (int k = 0; k < 2; ++k)
            for (int l = 0; l < 2; ++l) St[2 * k + l][ii * n + jj] += w * d[k][ii] * d[l][jj];
          for (int k = 0; k < 2; ++k)
            for (int c = 0; c < 3; ++c) Tt[3 * k + c][ii * n + jj] += w * d[k][ii] * dd[c][jj];
        }
    }
}

// Reference P_p triangle matrices on {xi, eta >= 0, xi + eta <= 1} with
// equispaced nodes (s/p, t/p), t outer: mass Mt[i][j] = (psi_j, psi_i) and
// Et[k][i][j] = (psi_j, d_k psi_i).  Integrated exactly (degree 2p) by a
// collapsed Gauss-Legendre product rule with p+2 points per direction
// (xi = (1+a)(1-b)/4, eta = (1+b)/2, weight (1-b)/8).
void reference_triangle(int p, std::vector<double>& Mt, std::vector<double> Et[2]) {
  std::vector<std::pair<int, int>> loc;
  for (int t = 0; t <= p; ++t)
    for (int s = 0; s <= p - t; ++s) loc.push_back({s, t});
  const int n = (int)loc.size();
  std::vector<double> t01, w01;
  gauss_legendre01(p + 2, t01, w01);
  Mt.assign(n * n, 0.0);
  Et[0].assign(n * n, 0.0);
  Et[1].assign(n * n, 0.0);
  std::vector<double> v(n), dx(n), dy(n);
  for (size_t qa = 0; qa < t01.size(); ++qa)
    for (size_t qb = 0; qb < t01.size(); ++qb) {
      const double a = 2 * t01[qa] - 1, b = 2 * t01[qb] - 1;
      const double xi = (1 + a) * (1 - b) / 4, eta = (1 + b) / 2;
      const double w = 4 * w01[qa] * w01[qb] * (1 - b) / 8;
      const double l1 = 1 - xi - eta;
      for (int m = 0; m < n; ++m) {
        const int j = loc[m].first, k = loc[m].second, i = p - j - k;
        double r1, d1, r2, d2, r3, d3;
        silvester(p, i, l1, r1, d1);
        silvester(p, j, xi, r2, d2);
        silvester(p, k, eta, r3, d3);
        v[m] = r1 * r2 * r3;
        dx[m] = r1 * d2 * r3 - d1 * r2 * r3;   // d/dxi  = d/dl2 - d/dl1
        dy[m] = r1 * r2 * d3 - d1 * r2 * r3;   // d/deta = d/dl3 - d/dl1
      }
      for (int ii = 0; ii < n; ++ii)
        for (int jj = 0; jj < n; ++jj) {
          Mt[ii * n + jj] += w * v[ii] * v[jj];
          Et[0][ii * n + jj] += w * v[jj] * dx[ii];
          Et[1][ii * n + jj] += w * v[jj] * dy[ii];
        }
    }
}

// 1D continuous P_p mass matrix on [0,1] split into 2^r equal segments.
std::vector<double> mass1d(int p, int r) {
  int m = 1 << r, P = m * p;
  std::vector<double> t, w;
  gauss_legendre01(p + 2, t, w);
  std::vector<double> M((P + 1) * (P + 1), 0.0);
  std::vector<double> phi(p + 1);
  for (int c = 0; c < m; ++c)
    for (size_t q = 0; q < t.size(); ++q) {
      lagrange1d(p, t[q], phi.data());
      for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b) M[(c * p + a) * (P + 1) + c * p + b] += w[q] / m * phi[a] * phi[b];
    }
  return M;
}

// Prolongation of the level-rc continuous P_p space to level rf >= rc:
// Pi[l][s] = phi_s(t_l), exact for piecewise polynomials.
std::vector<double> prolong1d(int p, int rc, int rf) {
  int mc = 1 << rc, Pc = mc * p, Pf = (1 << rf) * p;
  std::vector<double> Pi((Pf + 1) * (Pc + 1), 0.0);
  std::vector<double> phi(p + 1);
  for (int l = 0; l <= Pf; ++l) {
    double t = double(l) / Pf;
    int c = std::min(int(std::floor(t * mc)), mc - 1);
    double tau = t * mc - c;
    lagrange1d(p, tau, phi.data());
    for (int a = 0; a <= p; ++a) Pi[l * (Pc + 1) + c * p + a] = phi[a];
  }
  return Pi;
}

}  // namespace

// ---------------------------------------------------------------- templates
static void build_templates(mhdg_mesh* M) {
  const int p = M->p;
  std::vector<bool> present(kMaxLevel + 1, false);
  for (auto r : M->level) present[r] = true;
  // faces may carry levels present only through max()
  for (auto& f : M->faces) present[f.level] = true;
  std::vector<double>& B = M->tmpl;
  B.clear();
  auto take = [&](size_t n) { size_t o = B.size(); B.resize(o + ((n + 31) / 32) * 32, 0.0); return (int64_t)o; };
  std::vector<double> Mt, Et[2];
  reference_triangle(p, Mt, Et);
  const int nl = (p + 1) * (p + 2) / 2;
  Templates& T = M->T;
  T.p = p;
  for (int r = 0; r <= kMaxLevel; ++r) {
    LevelTemplates& L = T.lev[r];
    L.present = present[r] ? 1 : 0;
    const int m = 1 << r, P = m * p, Q = (P + 1) * (P + 2) / 2;
    L.P = P; L.Q = Q; L.N = 3 * Q;
    for (int k = 0; k <= kMaxLevel; ++k) L.T1[k] = -1;
    L.supg = -1;
    if (!present[r]) continue;
    auto idx = [&](int i, int j) { return j * (P + 1) - j * (j - 1) / 2 + i; };
    L.Mhat = take(size_t(Q) * Q);
    L.E0 = take(size_t(Q) * Q);
    L.E1 = take(size_t(Q) * Q);
    L.E0T = take(size_t(Q) * Q);
    L.E1T = take(size_t(Q) * Q);
    double* Mh = &B[L.Mhat];
    double* E0 = &B[L.E0];
    double* E1 = &B[L.E1];
    std::vector<std::pair<int, int>> loc;
    for (int t = 0; t <= p; ++t)
      for (int s = 0; s <= p - t; ++s) loc.push_back({s, t});
    // up sub-triangles: node (s,t) -> (ap+s, bp+t); map x = (a + xi)/m
    // down sub-triangles: node (s,t) -> ((a+1)p-s, (b+1)p-t); map x = (a+1 - xi)/m
    for (int pass = 0; pass < 2; ++pass) {
      int bmax = pass == 0 ? m : m - 1;
      for (int b = 0; b < bmax; ++b)
        for (int a = 0; a < bmax - b; ++a) {
          std::vector<int> g(nl);
          for (int n = 0; n < nl; ++n) {
            int s = loc[n].first, t = loc[n].second;
            g[n] = pass == 0 ? idx(a * p + s, b * p + t) : idx((a + 1) * p - s, (b + 1) * p - t);
          }
          const double sm = 1.0 / (double(m) * m), se = (pass == 0 ? 1.0 : -1.0) / m;
          for (int i = 0; i < nl; ++i)
            for (int j = 0; j < nl; ++j) {
              size_t o = size_t(g[i]) * Q + g[j];
              Mh[o] += sm * Mt[i * nl + j];
              E0[o] += se * Et[0][i * nl + j];
              E1[o] += se * Et[1][i * nl + j];
            }
        }
    }
    for (int a = 0; a < Q; ++a)
      for (int b = 0; b < Q; ++b) {
        B[L.E0T + size_t(b) * Q + a] = E0[size_t(a) * Q + b];
        B[L.E1T + size_t(b) * Q + a] = E1[size_t(a) * Q + b];
      }
    // 1D masses
    std::vector<double> M1 = mass1d(p, r), M1i = M1;
    invert(M1i, P + 1);
    L.M1 = take(M1.size());
    std::copy(M1.begin(), M1.end(), B.begin() + L.M1);
    L.M1inv = take(M1i.size());
    std::copy(M1i.begin(), M1i.end(), B.begin() + L.M1inv);
    // edge tables (int32 stored in the double blob)
    L.edge_node = take((3 * (P + 1) + 1) / 2);
    int32_t* en = reinterpret_cast<int32_t*>(&B[L.edge_node]);
    for (int s = 0; s <= P; ++s) {
      en[0 * (P + 1) + s] = idx(s, 0);          // edge 0: j = 0, from X0 to X1
      en[1 * (P + 1) + s] = idx(P - s, s);      // edge 1: i + j = P, from X1 to X2
      en[2 * (P + 1) + s] = idx(0, P - s);      // edge 2: i = 0, from X2 to X0
    }
    L.bnd_index = take((Q + 1) / 2);
    en = reinterpret_cast<int32_t*>(&B[L.edge_node]);   // take() may have moved the blob
    int32_t* bi = reinterpret_cast<int32_t*>(&B[L.bnd_index]);
    for (int n = 0; n < Q; ++n) bi[n] = -1;
    for (int k = 0; k < 3; ++k)
      for (int s = 0; s < P; ++s) bi[en[k * (P + 1) + s]] = k * P + s;
    L.node_epos = take((3 * Q + 1) / 2);
    int32_t* ep = reinterpret_cast<int32_t*>(&B[L.node_epos]);
    for (int j = 0; j <= P; ++j)
      for (int i = 0; i <= P - j; ++i) {
        int n = idx(i, j);
        ep[3 * n + 0] = j == 0 ? i : -1;
        ep[3 * n + 1] = i + j == P ? j : -1;
        ep[3 * n + 2] = i == 0 ? P - j : -1;
      }
  }
  // coupling of a level-r macro edge with a level-rf trace: T1 = (M1(rf) Pi)^T
  for (int r = 0; r <= kMaxLevel; ++r) {
    if (!present[r]) continue;
    for (int rf = r; rf <= kMaxLevel; ++rf) {
      if (!present[rf]) continue;
      const int Pc = (1 << r) * p, Pf = (1 << rf) * p;
      std::vector<double> M1f = mass1d(p, rf), Pi = prolong1d(p, r, rf);
      int64_t o = take(size_t(Pc + 1) * (Pf + 1));
      T.lev[r].T1[rf] = o;
      for (int s = 0; s <= Pc; ++s)
        for (int l = 0; l <= Pf; ++l) {
          double v = 0;
          for (int l2 = 0; l2 <= Pf; ++l2) v += M1f[l * (Pf + 1) + l2] * Pi[l2 * (Pc + 1) + s];
          B[o + size_t(s) * (Pf + 1) + l] = v;
        }
    }
  }
  // Dirichlet sampling basis: trace basis at kb Gauss-Legendre points of a segment
  T.kb = p + 2;
  std::vector<double> t, w;
  gauss_legendre01(T.kb, t, w);
  T.dir_basis = take(size_t(p + 1) * T.kb);
  T.dir_w = take(T.kb);
  std::vector<double> phi(p + 1);
  for (int q = 0; q < T.kb; ++q) {
    lagrange1d(p, t[q], phi.data());
    for (int a = 0; a <= p; ++a) B[T.dir_basis + a * T.kb + q] = phi[a];
    B[T.dir_w + q] = w[q];
  }
}

// ---------------------------------------------------------------- layout
static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------- flux elimination
// Offsets of the per-level templates of the flux-eliminated form (8 Q x Q
// arrays, the boundary block of Minv and the two transposed boundary blocks
// of PT_a per level present); returns the blob size in doubles.
static size_t qelim_plan(const mhdg_mesh* M, QTemplates* QT) {
  size_t o = 0;
  for (int r = 0; r <= kMaxLevel; ++r) {
    QLevel& q = QT->lev[r];
    q = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    if (!M->T.lev[r].present) continue;
    const size_t QQ = size_t(M->T.lev[r].Q) * M->T.lev[r].Q;
    const size_t step = (QQ + 31) / 32 * 32;
    int64_t* f[8] = {&q.Minv, &q.P0, &q.P1, &q.PT0, &q.PT1, &q.L00, &q.L01, &q.L11};
    for (auto* x : f) { *x = int64_t(o); o += step; }
    const size_t nb = 3 * size_t(M->T.lev[r].P);
    q.Mbb = int64_t(o);
    o += (nb * nb + 31) / 32 * 32;
    const size_t qb = (size_t(M->T.lev[r].Q) * nb + 31) / 32 * 32;
    q.PB0 = int64_t(o);
    o += qb;
    q.PB1 = int64_t(o);
    o += qb;
  }
  return o;
}

// Element offsets of the Schur blocks (Q x sld each, 64-element aligned) and
// of their pivot vectors; returns the element count of the factor region.
static int64_t qelim_factor_elems(const std::vector<MacroInfo>& macros) {
  int64_t fo = 0;
  for (auto& mi : macros) {
    fo += int64_t(mi.Q) * ((mi.Q + 15) & ~15);
    fo = (fo + 63) & ~int64_t(63);
  }
  return fo;
}
// SUPG templates per present level, appended to the template blob: the
// reference-macro integrals of section 3.4's stabilisation, assembled from the
// sub-triangle matrices (up sub-triangles x = (a + xi)/m, down x = (a+1 - xi)/m,
// so a first derivative scales by +-m, a second by m^2, the measure by 1/m^2).
static void build_supg_templates(mhdg_mesh* M) {
  const int p = M->p;
  std::vector<double> St[4], Tt[6];
  reference_triangle_supg(p, St, Tt);
  const int nl = (p + 1) * (p + 2) / 2;
  std::vector<std::pair<int, int>> loc;
  for (int t = 0; t <= p; ++t)
    for (int s = 0; s <= p - t; ++s) loc.push_back({s, t});
  std::vector<double>& B = M->tmpl;
  for (int r = 0; r <= kMaxLevel; ++r) {
    LevelTemplates& L = M->T.lev[r];
    if (!L.present || L.supg >= 0) continue;
    const int m = 1 << r, P = m * p, Q = (P + 1) * (P + 2) / 2;
    const size_t QQ = size_t(Q) * Q;
    const size_t o = B.size();
    B.resize(o + ((9 * QQ + 31) / 32) * 32, 0.0);
    L.supg = (int64_t)o;
    double* S = &B[o];
    auto idx = [&](int i, int j) { return j * (P + 1) - j * (j - 1) / 2 + i; };
    for (int pass = 0; pass < 2; ++pass) {
      const int bmax = pass == 0 ? m : m - 1;
      const double sg = pass == 0 ? 1.0 : -1.0;
      for (int b = 0; b < bmax; ++b)
        for (int a = 0; a < bmax - b; ++a) {
          std::vector<int> g(nl);
          for (int n = 0; n < nl; ++n) {
            const int s = loc[n].first, t = loc[n].second;
            g[n] = pass == 0 ? idx(a * p + s, b * p + t) : idx((a + 1) * p - s, (b + 1) * p - t);
          }
          for (int i = 0; i < nl; ++i)
            for (int j = 0; j < nl; ++j) {
              const size_t e = size_t(g[i]) * Q + g[j];
              const int ij = i * nl + j;
              S[e] += St[0][ij];
              S[QQ + e] += St[3][ij];
              S[2 * QQ + e] += St[1][ij] + St[2][ij];
              for (int c = 0; c < 3; ++c) {
                S[(3 + c) * QQ + e] += sg * m * Tt[c][ij];
                S[(6 + c) * QQ + e] += sg * m * Tt[3 + c][ij];
              }
            }
        }
    }
  }
}

static void qelim_offsets(std::vector<MacroInfo>& macros) {
  int64_t fo = 0, po = 0;
  for (auto& mi : macros) {
    mi.sld = (mi.Q + 15) & ~15;
    mi.sfac_off = fo;
    mi.sperm_off = po;
    fo += int64_t(mi.Q) * mi.sld;
    fo = (fo + 63) & ~int64_t(63);
    po += mi.Q;
  }
}

// Host build of the templates: Minv = Mhat^-1 (Cholesky; Mhat is the SPD
// reference macro mass), P_a = (Ehat^a)^T Minv, PT_a = P_a^T, L_ab = P_a Ehat^b.
// The row loops are split over host threads.
static void build_qelim_templates(mhdg_mesh* M) {
  if (!M->qtmpl.empty()) return;
  const size_t total = qelim_plan(M, &M->QT);
  std::vector<double>& B = M->qtmpl;
  B.assign(total, 0.0);
  const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto par_rows = [&](int n, const std::function<void(int)>& f) {
    std::vector<std::thread> th;
    std::atomic<int> next(0);
    for (unsigned t = 0; t < nth; ++t)
      th.emplace_back([&] { for (int i = next++; i < n; i = next++) f(i); });
    for (auto& x : th) x.join();
  };
  for (int r = 0; r <= kMaxLevel; ++r) {
    const LevelTemplates& LT = M->T.lev[r];
    if (!LT.present) continue;
    const QLevel& q = M->QT.lev[r];
    const int Q = LT.Q;
    const double* Mh = &M->tmpl[LT.Mhat];
    const double* E[2] = {&M->tmpl[LT.E0], &M->tmpl[LT.E1]};
    // Cholesky Mhat = C C^T (lower C), then Minv column by column
    std::vector<double> C(Mh, Mh + size_t(Q) * Q);
    for (int j = 0; j < Q; ++j) {
      double d = C[size_t(j) * Q + j];
      for (int k = 0; k < j; ++k) d -= C[size_t(j) * Q + k] * C[size_t(j) * Q + k];
      d = std::sqrt(d);
      C[size_t(j) * Q + j] = d;
      for (int i = j + 1; i < Q; ++i) {
        double v = C[size_t(i) * Q + j];
        for (int k = 0; k < j; ++k) v -= C[size_t(i) * Q + k] * C[size_t(j) * Q + k];
        C[size_t(i) * Q + j] = v / d;
      }
    }
    double* Minv = &B[q.Minv];
    par_rows(Q, [&](int c) {   // column c of Minv (= row c: symmetric)
      std::vector<double> y(Q, 0.0);
      for (int i = 0; i < Q; ++i) {   // C y = e_c
        double v = i == c ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) v -= C[size_t(i) * Q + k] * y[k];
        y[i] = v / C[size_t(i) * Q + i];
      }
      for (int i = Q - 1; i >= 0; --i) {   // C^T x = y
        double v = y[i];
        for (int k = i + 1; k < Q; ++k) v -= C[size_t(k) * Q + i] * y[k];
        y[i] = v / C[size_t(i) * Q + i];
      }
      for (int i = 0; i < Q; ++i) Minv[size_t(c) * Q + i] = y[i];
    });
    {   // boundary block of Minv, boundary order b = kP + s
      const int P = LT.P;
      const int32_t* en = reinterpret_cast<const int32_t*>(&M->tmpl[LT.edge_node]);
      double* Mbb = &B[q.Mbb];
      for (int b = 0; b < 3 * P; ++b)
        for (int b2 = 0; b2 < 3 * P; ++b2) {
          const int n1 = en[(b / P) * (P + 1) + b % P], n2 = en[(b2 / P) * (P + 1) + b2 % P];
          Mbb[size_t(b) * 3 * P + b2] = Minv[size_t(n1) * Q + n2];
        }
    }
    double* Pa[2] = {&B[q.P0], &B[q.P1]};
    double* PTa[2] = {&B[q.PT0], &B[q.PT1]};
    for (int a = 0; a < 2; ++a) {
      par_rows(Q, [&](int i) {   // P_a[i][j] = sum_k Ehat^a[k][i] Minv[k][j]
        double* row = Pa[a] + size_t(i) * Q;
        for (int k = 0; k < Q; ++k) {
          const double e = E[a][size_t(k) * Q + i];
          if (e == 0.0) continue;
          const double* mk = Minv + size_t(k) * Q;
          for (int j = 0; j < Q; ++j) row[j] += e * mk[j];
        }
      });
      for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) PTa[a][size_t(j) * Q + i] = Pa[a][size_t(i) * Q + j];
      // boundary rows of PT_a, transposed (row j, boundary position b)
      const int P = LT.P, NB = 3 * P;
      const int32_t* en = reinterpret_cast<const int32_t*>(&M->tmpl[LT.edge_node]);
      double* PB = &B[a == 0 ? q.PB0 : q.PB1];
      for (int b = 0; b < NB; ++b) {
        const int nb = en[(b / P) * (P + 1) + b % P];
        for (int j = 0; j < Q; ++j) PB[size_t(j) * NB + b] = PTa[a][size_t(nb) * Q + j];
      }
    }
    const int ab[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    double* Lab[3] = {&B[q.L00], &B[q.L01], &B[q.L11]};
    for (int t = 0; t < 3; ++t) {
      const double* Pl = Pa[ab[t][0]];
      const double* Er = E[ab[t][1]];
      par_rows(Q, [&](int i) {   // L[i][j] = sum_k P_a[i][k] Ehat^b[k][j]
        double* row = Lab[t] + size_t(i) * Q;
        for (int k = 0; k < Q; ++k) {
          const double pv = Pl[size_t(i) * Q + k];
          const double* ek = Er + size_t(k) * Q;
          for (int j = 0; j < Q; ++j) row[j] += pv * ek[j];
        }
      });
    }
  }
}

// scratch of the split LU for every class it may factor (the LU variant can
// change between factorisations); the flux-eliminated form factors Q x Q blocks
static size_t split_lu_scratch(const mhdg_mesh* M, bool schur) {
  size_t b = 0;
  for (SizeClass c : M->classes) {
    if (schur) c.N /= 3;
    b += lu_split_scratch_bytes(c);
  }
  return b;
}

static FactorLayout factor_layout(const mhdg_mesh* M, int precision) {
  FactorLayout L{};
  size_t o = 0;
  L.meta = o;   o = align_up(o + M->macros.size() * sizeof(MacroInfo));
  L.faces = o;  o = align_up(o + M->faces.size() * sizeof(FaceInfo));
  L.bfaces = o; o = align_up(o + M->bfaces.size() * sizeof(BndFaceInfo));
  L.tmpl = o;   o = align_up(o + M->tmpl.size() * sizeof(double));
  L.order = o;  o = align_up(o + size_t(M->n_macro) * sizeof(int32_t));
  L.perm = o;   o = align_up(o + size_t(M->n_local) * sizeof(int32_t));
  L.status = o; o = align_up(o + size_t(M->n_macro) * sizeof(int32_t));
  L.R = o;      o = align_up(o + size_t(M->n_local) * sizeof(double));
  L.slots = o;  o = align_up(o + size_t(M->n_slots) * sizeof(double));
  L.lamD = o;   o = align_up(o + size_t(std::max<int64_t>(M->n_lamD, 1)) * sizeof(double));
  L.work1 = o;  o = align_up(o + size_t(M->n_local) * sizeof(double));
  L.work2 = o;  o = align_up(o + size_t(M->n_local) * sizeof(double));
  L.factors = o;
  // element count of the factor blocks: offsets are padded to 64 elements per
  // macro, and the column-streaming solves may read up to 64 x 64 elements
  // past a block's end (guard tail)
  const MacroInfo& last = M->macros.back();
  if (precision == MHDG_QELIM) {
    const size_t nf = size_t(qelim_factor_elems(M->macros)) + kFactorGuard;
    o = align_up(o + nf * 8);
    L.factors16 = o;
    QTemplates qt;
    L.qtmpl = o;   o = align_up(o + qelim_plan(M, &qt) * sizeof(double));
    L.info_lu = o; o = align_up(o + M->macros.size() * sizeof(MacroInfo));
    L.lu_scr = o;  L.lu_scr_bytes = split_lu_scratch(M, true);
    o = align_up(o + L.lu_scr_bytes);
    L.total = o;
    return L;
  }
  const size_t nf = size_t(last.fac_off) + size_t(last.N) * last.ld + kFactorGuard;
  const size_t es = precision == MHDG_FP64 ? 8 : 4;   // BF16 factors are factored in FP32
  o = align_up(o + nf * es);
  L.factors16 = o;
  if (precision == MHDG_BF16) o = align_up(o + nf * 2);
  L.lu_scr = o;  L.lu_scr_bytes = split_lu_scratch(M, false);
  o = align_up(o + L.lu_scr_bytes);
  L.total = o;
  return L;
}

static size_t solve_bytes_impl(const mhdg_mesh* M, int R);
// precision the assembly and LU run in (BF16 factors are factored in FP32)
static int lu_precision(int precision) { return precision == MHDG_BF16 ? MHDG_FP32 : precision; }
// scratch of the split LU (row moves and inverse diagonal blocks per macro)
static char* lu_scratch(mhdg_mesh* M) { return M->ws + M->L.lu_scr; }
static size_t lu_scratch_bytes(const mhdg_mesh* M) { return M->L.lu_scr_bytes; }
// the factors the per-macro solves read
static const void* solve_factors(const mhdg_mesh* M) {
  return M->ws + (M->precision == MHDG_BF16 ? M->L.factors16 : M->L.factors);
}
static mhdg_status run_macro_solve(mhdg_mesh* M, int mode, int transpose, const double* lam,
                                   const double* xin, double* yout, hipStream_t s,
                                   const int32_t* skip = nullptr);

// Interior-face trace dofs of a macro (the order of its contribution slots).
static int fold_L(const mhdg_mesh* M, const MacroInfo& mi) {
  int L = 0;
  for (int k = 0; k < 3; ++k)
    if (mi.tr_off[k] >= 0) L += (1 << mi.flevel[k]) * M->p + 1;
  return L;
}

// Fold workspace: T_K offsets int64[n_macro], then every T_K (FP64, column-major).
struct FoldLayout { size_t toff, T, total; int64_t nT; };
static FoldLayout fold_layout(const mhdg_mesh* M) {
  FoldLayout F{};
  size_t o = 0;
  F.toff = o;   o = align_up(o + size_t(M->n_macro) * 8);
  F.T = o;
  int64_t nT = 0;
  for (auto& mi : M->macros) { const int64_t L = fold_L(M, mi); nT += L * L; }
  F.nT = nT;
  F.total = align_up(o + size_t(nT) * 8);
  return F;
}
static size_t solve_bytes(const mhdg_mesh* M, int restart) { return solve_bytes_impl(M, restart); }

// Boundary-condensed workspace: W_K offsets int64[n_macro] (elements from the
// start of the block area), then every W_K (FP64, column-major, 9P x 9P).
struct BoundaryLayout { size_t off, W, total; int64_t nW; };
static BoundaryLayout boundary_layout(const mhdg_mesh* M) {
  BoundaryLayout B{};
  size_t o = 0;
  B.off = o;   o = align_up(o + size_t(M->n_macro) * 8);
  B.W = o;
  int64_t nW = 0;
  for (auto& mi : M->macros) { const int64_t nb = 9 * int64_t(mi.P); nW += nb * nb; }
  B.nW = nW;
  B.total = align_up(o + size_t(nW) * 8);
  return B;
}

// Block table of the assembled trace matrix: for every macro, every ordered
// pair of its interior faces gives a block (F, F') fed by that macro's T_K
// sub-block; the diagonal block of a face is fed by both of its macros.
// Rows in the FaceInfo order, blocks of a row in the order of first
// appearance.  T_K offsets follow mhdg_fold_operator's layout.
struct TracePlan {
  std::vector<int32_t> row_ptr;
  std::vector<TraceBlock> blocks;
  int64_t n_values = 0;
  size_t off_row = 0, off_blk = 0, off_val = 0, off_pval = 0, total = 0;
};
static TracePlan trace_plan(const mhdg_mesh* M) {
  TracePlan P;
  const int64_t nf = M->n_int;
  std::map<int64_t, int32_t> face_of_tr;   // trace offset -> interior face index
  for (int64_t f = 0; f < nf; ++f) face_of_tr[M->faces[f].tr_off] = int32_t(f);
  std::vector<std::map<int32_t, int32_t>> rowmap(nf);   // col face -> block index
  std::vector<std::vector<int32_t>> rows(nf);
  std::vector<TraceBlock> tmp;
  int64_t toff = 0;
  for (const MacroInfo& mi : M->macros) {
    const int L = fold_L(M, mi);
    int face[3], nF[3], r0[3], cnt = 0, o = 0;
    for (int k = 0; k < 3; ++k) {
      if (mi.tr_off[k] < 0) continue;
      face[cnt] = face_of_tr.at(mi.tr_off[k]);
      nF[cnt] = (1 << mi.flevel[k]) * M->p + 1;
      r0[cnt] = o;
      o += nF[cnt];
      ++cnt;
    }
    for (int a = 0; a < cnt; ++a)
      for (int b = 0; b < cnt; ++b) {
        auto it = rowmap[face[a]].find(face[b]);
        int32_t bi;
        if (it == rowmap[face[a]].end()) {
          bi = int32_t(tmp.size());
          TraceBlock tb{};
          tb.row_face = face[a];
          tb.col_face = face[b];
          tb.nF = nF[a];
          tb.nC = nF[b];
          tb.col_off = int32_t(M->faces[face[b]].tr_off);
          tmp.push_back(tb);
          rowmap[face[a]][face[b]] = bi;
          rows[face[a]].push_back(bi);
        } else {
          bi = it->second;
        }
        TraceBlock& tb = tmp[bi];
        const int c = tb.ncontrib++;
        tb.toff[c] = toff;
        tb.L[c] = L;
        tb.r0[c] = r0[a];
        tb.c0[c] = r0[b];
      }
    toff += int64_t(L) * L;
  }
  P.row_ptr.assign(nf + 1, 0);
  for (int64_t f = 0; f < nf; ++f) {
    P.row_ptr[f + 1] = P.row_ptr[f] + int32_t(rows[f].size());
    for (int32_t bi : rows[f]) {
      TraceBlock tb = tmp[bi];
      tb.voff = P.n_values;
      P.n_values += int64_t(tb.nF) * tb.nC;
      P.blocks.push_back(tb);
    }
  }
  size_t o = 0;
  P.off_row = o;  o = align_up(o + P.row_ptr.size() * sizeof(int32_t));
  P.off_blk = o;  o = align_up(o + P.blocks.size() * sizeof(TraceBlock));
  P.off_val = o;  o = align_up(o + size_t(P.n_values) * sizeof(double));
  P.off_pval = o; o = align_up(o + size_t(P.n_values) * sizeof(double));
  P.total = o;
  return P;
}
static const TracePlan& trace_plan_cached(const mhdg_mesh* M) {
  if (!M->tm_plan) M->tm_plan = std::make_shared<const TracePlan>(trace_plan(M));
  return *M->tm_plan;
}

// ---------------------------------------------------------------- GMRES
namespace {

// MHDG_PROGRESS=k in the environment prints the GMRES residual every k
// iterations to stderr (long solves on large meshes).
const int g_progress = [] {
  const char* e = std::getenv("MHDG_PROGRESS");
  return e ? std::max(0, std::atoi(e)) : 0;
}();

// Device vectors of one solve, carved from the caller's solve workspace.
// With n_inst coefficient instances every vector holds nseg = n_inst
// independent segments of length n (instance-major); the Krylov recurrences
// run per segment in lockstep.
struct Gm {
  int64_t n = 0, ld = 0;                  // segment length, column stride of V
  int nseg = 1, nblk = 1;
  int32_t op_flags = MHDG_PRECONDITION;   // MHDG_TRANSPOSE added for adjoint solves
  double *V = nullptr, *wv = nullptr, *rv = nullptr, *tv = nullptr, *fh = nullptr, *pf = nullptr;
  double* xin = nullptr;                  // fixed apply input of the captured graph
  double *partial = nullptr, *hdev = nullptr, *ydev = nullptr, *adev = nullptr;
  int32_t* skip = nullptr;                // per-segment flags: 1 = take no part in applies
  std::vector<int> seg_applies;           // applies each segment took part in
  int reorth = 0;                         // second Gram-Schmidt passes taken
  bool classic = false;                   // CGS2 instead of the delayed form
  double *pq = nullptr, *hy = nullptr, *coef = nullptr, *Hb = nullptr;  // delayed form
  double *U = nullptr, *dl = nullptr, *cl = nullptr;  // precision-refinement state
  // device-resident recurrences (gmres_device): state in the workspace, the
  // per-cycle status block (doubles then ints, one copy to the host)
  bool device = false;
  int cycles = 0, waits = 0;              // restart cycles, host waits on the stream
  GmDev dev{};
  char* stat = nullptr;
  size_t stat_bytes = 0;
  const double* fh_true = nullptr;        // f^ when stopping on the unpreconditioned residual
  int64_t len() const { return n * nseg; }
};

// Per-segment inner products <a_s, b_s> into host[0..nseg).
mhdg_status dot(mhdg_mesh* M, Gm& G, const double* a, const double* b, double* host, hipStream_t s) {
  HIP_TRY(M, launch_dots(a, G.ld, 1, b, G.n, G.partial, G.nblk, G.hdev, s, G.nseg));
  HIP_TRY(M, hipMemcpyAsync(host, G.hdev, G.nseg * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(M, hipStreamSynchronize(s));
  return MHDG_OK;
}

mhdg_status apply_op(mhdg_mesh* M, const double* lam, double* out, int32_t flags,
                     const int32_t* skip, hipStream_t s);

// Left-preconditioned restarted GMRES on D^-1 S x = b (b already
// preconditioned) with classical Gram-Schmidt and a conditional second pass
// (taken when the first leaves less than 1/sqrt(2) of the norm); all
// vectors and inner products in FP64 on the device, the Hessenberg
// least-squares problems by Givens rotations on the host.  Segment s stops
// when ||b_s - D^-1 S x_s|| <= rtol * bref[s] (checked on the true
// preconditioned residual at the start of each cycle); a segment whose
// estimate converges inside a cycle is masked out of the applies and its
// Krylov columns are zero from then on.  x holds the initial guess.
mhdg_status gmres_cgs2(mhdg_mesh* M, Gm& G, const double* b, const double* bref, double* x,
                       double rtol, int R, int max_iter, std::vector<int>& iters,
                       std::vector<double>& rel, int& applies, std::vector<char>& done,
                       hipStream_t s) {
  const int64_t n = G.n, ld = G.ld, len = G.len();
  const int ns = G.nseg;
  mhdg_status st;
  std::vector<double> H(size_t(ns) * (R + 1) * R), cs(size_t(ns) * R), sn(size_t(ns) * R),
      g(size_t(ns) * (R + 1)), h(size_t(ns) * (R + 2)), y(size_t(ns) * (R + 1)), beta(ns),
      alpha(ns), nrm(ns), w2h(2 * size_t(ns));
  std::vector<int32_t> skip(ns), skip_dev_copy(ns, -1);
  std::vector<char> active(ns);
  std::vector<int> jc(ns);
  iters.assign(ns, 0);
  rel.assign(ns, 0.0);
  done.assign(ns, 0);
  int it = 0;   // lockstep iterations
  auto push_skip = [&]() -> mhdg_status {
    if (skip == skip_dev_copy) return MHDG_OK;
    HIP_TRY(M, hipMemcpyAsync(G.skip, skip.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
    skip_dev_copy = skip;
    return MHDG_OK;
  };
  auto push_alpha = [&]() -> mhdg_status {
    HIP_TRY(M, hipMemcpyAsync(G.adev, alpha.data(), ns * sizeof(double), hipMemcpyHostToDevice, s));
    return MHDG_OK;
  };
  for (int q = 0; q < ns; ++q) {
    if (bref[q] == 0.0) {   // zero right-hand side: the solution is zero
      HIP_TRY(M, hipMemsetAsync(x + q * n, 0, n * sizeof(double), s));
      done[q] = 1;
    }
    skip[q] = done[q];
  }
  while (true) {
    if ((st = push_skip())) return st;
    if ((st = apply_op(M, x, G.tv, G.op_flags, G.skip, s))) return st;
    ++applies;
    for (int q = 0; q < ns; ++q) G.seg_applies[q] += !skip[q];
    HIP_TRY(M, launch_scale_copy(1.0, b, G.rv, len, s));
    HIP_TRY(M, launch_axpby(-1.0, G.tv, 1.0, G.rv, len, s));
    ++G.waits;
    if ((st = dot(M, G, G.rv, G.rv, nrm.data(), s))) return st;
    bool any = false;
    jc.assign(ns, 0);
    for (int q = 0; q < ns; ++q) {
      if (done[q]) { active[q] = 0; alpha[q] = 0.0; skip[q] = 1; continue; }
      beta[q] = std::sqrt(nrm[q]);
      if (!std::isfinite(beta[q]) || !std::isfinite(bref[q]))
        return fail(M, MHDG_ERR_NOT_CONVERGED, "gmres: non-finite residual");
      rel[q] = beta[q] / bref[q];
      if (rel[q] <= rtol) done[q] = 1;
      active[q] = !done[q];
      alpha[q] = active[q] && beta[q] > 0 ? 1.0 / beta[q] : 0.0;
      skip[q] = !active[q];
      any |= active[q] != 0;
      std::fill(g.begin() + q * (R + 1), g.begin() + (q + 1) * (R + 1), 0.0);
      g[q * (R + 1)] = beta[q];
    }
    if (!any || it >= max_iter) return MHDG_OK;
    ++G.cycles;
    if ((st = push_skip()) || (st = push_alpha())) return st;
    HIP_TRY(M, launch_seg_scale_copy(G.adev, G.rv, G.V, n, ns, s));
    int j = 0;
    for (; j < R && it < max_iter; ++j) {
      ++it;
      const double* vj = G.V + j * ld;
      if (G.op_flags & MHDG_GRAPH) {   // the graph reads a fixed input vector
        HIP_TRY(M, hipMemcpyAsync(G.xin, vj, len * sizeof(double), hipMemcpyDeviceToDevice, s));
        vj = G.xin;
      }
      if ((st = apply_op(M, vj, G.wv, G.op_flags, G.skip, s))) return st;
      ++applies;
      for (int q = 0; q < ns; ++q) G.seg_applies[q] += !skip[q];
      // classical Gram-Schmidt; a second pass only where the first removed
      // most of w (||w_after||^2 < ||w_before||^2 / 2, the "twice is enough"
      // criterion), so most iterations read the basis twice, not four times.
      // One host synchronisation per pass: projections and both norms together.
      double* w2 = G.ydev;   // [0, ns): ||w||^2 before the pass, [ns, 2 ns): after
      for (int pass = 0; pass < 2; ++pass) {
        HIP_TRY(M, launch_dots(G.V, ld, j + 1, G.wv, n, G.partial, G.nblk, G.hdev, s, ns));
        HIP_TRY(M, launch_dots(G.wv, ld, 1, G.wv, n, G.partial, G.nblk, w2, s, ns));
        HIP_TRY(M, launch_gemv_sub(G.V, ld, j + 1, G.hdev, G.wv, n, -1.0, s, ns));
        HIP_TRY(M, launch_dots(G.wv, ld, 1, G.wv, n, G.partial, G.nblk, w2 + ns, s, ns));
        HIP_TRY(M, hipMemcpyAsync(h.data(), G.hdev, size_t(j + 1) * ns * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
        HIP_TRY(M, hipMemcpyAsync(w2h.data(), w2, 2 * ns * sizeof(double), hipMemcpyDeviceToHost, s));
        ++G.waits;
        HIP_TRY(M, hipStreamSynchronize(s));
        bool again = false;
        for (int q = 0; q < ns; ++q) {
          if (!active[q]) continue;
          double* Hq = &H[size_t(q) * (R + 1) * R];
          for (int i = 0; i <= j; ++i) Hq[i * R + j] = (pass ? Hq[i * R + j] : 0.0) + h[i * ns + q];
          nrm[q] = w2h[ns + q];
          again |= !(w2h[ns + q] >= 0.5 * w2h[q]);
        }
        if (!again) break;
        ++G.reorth;
      }
      any = false;
      for (int q = 0; q < ns; ++q) {
        if (!active[q]) { alpha[q] = 0.0; continue; }
        double* Hq = &H[size_t(q) * (R + 1) * R];
        double* c = &cs[size_t(q) * R];
        double* sq = &sn[size_t(q) * R];
        double* gq = &g[size_t(q) * (R + 1)];
        const double hn = std::sqrt(nrm[q]);
        Hq[(j + 1) * R + j] = hn;
        alpha[q] = hn > 0 ? 1.0 / hn : 0.0;
        for (int i = 0; i < j; ++i) {
          const double a = Hq[i * R + j], bb = Hq[(i + 1) * R + j];
          Hq[i * R + j] = c[i] * a + sq[i] * bb;
          Hq[(i + 1) * R + j] = -sq[i] * a + c[i] * bb;
        }
        const double a = Hq[j * R + j], bb = Hq[(j + 1) * R + j];
        const double rr = std::hypot(a, bb);
        c[j] = rr == 0 ? 1.0 : a / rr;
        sq[j] = rr == 0 ? 0.0 : bb / rr;
        Hq[j * R + j] = rr;
        Hq[(j + 1) * R + j] = 0.0;
        gq[j + 1] = -sq[j] * gq[j];
        gq[j] = c[j] * gq[j];
        rel[q] = std::fabs(gq[j + 1]) / bref[q];
        jc[q] = j + 1;
        ++iters[q];
        if (rel[q] <= rtol || hn == 0.0) {   // this cycle is done for q
          active[q] = 0;
          alpha[q] = 0.0;
          skip[q] = 1;
        }
        any |= active[q] != 0;
      }
      if (g_progress && it % g_progress == 0) {
        double worst = 0;
        for (int q = 0; q < ns; ++q)
          if (!done[q]) worst = std::max(worst, rel[q]);
        std::fprintf(stderr, "[mhdg] gmres iteration %d relative residual %.3e (%d second passes)\n",
                     it, worst, G.reorth);
        std::fflush(stderr);
      }
      if ((st = push_alpha())) return st;
      HIP_TRY(M, launch_seg_scale_copy(G.adev, G.wv, G.V + (j + 1) * ld, n, ns, s));
      if ((st = push_skip())) return st;
      if (!any) { ++j; break; }
    }
    // x_q += V y_q with R_q y_q = g_q over segment q's jc[q] columns
    int jmax = 0;
    std::fill(y.begin(), y.end(), 0.0);
    for (int q = 0; q < ns; ++q) {
      const int jq = jc[q];
      jmax = std::max(jmax, jq);
      const double* Hq = &H[size_t(q) * (R + 1) * R];
      const double* gq = &g[size_t(q) * (R + 1)];
      std::vector<double> yq(jq);
      for (int i = jq - 1; i >= 0; --i) {
        double v = gq[i];
        for (int kk = i + 1; kk < jq; ++kk) v -= Hq[i * R + kk] * yq[kk];
        yq[i] = v / Hq[i * R + i];
      }
      for (int i = 0; i < jq; ++i) y[size_t(i) * ns + q] = yq[i];
    }
    if (jmax > 0) {
      HIP_TRY(M, hipMemcpyAsync(G.ydev, y.data(), size_t(jmax) * ns * sizeof(double),
                                hipMemcpyHostToDevice, s));
      HIP_TRY(M, launch_gemv_sub(G.V, ld, jmax, G.ydev, x, n, 1.0, s, ns));
    }
    ++G.waits;
    HIP_TRY(M, hipStreamSynchronize(s));
    for (int q = 0; q < ns; ++q) skip[q] = done[q];
  }
}

// GMRES with delayed reorthogonalisation: the same left-preconditioned,
// restarted GMRES and stopping rule as gmres_cgs2, with the Arnoldi basis
// built so that each iteration makes one host synchronisation and reads the
// basis twice (classical Gram-Schmidt applied twice reads it four times):
//   u_j      the new direction after one projection against q_0..q_{j-1},
//            not yet normalised, kept in V column j;
//   z = D^-1 S u_j                              (apply to u_j, not to q_j)
//   p = [q_0..q_{j-1}, u_j]^T u_j, c = [q_0..q_{j-1}, u_j]^T z   (one pass)
//   a = p[0..j), beta = sqrt(p_j - a.a): u_j's second projection and norm,
//            which complete Arnoldi column j-1 = [h_{j-1} + a; beta]
//   q_j = (u_j - Q a) / beta
//   D^-1 S q_j = (z - Q_j Hbar a) / beta   (Arnoldi relation for the columns
//            before), so the first projection of D^-1 S q_j onto Q_j is
//            h_j = ([c_0..c_{j-1}, (c_j - a.c) / beta] - Hbar a) / beta and
//   u_{j+1} = (z - Q_j [c; (c_j - a.c) / beta]) / beta      (one pass for both)
// Hbar a is formed on the device from the finished columns.  A column is
// complete one iteration after its apply, so the convergence test lags one
// apply; the last column of a cycle is completed by a projection pass
// without an apply.
mhdg_status gmres_delayed(mhdg_mesh* M, Gm& G, const double* b, const double* bref, double* x,
                          double rtol, int R, int max_iter, std::vector<int>& iters,
                          std::vector<double>& rel, int& applies, std::vector<char>& done,
                          hipStream_t s) {
  const int64_t n = G.n, ld = G.ld, len = G.len();
  const int ns = G.nseg;
  const int64_t hld = R + 1;   // rows of Hbar
  mhdg_status st;
  std::vector<double> Hr(size_t(ns) * (R + 1) * R), cs(size_t(ns) * R), sn(size_t(ns) * R),
      g(size_t(ns) * (R + 1)), hprev(size_t(ns) * (R + 1)), beta(ns), nrm(ns), y(size_t(ns) * R),
      alpha(ns);
  // the buffers that cross to and from the device every iteration, page-locked:
  // dual products and Hbar a (read back), the finished Hbar column and the update
  // coefficients (sent).  Each is rewritten by the host only after the stream
  // synchronisation of the next iteration, so an earlier copy has always run.
  const size_t n_pq = 3 * size_t(R + 2) * ns, n_col = size_t(R + 2) * ns,
               n_coef = (2 * size_t(R) + 3) * ns;
  double* const pin = M->host_buffer(n_pq + n_col + n_coef);
  if (!pin) return fail(M, MHDG_ERR_HIP, "solve: page-locked host buffer not available");
  double* const pq = pin;
  double* const col = pin + n_pq;
  double* const coef = col + n_col;
  std::fill(pin, pin + n_pq + n_col + n_coef, 0.0);
  std::vector<int32_t> skip(ns), skip_dev_copy(ns, -1);
  std::vector<char> active(ns);
  std::vector<int> jc(ns);
  iters.assign(ns, 0);
  rel.assign(ns, 0.0);
  done.assign(ns, 0);
  int it = 0;
  auto push_skip = [&]() -> mhdg_status {
    if (skip == skip_dev_copy) return MHDG_OK;
    HIP_TRY(M, hipMemcpyAsync(G.skip, skip.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
    skip_dev_copy = skip;
    return MHDG_OK;
  };
  for (int q = 0; q < ns; ++q) {
    if (bref[q] == 0.0) {
      HIP_TRY(M, hipMemsetAsync(x + q * n, 0, n * sizeof(double), s));
      done[q] = 1;
    }
    skip[q] = done[q];
  }
  // q_j / u_{j+1} coefficients, packed per iteration as [ca (j ns) | cd (j ns) |
  // sc (3 ns)] in one host buffer and one device buffer, one copy per iteration
  double* const coefd = G.coef;
  while (true) {
    // ---- true preconditioned residual, cycle start
    if ((st = push_skip())) return st;
    if ((st = apply_op(M, x, G.tv, G.op_flags, G.skip, s))) return st;
    ++applies;
    for (int q = 0; q < ns; ++q) G.seg_applies[q] += !skip[q];
    HIP_TRY(M, launch_scale_copy(1.0, b, G.rv, len, s));
    HIP_TRY(M, launch_axpby(-1.0, G.tv, 1.0, G.rv, len, s));
    ++G.waits;
    if ((st = dot(M, G, G.rv, G.rv, nrm.data(), s))) return st;
    bool any = false;
    jc.assign(ns, 0);
    for (int q = 0; q < ns; ++q) {
      if (!done[q]) {
        beta[q] = std::sqrt(nrm[q]);
        if (!std::isfinite(beta[q]) || !std::isfinite(bref[q]))
          return fail(M, MHDG_ERR_NOT_CONVERGED, "gmres: non-finite residual");
        rel[q] = beta[q] / bref[q];
        if (rel[q] <= rtol || beta[q] == 0.0) done[q] = 1;
      }
      active[q] = !done[q];
      alpha[q] = active[q] ? 1.0 : 0.0;
      skip[q] = !active[q];
      any |= active[q] != 0;
      std::fill(g.begin() + q * (R + 1), g.begin() + (q + 1) * (R + 1), 0.0);
      g[q * (R + 1)] = active[q] ? beta[q] : 0.0;
    }
    if (!any || it >= max_iter) return MHDG_OK;
    ++G.cycles;
    if ((st = push_skip())) return st;
    HIP_TRY(M, hipMemcpyAsync(G.adev, alpha.data(), ns * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(M, launch_seg_scale_copy(G.adev, G.rv, G.V, n, ns, s));   // u_0 = r
    int j = 0;
    while (true) {
      const bool last = j == R || it >= max_iter;
      double* u = G.V + j * ld;
      if (!last) {
        const double* uin = u;
        if (G.op_flags & MHDG_GRAPH) {   // the captured graph reads a fixed input vector;
          // after the first column the previous dual update wrote u_j there too
          if (j == 0)
            HIP_TRY(M, hipMemcpyAsync(G.xin, u, len * sizeof(double), hipMemcpyDeviceToDevice, s));
          uin = G.xin;
        }
        if ((st = apply_op(M, uin, G.wv, G.op_flags, G.skip, s))) return st;   // z = A u_j
        ++applies;
        ++it;
        for (int q = 0; q < ns; ++q) G.seg_applies[q] += !skip[q];
        HIP_TRY(M, launch_dots2(G.V, ld, j + 1, u, G.wv, n, G.partial, G.nblk, G.pq, s, ns));
      } else {
        // complete the last column: projections of u_j only
        HIP_TRY(M, launch_dots(G.V, ld, j + 1, u, n, G.partial, G.nblk, G.hy, s, ns));
      }
      // Hbar a lands right after the 2 (j + 1) ns dual products (the pq and hy
      // regions of the workspace are contiguous), so one copy brings both back
      const size_t npq = 2 * size_t(j + 1) * ns;
      if (!last && j >= 2)
        HIP_TRY(M, launch_hbar_gemv(G.Hb, hld, ns, j - 1, j, G.pq, G.pq + npq, s));
      const double* hyv = pq + npq;
      if (!last) {
        HIP_TRY(M, hipMemcpyAsync(pq, G.pq,
                                  (npq + (j >= 2 ? size_t(j) * ns : 0)) * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
      } else {
        // same layout as dots2's first products: pq[(2c) ns + q]
        std::vector<double> pl(size_t(j + 1) * ns);
        HIP_TRY(M, hipMemcpyAsync(pl.data(), G.hy, pl.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
        ++G.waits;
        HIP_TRY(M, hipStreamSynchronize(s));
        for (int c = 0; c <= j; ++c)
          for (int q = 0; q < ns; ++q) pq[(2 * size_t(c)) * ns + q] = pl[size_t(c) * ns + q];
      }
      ++G.waits;
      HIP_TRY(M, hipStreamSynchronize(s));
      any = false;
      for (int q = 0; q < ns; ++q) {
        if (!active[q]) continue;
        // u_j's second projection and norm
        double aa = 0.0;
        for (int c = 0; c < j; ++c) { const double ac = pq[(2 * size_t(c)) * ns + q]; aa += ac * ac; }
        const double om = pq[(2 * size_t(j)) * ns + q];
        const double bt = std::sqrt(std::max(om - aa, 0.0));
        beta[q] = bt;
        if (j >= 1) {
          // finish Arnoldi column j-1 = [h_{j-1} + a; beta], rotate, test
          double* Hq = &Hr[size_t(q) * (R + 1) * R];
          double* c_ = &cs[size_t(q) * R];
          double* s_ = &sn[size_t(q) * R];
          double* gq = &g[size_t(q) * (R + 1)];
          const int jj = j - 1;
          for (int i = 0; i < j; ++i) {
            const double v = hprev[size_t(q) * (R + 1) + i] + pq[(2 * size_t(i)) * ns + q];
            col[size_t(i) * ns + q] = v;
            Hq[i * R + jj] = v;
          }
          col[size_t(j) * ns + q] = bt;
          Hq[j * R + jj] = bt;
          for (int i = 0; i < jj; ++i) {
            const double a_ = Hq[i * R + jj], b_ = Hq[(i + 1) * R + jj];
            Hq[i * R + jj] = c_[i] * a_ + s_[i] * b_;
            Hq[(i + 1) * R + jj] = -s_[i] * a_ + c_[i] * b_;
          }
          const double a_ = Hq[jj * R + jj], b_ = Hq[(jj + 1) * R + jj];
          const double rr = std::hypot(a_, b_);
          c_[jj] = rr == 0 ? 1.0 : a_ / rr;
          s_[jj] = rr == 0 ? 0.0 : b_ / rr;
          Hq[jj * R + jj] = rr;
          Hq[(jj + 1) * R + jj] = 0.0;
          gq[jj + 1] = -s_[jj] * gq[jj];
          gq[jj] = c_[jj] * gq[jj];
          rel[q] = std::fabs(gq[jj + 1]) / bref[q];
          jc[q] = j;
          ++iters[q];
          if (rel[q] <= rtol || bt == 0.0) { active[q] = 0; skip[q] = 1; }
        } else if (bt == 0.0) {
          active[q] = 0;
          skip[q] = 1;
        }
        any |= active[q] != 0;
      }
      if (g_progress && !last && it % g_progress == 0) {
        double worst = 0;
        for (int q = 0; q < ns; ++q)
          if (!done[q]) worst = std::max(worst, rel[q]);
        std::fprintf(stderr, "[mhdg] gmres iteration %d relative residual %.3e\n", it, worst);
        std::fflush(stderr);
      }
      if (j >= 1) {   // finished column j-1 of every segment to the device copy of Hbar
        for (int q = 0; q < ns; ++q)
          if (jc[q] != j)   // segments that were already inactive: zero column
            for (int i = 0; i <= j; ++i) col[size_t(i) * ns + q] = 0.0;
        HIP_TRY(M, hipMemcpyAsync(G.Hb + (size_t(j - 1) * hld) * ns, col,
                                  size_t(j + 1) * ns * sizeof(double), hipMemcpyHostToDevice, s));
      }
      if (last || !any) break;
      // coefficients of q_j and u_{j+1}
      for (int q = 0; q < ns; ++q) {
        double* cc = coef;
        double* cdd = coef + size_t(j) * ns;
        double* scc = coef + 2 * size_t(j) * ns;
        if (!active[q]) {
          for (int c = 0; c < j; ++c) { cc[size_t(c) * ns + q] = 0.0; cdd[size_t(c) * ns + q] = 0.0; }
          scc[q] = scc[ns + q] = scc[2 * ns + q] = 0.0;
          continue;
        }
        const double bt = beta[q];
        double ab = 0.0;
        for (int c = 0; c < j; ++c) ab += pq[(2 * size_t(c)) * ns + q] * pq[(2 * size_t(c) + 1) * ns + q];
        const double cj = (pq[(2 * size_t(j) + 1) * ns + q] - ab) / bt;
        // Hbar a: device part (columns < j-1) plus the column just finished
        double* hp = &hprev[size_t(q) * (R + 1)];
        const double aj1 = j >= 1 ? pq[(2 * size_t(j - 1)) * ns + q] : 0.0;
        for (int i = 0; i <= j; ++i) {
          double hba = (j >= 2 && i < j) ? hyv[size_t(i) * ns + q] : 0.0;
          if (j >= 1) hba += aj1 * col[size_t(i) * ns + q];
          const double ci = i < j ? pq[(2 * size_t(i) + 1) * ns + q] : cj;
          hp[i] = (ci - hba) / bt;
        }
        for (int c = 0; c < j; ++c) {
          const double ac = pq[(2 * size_t(c)) * ns + q];
          cc[size_t(c) * ns + q] = ac / bt;
          cdd[size_t(c) * ns + q] = (pq[(2 * size_t(c) + 1) * ns + q] - (cj / bt) * ac) / bt;
        }
        scc[q] = 1.0 / bt;
        scc[ns + q] = 1.0 / bt;
        scc[2 * ns + q] = -cj / (bt * bt);
      }
      HIP_TRY(M, hipMemcpyAsync(coefd, coef, (2 * size_t(j) + 3) * ns * sizeof(double),
                                hipMemcpyHostToDevice, s));
      HIP_TRY(M, launch_dual_update(G.V, ld, j, n, ns, coefd, coefd + size_t(j) * ns,
                                    coefd + 2 * size_t(j) * ns, G.wv,
                                    (G.op_flags & MHDG_GRAPH) ? G.xin : nullptr, s));
      if ((st = push_skip())) return st;
      ++j;
    }
    // ---- x_q += Q y_q with R_q y_q = g_q over jc[q] columns
    int jmax = 0;
    std::fill(y.begin(), y.end(), 0.0);
    for (int q = 0; q < ns; ++q) {
      const int jq = jc[q];
      jmax = std::max(jmax, jq);
      const double* Hq = &Hr[size_t(q) * (R + 1) * R];
      const double* gq = &g[size_t(q) * (R + 1)];
      std::vector<double> yq(jq);
      for (int i = jq - 1; i >= 0; --i) {
        double v = gq[i];
        for (int kk = i + 1; kk < jq; ++kk) v -= Hq[i * R + kk] * yq[kk];
        yq[i] = v / Hq[i * R + i];
      }
      for (int i = 0; i < jq; ++i) y[size_t(i) * ns + q] = yq[i];
    }
    if (jmax > 0) {
      HIP_TRY(M, hipMemcpyAsync(G.ydev, y.data(), size_t(jmax) * ns * sizeof(double),
                                hipMemcpyHostToDevice, s));
      HIP_TRY(M, launch_gemv_sub(G.V, ld, jmax, G.ydev, x, n, 1.0, s, ns));
    }
    ++G.waits;
    HIP_TRY(M, hipStreamSynchronize(s));
    for (int q = 0; q < ns; ++q) skip[q] = done[q];
  }
}

mhdg_status apply_launches(mhdg_mesh* M, const double* lam, double* out, int32_t flags,
                           const int32_t* skip, hipStream_t s);

// Columns per captured graph of a cycle (the cycle's graphs are launched back
// to back; the host waits once per cycle).
constexpr int kGmChunk = 32;
// Longest restart of the device driver (gm_step keeps 3 (R + 2) doubles in LDS).
constexpr int kDeviceMaxRestart = 2048;

// Restarted GMRES with the per-segment recurrences on the device
// (gmres_dev.hip): the same left-preconditioned Arnoldi process with delayed
// reorthogonalisation and the same stopping rule as gmres_delayed, but the
// scalar work between kernels (projections, Givens rotations, residual
// estimate, update coefficients, the triangular solve) runs in kernels, so a
// restart cycle is a fixed sequence of launches that ends with the residual
// of the next cycle.  With MHDG_GRAPH in G.op_flags each cycle replays
// hipGraphs captured once per (vectors, restart, flags); otherwise the same
// launches run directly.  The host synchronises once per cycle, to read the
// per-segment status.  A segment that converges, or reaches max_iter
// finished columns, inside a cycle is masked out of every later launch.
// With G.fh_true set the test is on the unpreconditioned residual:
// ||f^_s - S x_s|| <= rtol ||f^_s||, checked exactly at each cycle start; in
// the cycle the estimate of the preconditioned residual is compared with a
// target scaled by the ratio of the two norms at the cycle start.
mhdg_status gmres_device(mhdg_mesh* M, Gm& G, const double* b, const double* bref, double* x,
                         double rtol, int R, int max_iter, std::vector<int>& iters,
                         std::vector<double>& rel, std::vector<double>& rel_true, int& applies,
                         std::vector<char>& done, hipStream_t s) {
  const int64_t n = G.n, ld = G.ld, len = G.len();
  const int ns = G.nseg;
  const int64_t hld = R + 1;
  GmDev& d = G.dev;
  const bool use_graph = (G.op_flags & MHDG_GRAPH) != 0;
  const int32_t aflags = G.op_flags & ~MHDG_GRAPH;
  const bool true_norm = G.fh_true != nullptr;
  if (!true_norm) d.nrm_true = nullptr;   // gm_start tests the preconditioned residual
  // the first kGmColumnMax columns of a cycle finish in one launch after the
  // products (MHDG_GM_COLUMN_LAUNCHES=3 keeps the three separate launches;
  // both give the same bits)
  const char* cl_env = std::getenv("MHDG_GM_COLUMN_LAUNCHES");
  const bool fused_column = !(cl_env && std::atoi(cl_env) == 3);
  mhdg_status st;
  // ---- initial state: parameters, reference norms, flags
  const size_t nd_in = 2 + 2 * size_t(ns);   // prm, bref, fref
  const size_t ni = 7 * size_t(ns) + 1;      // the int block (see carve)
  double* const pin = M->host_buffer(nd_in + G.stat_bytes / sizeof(double) + ni);
  if (!pin) return fail(M, MHDG_ERR_HIP, "solve: page-locked host buffer not available");
  double* const hin = pin;
  char* const hstat = (char*)(pin + nd_in);
  int32_t* const hint = (int32_t*)(hstat + G.stat_bytes);
  hin[0] = rtol;
  hin[1] = double(max_iter);
  std::vector<double> fref(ns, 0.0);
  if (true_norm) {
    HIP_TRY(M, launch_dots(G.fh_true, ld, 1, G.fh_true, n, G.partial, G.nblk, G.hdev, s, ns));
    HIP_TRY(M, hipMemcpyAsync(fref.data(), G.hdev, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    ++G.waits;
    HIP_TRY(M, hipStreamSynchronize(s));
    for (auto& v : fref) v = std::sqrt(v);
  }
  done.assign(ns, 0);
  std::fill(hint, hint + ni, 0);
  for (int q = 0; q < ns; ++q) {
    hin[2 + q] = bref[q];
    hin[2 + ns + q] = fref[q];
    if (bref[q] == 0.0 || (true_norm && fref[q] == 0.0)) {
      HIP_TRY(M, hipMemsetAsync(x + q * n, 0, n * sizeof(double), s));
      done[q] = 1;
    }
    hint[2 * ns + q] = done[q];   // done
    hint[6 * ns + q] = done[q];   // skip
  }
  HIP_TRY(M, hipMemcpyAsync(d.prm, hin, nd_in * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(M, hipMemcpyAsync(d.active, hint, ni * sizeof(int32_t), hipMemcpyHostToDevice, s));

  // ---- the launch sequences of a cycle
  auto seq_start = [&](hipStream_t t) -> mhdg_status {
    mhdg_status e;
    if (true_norm) {   // r = f^ - S x, ||r||, then D^-1 r
      if ((e = apply_launches(M, x, G.tv, aflags & ~MHDG_PRECONDITION, d.skip, t))) return e;
      HIP_TRY(M, launch_scale_copy(1.0, G.fh_true, G.cl, len, t));
      HIP_TRY(M, launch_axpby(-1.0, G.tv, 1.0, G.cl, len, t));
      HIP_TRY(M, launch_dots(G.cl, ld, 1, G.cl, n, G.partial, G.nblk, d.nrm_true, t, ns));
      FactorLayout& L = M->L;
      HIP_TRY(M, launch_face_combine(FACE_DINV, (const FaceInfo*)(M->ws + L.faces), M->n_int,
                                     (const double*)(M->ws + L.tmpl), M->T, M->tau, G.cl,
                                     nullptr, G.rv, t));
    } else {           // r = b - D^-1 S x
      if ((e = apply_launches(M, x, G.tv, aflags, d.skip, t))) return e;
      HIP_TRY(M, launch_scale_copy(1.0, b, G.rv, len, t));
      HIP_TRY(M, launch_axpby(-1.0, G.tv, 1.0, G.rv, len, t));
    }
    HIP_TRY(M, launch_dots(G.rv, ld, 1, G.rv, n, G.partial, G.nblk, d.nrm, t, ns));
    HIP_TRY(M, launch_gm_start(d, R, t));
    HIP_TRY(M, launch_seg_scale_copy(d.alpha, G.rv, G.V, n, ns, t));   // u_0 = r
    return MHDG_OK;
  };
  auto seq_column = [&](int j, hipStream_t t) -> mhdg_status {
    double* u = G.V + j * ld;
    mhdg_status e;
    if ((e = apply_launches(M, u, G.wv, aflags, d.skip, t))) return e;   // z = D^-1 S u_j
    if (fused_column && j + 1 <= kGmColumnMax) {   // the same sums in one launch
      HIP_TRY(M, launch_dots2_partial(G.V, ld, j + 1, u, G.wv, n, G.partial, G.nblk, t, ns,
                                      d.skip));
      HIP_TRY(M, launch_gm_column(d, G.partial, G.nblk, R, j, t));
    } else {
      HIP_TRY(M, launch_dots2(G.V, ld, j + 1, u, G.wv, n, G.partial, G.nblk, d.pq, t, ns, d.skip));
      if (j >= 2)
        HIP_TRY(M, launch_hbar_gemv(G.Hb, hld, ns, j - 1, j, d.pq, d.pq + 2 * size_t(j + 1) * ns, t));
      HIP_TRY(M, launch_gm_step(d, R, j, 0, t));
    }
    HIP_TRY(M, launch_dual_update(G.V, ld, j, n, ns, d.coef, d.coef + size_t(j) * ns,
                                  d.coef + 2 * size_t(j) * ns, G.wv, nullptr, t, d.skip));
    return MHDG_OK;
  };
  auto seq_close = [&](hipStream_t t) -> mhdg_status {
    // the last column: projections of u_R only; then y and x += V y
    HIP_TRY(M, launch_dots(G.V, ld, R + 1, G.V + R * ld, n, G.partial, G.nblk, d.hy, t, ns,
                           d.skip));
    HIP_TRY(M, launch_gm_step(d, R, R, 1, t));
    HIP_TRY(M, launch_gm_lsq(d, R, t));
    HIP_TRY(M, launch_gemv_sub(G.V, ld, R, d.y, x, n, 1.0, t, ns, d.jc));
    return seq_start(t);
  };
  const int nchunk = (R + kGmChunk - 1) / kGmChunk;
  // graph p < nchunk: columns [p kGmChunk, ...) (the last one with the close);
  // graph nchunk: the first cycle start
  auto seq_graph = [&](int p, hipStream_t t) -> mhdg_status {
    if (p == nchunk) return seq_start(t);
    mhdg_status e;
    for (int j = p * kGmChunk; j < std::min(R, (p + 1) * kGmChunk); ++j)
      if ((e = seq_column(j, t))) return e;
    return p == nchunk - 1 ? seq_close(t) : MHDG_OK;
  };
  mhdg_mesh::GmGraphs* gg = nullptr;
  if (use_graph) {
    const mhdg_mesh::GmKey key{G.V, x, b, G.fh_true, R, ns, aflags};
    for (auto& e : M->gm_graphs)
      if (e.key == key) gg = &e;
    if (!gg) {
      if (!M->cap) HIP_TRY(M, hipStreamCreateWithFlags(&M->cap, hipStreamNonBlocking));
      mhdg_mesh::GmGraphs ng;
      ng.key = key;
      const bool prof = M->prof;
      M->prof = false;   // no event records inside the graphs
      for (int p = 0; p <= nchunk; ++p) {
        HIP_TRY(M, hipStreamBeginCapture(M->cap, hipStreamCaptureModeThreadLocal));
        mhdg_status e = seq_graph(p, M->cap);
        hipGraph_t g = nullptr;
        hipError_t he = hipStreamEndCapture(M->cap, &g);
        hipGraphExec_t gx = nullptr;
        if (!e && he == hipSuccess) he = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e || he != hipSuccess) {
          M->prof = prof;
          for (auto xg : ng.x) (void)hipGraphExecDestroy(xg);
          if (e) return e;
          return fail(M, MHDG_ERR_HIP, std::string("solve: graph capture: ") + hipGetErrorString(he));
        }
        ng.x.push_back(gx);
      }
      M->prof = prof;
      if (M->gm_graphs.size() >= 4) {   // bounded cache: drop the oldest
        for (auto xg : M->gm_graphs.front().x) (void)hipGraphExecDestroy(xg);
        M->gm_graphs.erase(M->gm_graphs.begin());
      }
      M->gm_graphs.push_back(std::move(ng));
      gg = &M->gm_graphs.back();
    }
  }
  // status after a cycle: rel | rel_true | est (doubles), then the int block
  const double* srel = (const double*)hstat;
  const double* srel_true = srel + ns;
  const int32_t* sint = (const int32_t*)(hstat + G.stat_bytes - ni * sizeof(int32_t));
  const int32_t* s_done = sint + 2 * ns;
  const int32_t* s_iters = sint + 3 * ns;
  const int32_t* s_flag = sint + 4 * ns;
  const int32_t* s_napp = sint + 5 * ns;
  const int32_t* s_any = sint + 7 * ns;
  std::vector<int32_t> napp_prev(ns, 0);
  auto read_status = [&]() -> mhdg_status {
    HIP_TRY(M, hipMemcpyAsync(hstat, G.stat, G.stat_bytes, hipMemcpyDeviceToHost, s));
    ++G.waits;
    HIP_TRY(M, hipStreamSynchronize(s));
    for (int q = 0; q < ns; ++q)
      if (s_flag[q]) return fail(M, MHDG_ERR_NOT_CONVERGED, "gmres: non-finite residual");
    for (int q = 0; q < ns; ++q) {
      // applies per segment: its residual apply (when not done before the
      // cycle start) plus the Krylov applies it took part in
      G.seg_applies[q] += s_napp[q] - napp_prev[q];
      napp_prev[q] = s_napp[q];
    }
    return MHDG_OK;
  };
  auto run = [&](int p) -> mhdg_status {
    if (use_graph) {
      HIP_TRY(M, hipGraphLaunch(gg->x[p], s));
      return MHDG_OK;
    }
    return seq_graph(p, s);
  };
  // cycle starts: residual apply for the segments not yet done
  auto count_start = [&]() {
    int any = 0;
    for (int q = 0; q < ns; ++q)
      if (!done[q]) { ++G.seg_applies[q]; any = 1; }
    applies += any;
  };
  count_start();
  if ((st = run(nchunk))) return st;
  if ((st = read_status())) return st;
  int cycles = 0;
  // every cycle finishes at least one column of each segment that iterates in
  // it (or retires the segment), so max_iter bounds the cycles; the second
  // bound only guards against a cycle that makes no progress
  while (*s_any && cycles <= max_iter) {
    int prev_max = 0;
    for (int q = 0; q < ns; ++q) prev_max = std::max(prev_max, s_napp[q]);
    for (int q = 0; q < ns; ++q) done[q] = s_done[q] != 0;
    if (use_graph || nchunk <= 2) {
      for (int p = 0; p < nchunk; ++p)
        if ((st = run(p))) return st;
    } else {
      // direct launches of a long cycle: keep two chunks queued and look at the
      // active flags of the chunk before the last one queued; once no segment is
      // active the rest of the cycle is skipped (the closing step still runs)
      int32_t* act_h = hint;   // the init staging area is free again: [2][ns]
      hipEvent_t* ev = M->chunk_events();
      if (!ev) return fail(M, MHDG_ERR_HIP, "solve: events not available");
      int p = 0;
      for (; p < nchunk - 1; ++p) {
        if (p >= 2) {
          ++G.waits;
          HIP_TRY(M, hipEventSynchronize(ev[p % 2]));
          bool any = false;
          for (int q = 0; q < ns; ++q) any |= act_h[(p % 2) * ns + q] != 0;
          if (!any) break;
        }
        if ((st = seq_graph(p, s))) return st;
        HIP_TRY(M, hipMemcpyAsync(act_h + (p % 2) * ns, d.active, ns * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s));
        HIP_TRY(M, hipEventRecord(ev[p % 2], s));
      }
      if (p == nchunk - 1) {
        if ((st = seq_graph(p, s))) return st;   // last columns and the close
      } else {
        if ((st = seq_close(s))) return st;
      }
    }
    ++cycles;
    ++G.cycles;
    if ((st = read_status())) return st;
    int now_max = 0;
    for (int q = 0; q < ns; ++q) now_max = std::max(now_max, s_napp[q]);
    applies += now_max - prev_max;   // launches in which some segment took part
    count_start();
    if (g_progress) {
      double worst = 0;
      int it = 0;
      for (int q = 0; q < ns; ++q) {
        if (!s_done[q]) worst = std::max(worst, srel[q]);
        it = std::max(it, s_iters[q]);
      }
      std::fprintf(stderr, "[mhdg] gmres cycle %d, %d iterations, relative residual %.3e\n",
                   cycles, it, worst);
      std::fflush(stderr);
    }
  }
  iters.assign(ns, 0);
  rel.assign(ns, 0.0);
  rel_true.assign(ns, -1.0);
  for (int q = 0; q < ns; ++q) {
    iters[q] = s_iters[q];
    done[q] = s_done[q] != 0;
    rel[q] = bref[q] == 0.0 ? 0.0 : srel[q];
    if (true_norm) rel_true[q] = fref[q] == 0.0 ? 0.0 : srel_true[q];
  }
  return MHDG_OK;
}

mhdg_status gmres(mhdg_mesh* M, Gm& G, const double* b, const double* bref, double* x, double rtol,
                  int R, int max_iter, std::vector<int>& iters, std::vector<double>& rel,
                  int& applies, std::vector<char>& done, hipStream_t s,
                  std::vector<double>* rel_true = nullptr) {
  if (G.device) {
    std::vector<double> rt;
    mhdg_status st = gmres_device(M, G, b, bref, x, rtol, R, max_iter, iters, rel, rt, applies,
                                  done, s);
    if (rel_true) *rel_true = rt;
    return st;
  }
  return G.classic ? gmres_cgs2(M, G, b, bref, x, rtol, R, max_iter, iters, rel, applies, done, s)
                   : gmres_delayed(M, G, b, bref, x, rtol, R, max_iter, iters, rel, applies, done, s);
}

mhdg_status carve(mhdg_mesh* M, void* ws, int R, Gm& G) {
  G.nseg = M->n_inst;
  G.n = M->n_trace / M->n_inst;
  G.seg_applies.assign(G.nseg, 0);
  char* w = (char*)ws;
  const size_t vb = align_up(size_t(G.len()) * sizeof(double));
  G.ld = int64_t(vb / sizeof(double));
  G.V = (double*)w;
  G.wv = (double*)(w + vb * (R + 1));
  G.rv = (double*)(w + vb * (R + 2));
  G.fh = (double*)(w + vb * (R + 3));
  G.pf = (double*)(w + vb * (R + 4));
  G.tv = (double*)(w + vb * (R + 5));
  G.dl = (double*)(w + vb * (R + 6));
  G.cl = (double*)(w + vb * (R + 7));
  G.xin = (double*)(w + vb * (R + 8));
  size_t off = align_up(vb * (R + 9));
  G.nblk = dots_nblk(G.n);
  G.partial = (double*)(w + off);
  off += align_up(2 * size_t(G.nblk) * G.nseg * (R + 2) * sizeof(double));
  G.pq = (double*)(w + off);
  off += align_up(2 * size_t(R + 2) * G.nseg * 8);
  G.hy = (double*)(w + off);
  off += align_up(size_t(R + 2) * G.nseg * 8);
  G.coef = (double*)(w + off);
  off += align_up((2 * size_t(R) + 3) * G.nseg * 8);
  G.Hb = (double*)(w + off);
  off += align_up(size_t(R + 1) * R * G.nseg * 8);
  G.hdev = (double*)(w + off);
  off += align_up(size_t(R + 2) * G.nseg * 8);
  G.ydev = (double*)(w + off);
  off += align_up(size_t(R + 2) * G.nseg * 8);
  G.adev = (double*)(w + off);
  off += align_up(size_t(G.nseg) * 8);
  G.skip = (int32_t*)(w + off);
  off += align_up(size_t(G.nseg) * 4);
  G.U = (double*)(w + off);
  off += align_up(size_t(M->n_local) * sizeof(double));
  // device-resident GMRES state (gmres_device)
  const size_t ns = size_t(G.nseg), Rs = size_t(R);
  GmDev& d = G.dev;
  d.ns = G.nseg;
  d.Hb = G.Hb;
  d.pq = G.pq;
  d.hy = G.hy;
  d.coef = G.coef;
  d.y = G.ydev;
  d.alpha = G.adev;
  auto take = [&](size_t n_doubles) {
    double* p = (double*)(w + off);
    off += align_up(n_doubles * sizeof(double));
    return p;
  };
  d.H = take(ns * Rs * (Rs + 1));
  d.cs = take(ns * Rs);
  d.sn = take(ns * Rs);
  d.g = take(ns * (Rs + 1));
  d.hprev = take(ns * (Rs + 1));
  d.nrm = take(ns);
  d.nrm_true = take(ns);
  d.tgt = take(ns);
  d.prm = take(2 + 2 * ns);   // rtol, max_iter | bref | fref: one copy from the host
  d.bref = d.prm + 2;
  d.fref = d.prm + 2 + ns;
  // status block read back once per cycle: rel | rel_true | est, then
  // active | jc | done | iters | flag | napp | skip | any
  G.stat = w + off;
  G.stat_bytes = 3 * ns * sizeof(double) + (7 * ns + 1) * sizeof(int32_t);
  d.rel = (double*)G.stat;
  d.rel_true = d.rel + ns;
  d.est = d.rel + 2 * ns;
  int32_t* ib = (int32_t*)(G.stat + 3 * ns * sizeof(double));
  d.active = ib;
  d.jc = ib + ns;
  d.done = ib + 2 * ns;
  d.iters = ib + 3 * ns;
  d.flag = ib + 4 * ns;
  d.napp = ib + 5 * ns;
  d.skip = ib + 6 * ns;
  d.any = ib + 7 * ns;
  return MHDG_OK;
}

// Bytes of the device-resident GMRES state after the vectors (see carve).
size_t gm_dev_bytes(int R, int nseg) {
  const size_t ns = size_t(nseg), Rs = size_t(R);
  return align_up(ns * Rs * (Rs + 1) * 8) + 2 * align_up(ns * Rs * 8) +
         2 * align_up(ns * (Rs + 1) * 8) + 3 * align_up(ns * 8) + align_up((2 + 2 * ns) * 8) +
         align_up(3 * ns * 8 + (7 * ns + 1) * 4);
}

// Kernel choices of earlier autotuning runs in this process, per (local
// size, precision, log2 of the class size): later handles with the same
// shapes start from them.
// Shared by every handle of the process, so guarded by a mutex: distinct
// handles may be factored and tuned from different threads.
std::mutex& tune_mutex() {
  static std::mutex mu;
  return mu;
}
std::map<std::array<int, 3>, std::pair<int, int>>& tune_cache() {
  static std::map<std::array<int, 3>, std::pair<int, int>> m;
  return m;
}
bool tune_lookup(const std::array<int, 3>& key, std::pair<int, int>* out) {
  std::lock_guard<std::mutex> g(tune_mutex());
  auto it = tune_cache().find(key);
  if (it == tune_cache().end()) return false;
  *out = it->second;
  return true;
}
void tune_store(const std::array<int, 3>& key, std::pair<int, int> v) {
  std::lock_guard<std::mutex> g(tune_mutex());
  tune_cache()[key] = v;
}
std::array<int, 3> tune_key(const SizeClass& c, int precision) {
  int b = 0;
  while ((int64_t(1) << b) < c.count) ++b;
  return {c.N, precision, b};
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

const char* mhdg_status_string(int32_t s) {
  switch (s) {
    case MHDG_OK: return "ok";
    case MHDG_ERR_INVALID_ARG: return "invalid argument";
    case MHDG_ERR_MESH: return "invalid mesh";
    case MHDG_ERR_SINGULAR: return "singular local matrix";
    case MHDG_ERR_NOT_CONVERGED: return "not converged";
    case MHDG_ERR_WORKSPACE: return "workspace too small";
    case MHDG_ERR_HIP: return "HIP error";
    case MHDG_ERR_STATE: return "invalid call order";
    case MHDG_ERR_NONFINITE: return "non-finite local matrix";
  }
  return "unknown status";
}

const char* mhdg_last_error(const mhdg_mesh* m) { return m ? m->err.c_str() : "null handle"; }

void mhdg_destroy(mhdg_mesh* m) { delete m; }

mhdg_status mhdg_setup_macro_mesh(int64_t n_vertices, const double* xy, int64_t n_macro,
                                  const int32_t* tri, const int32_t* level, int32_t uniform_level,
                                  int32_t p, mhdg_mesh** out) {
  if (!out) return MHDG_ERR_INVALID_ARG;
  *out = nullptr;
  if (!xy || !tri || n_vertices < 3 || n_macro < 1 || p < 1 || p > 4) return MHDG_ERR_INVALID_ARG;
  if (!level && (uniform_level < 0 || uniform_level > kMaxLevel)) return MHDG_ERR_INVALID_ARG;
  if (n_macro > (int64_t(1) << 28)) return MHDG_ERR_INVALID_ARG;
  mhdg_mesh* M = new mhdg_mesh();
  M->p = p;
  M->n_vertices = n_vertices;
  M->n_macro = n_macro;
  M->xy.assign(xy, xy + 2 * n_vertices);
  M->tri.assign(tri, tri + 3 * n_macro);
  M->level.resize(n_macro);
  for (int64_t e = 0; e < n_macro; ++e) {
    int r = level ? level[e] : uniform_level;
    if (r < 0 || r > kMaxLevel) { delete M; return MHDG_ERR_INVALID_ARG; }
    M->level[e] = r;
    {
      const int P = (1 << r) * p;
      if (3 * (P + 1) * (P + 2) / 2 > 4096) { delete M; return MHDG_ERR_INVALID_ARG; }
    }
    for (int k = 0; k < 3; ++k)
      if (tri[3 * e + k] < 0 || tri[3 * e + k] >= n_vertices) { delete M; return MHDG_ERR_INVALID_ARG; }
    M->max_level = std::max(M->max_level, r);
  }
  // orientation / degeneracy
  M->macros.resize(n_macro);
  for (int64_t e = 0; e < n_macro; ++e) {
    const int32_t* t = &tri[3 * e];
    if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) { delete M; return MHDG_ERR_MESH; }
    double x0 = xy[2 * t[0]], y0 = xy[2 * t[0] + 1];
    double e1x = xy[2 * t[1]] - x0, e1y = xy[2 * t[1] + 1] - y0;
    double e2x = xy[2 * t[2]] - x0, e2y = xy[2 * t[2] + 1] - y0;
    double det = e1x * e2y - e1y * e2x;
    if (!(det > 0.0) || !std::isfinite(det)) { delete M; return MHDG_ERR_MESH; }
    MacroInfo& mi = M->macros[e];
    std::memset(&mi, 0, sizeof(mi));
    // J = [e1 e2] (columns); G = J^-1
    mi.G[0] = e2y / det;  mi.G[1] = -e2x / det;
    mi.G[2] = -e1y / det; mi.G[3] = e1x / det;
    mi.dJ = det;
    for (int k = 0; k < 3; ++k) {
      int a = t[k], b = t[(k + 1) % 3];
      double tx = xy[2 * b] - xy[2 * a], ty = xy[2 * b + 1] - xy[2 * a + 1];
      double Lk = std::sqrt(tx * tx + ty * ty);
      mi.len[k] = Lk;
      mi.nrm[2 * k] = ty / Lk;
      mi.nrm[2 * k + 1] = -tx / Lk;
    }
    int r = M->level[e];
    mi.level = r;
    mi.P = (1 << r) * p;
    mi.Q = (mi.P + 1) * (mi.P + 2) / 2;
    mi.N = 3 * mi.Q;
    mi.ld = (mi.N + 15) & ~15;   // 128-byte aligned FP64 columns
    M->max_N = std::max(M->max_N, mi.N);
  }
  // faces: unique edges sorted by (low, high)
  std::vector<std::array<int64_t, 4>> edges;  // low, high, macro, k
  edges.reserve(3 * n_macro);
  for (int64_t e = 0; e < n_macro; ++e)
    for (int k = 0; k < 3; ++k) {
      int64_t a = tri[3 * e + k], b = tri[3 * e + (k + 1) % 3];
      edges.push_back({std::min(a, b), std::max(a, b), e, k});
    }
  std::sort(edges.begin(), edges.end());
  struct FaceTmp { int64_t lo, hi; int64_t mac[2]; int k[2]; int cnt; };
  std::vector<FaceTmp> ft;
  for (size_t i = 0; i < edges.size();) {
    size_t j = i;
    while (j < edges.size() && edges[j][0] == edges[i][0] && edges[j][1] == edges[i][1]) ++j;
    if (j - i > 2) { delete M; return MHDG_ERR_MESH; }
    FaceTmp f{edges[i][0], edges[i][1], {edges[i][2], -1}, {int(edges[i][3]), -1}, int(j - i)};
    if (j - i == 2) {
      f.mac[1] = edges[i + 1][2];
      f.k[1] = int(edges[i + 1][3]);
      // a shared edge must be traversed in opposite directions (conforming, consistently oriented)
      int64_t e0 = f.mac[0], e1 = f.mac[1];
      int d0 = tri[3 * e0 + f.k[0]] < tri[3 * e0 + (f.k[0] + 1) % 3];
      int d1 = tri[3 * e1 + f.k[1]] < tri[3 * e1 + (f.k[1] + 1) % 3];
      if (d0 == d1) { delete M; return MHDG_ERR_MESH; }
    }
    ft.push_back(f);
    i = j;
  }
  M->n_faces = (int64_t)ft.size();
  int64_t tr = 0, gb = 0, ld = 0;
  for (size_t fi = 0; fi < ft.size(); ++fi) {
    FaceTmp& f = ft[fi];
    int lev = M->level[f.mac[0]];
    if (f.cnt == 2) lev = std::max(lev, M->level[f.mac[1]]);
    int nF = (1 << lev) * p + 1;
    double dx = xy[2 * f.hi] - xy[2 * f.lo], dy = xy[2 * f.hi + 1] - xy[2 * f.lo + 1];
    double len = std::sqrt(dx * dx + dy * dy);
    for (int s = 0; s < f.cnt; ++s) {
      MacroInfo& mi = M->macros[f.mac[s]];
      int k = f.k[s];
      mi.face[k] = (int32_t)fi;
      mi.orient[k] = tri[3 * f.mac[s] + k] < tri[3 * f.mac[s] + (k + 1) % 3] ? 1 : -1;
      mi.flevel[k] = lev;
      mi.tr_off[k] = -1;
      mi.bnd_face[k] = -1;
      mi.slot_off[k] = -1;
    }
    if (f.cnt == 2) {
      FaceInfo fi2{};
      fi2.len = len;
      fi2.tr_off = (int32_t)tr;
      fi2.nF = nF;
      fi2.level = lev;
      int a = f.mac[0] < f.mac[1] ? 0 : 1;
      for (int s = 0; s < 2; ++s) {
        MacroInfo& mi = M->macros[f.mac[s]];
        mi.tr_off[f.k[s]] = (int32_t)tr;
      }
      // slots assigned below; remember macro/edge pairs
      fi2.slot[0] = f.mac[a] * 3 + f.k[a];
      fi2.slot[1] = f.mac[1 - a] * 3 + f.k[1 - a];
      M->faces.push_back(fi2);
      tr += nF;
    } else {
      BndFaceInfo b{};
      b.len = len;
      b.g_off = gb;
      b.lam_off = ld;
      b.nF = nF;
      b.level = lev;
      M->macros[f.mac[0]].bnd_face[f.k[0]] = (int32_t)M->bfaces.size();
      M->bfaces.push_back(b);
      gb += int64_t(1 << lev) * (p + 2);
      ld += nF;
    }
  }
  M->n_int = (int64_t)M->faces.size();
  M->n_bnd = (int64_t)M->bfaces.size();
  M->n_trace = tr;
  M->n_bnd_points = gb;
  M->n_lamD = ld;
  // offsets
  int64_t lo = 0, no = 0, so = 0;
  for (int64_t e = 0; e < n_macro; ++e) {
    MacroInfo& mi = M->macros[e];
    mi.loc_off = lo;
    mi.node_off = no;
    lo += mi.N;
    no += mi.Q;
    for (int k = 0; k < 3; ++k)
      if (mi.tr_off[k] >= 0) {
        mi.slot_off[k] = so;
        so += (1 << mi.flevel[k]) * p + 1;
      }
  }
  M->n_local = lo;
  M->n_nodes = no;
  M->n_slots = so;
  for (auto& f : M->faces) {
    int64_t e0 = f.slot[0] / 3, k0 = f.slot[0] % 3, e1 = f.slot[1] / 3, k1 = f.slot[1] % 3;
    f.slot[0] = M->macros[e0].slot_off[k0];
    f.slot[1] = M->macros[e1].slot_off[k1];
  }
  // processing order: largest local size first (stable), factor offsets in that order
  M->order.resize(n_macro);
  for (int64_t e = 0; e < n_macro; ++e) M->order[e] = (int32_t)e;
  std::stable_sort(M->order.begin(), M->order.end(),
                   [&](int32_t a, int32_t b) { return M->macros[a].N > M->macros[b].N; });
  for (int64_t i = 0; i < n_macro;) {
    const int N = M->macros[M->order[i]].N;
    int64_t j = i;
    while (j < n_macro && M->macros[M->order[j]].N == N) ++j;
    M->classes.push_back({N, M->macros[M->order[i]].P, i, j - i});
    i = j;
  }
  int64_t fo = 0;
  for (int64_t e = 0; e < n_macro; ++e) {
    MacroInfo& mi = M->macros[e];
    mi.fac_off = fo;
    fo += int64_t(mi.N) * mi.ld;
    fo = (fo + 63) & ~int64_t(63);
  }
  build_templates(M);
  M->one = {M->n_macro, M->n_faces, M->n_int, M->n_bnd, M->n_trace, M->n_nodes, M->n_local,
            M->n_bnd_points, M->n_slots, M->n_lamD, fo, M->macros, M->faces, M->bfaces,
            M->order, M->classes};
  *out = M;
  return MHDG_OK;
}

mhdg_status mhdg_set_instances(mhdg_mesh* M, int32_t n_inst) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  const auto& o = M->one;
  if (n_inst < 1 || int64_t(n_inst) * o.n_macro > (int64_t(1) << 28) ||
      int64_t(n_inst) * o.n_trace > INT32_MAX)
    return fail(M, MHDG_ERR_INVALID_ARG, "set_instances: instance count out of range");
  M->factored = false;
  M->have_rhs = false;
  M->tm_plan.reset();
  M->folded = false;
  M->assembled = false;
  M->bcond = false;
  M->ws = nullptr;
  M->drop_graphs();
  M->n_inst = n_inst;
  M->n_macro = o.n_macro * n_inst;
  M->n_faces = o.n_faces * n_inst;
  M->n_int = o.n_int * n_inst;
  M->n_bnd = o.n_bnd * n_inst;
  M->n_trace = o.n_trace * n_inst;
  M->n_nodes = o.n_nodes * n_inst;
  M->n_local = o.n_local * n_inst;
  M->n_bnd_points = o.n_bnd_points * n_inst;
  M->n_slots = o.n_slots * n_inst;
  M->n_lamD = o.n_lamD * n_inst;
  M->macros.resize(M->n_macro);
  M->faces.resize(M->n_int);
  M->bfaces.resize(M->n_bnd);
  for (int32_t i = 0; i < n_inst; ++i) {
    for (int64_t e = 0; e < o.n_macro; ++e) {
      MacroInfo mi = o.macros[e];
      mi.inst = i;
      mi.fac_off += i * o.fac_total;
      mi.loc_off += i * o.n_local;
      mi.node_off += i * o.n_nodes;
      for (int k = 0; k < 3; ++k) {
        mi.face[k] += int32_t(i * o.n_faces);
        if (mi.slot_off[k] >= 0) mi.slot_off[k] += i * o.n_slots;
        if (mi.tr_off[k] >= 0) mi.tr_off[k] += int32_t(i * o.n_trace);
        if (mi.bnd_face[k] >= 0) mi.bnd_face[k] += int32_t(i * o.n_bnd);
      }
      M->macros[i * o.n_macro + e] = mi;
    }
    for (int64_t f = 0; f < o.n_int; ++f) {
      FaceInfo fi = o.faces[f];
      fi.inst = i;
      fi.slot[0] += i * o.n_slots;
      fi.slot[1] += i * o.n_slots;
      fi.tr_off += int32_t(i * o.n_trace);
      M->faces[i * o.n_int + f] = fi;
    }
    for (int64_t f = 0; f < o.n_bnd; ++f) {
      BndFaceInfo b = o.bfaces[f];
      b.g_off += i * o.n_bnd_points;
      b.lam_off += i * o.n_lamD;
      M->bfaces[i * o.n_bnd + f] = b;
    }
  }
  // one launch per size class covers every instance
  M->order.clear();
  M->classes.clear();
  for (const SizeClass& c : o.classes) {
    SizeClass c2 = c;
    c2.start = (int64_t)M->order.size();
    c2.count = c.count * n_inst;
    for (int32_t i = 0; i < n_inst; ++i)
      for (int64_t j = 0; j < c.count; ++j)
        M->order.push_back(int32_t(o.order[c.start + j] + i * o.n_macro));
    M->classes.push_back(c2);
  }
  return MHDG_OK;
}

mhdg_status mhdg_profile(mhdg_mesh* M, int32_t enable, mhdg_kernel_times* out) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (out) std::memset(out, 0, sizeof(*out));
  for (int k = 0; k < 6; ++k) {
    for (auto& p : M->ev[k]) {
      if (!enable && out) {
        HIP_TRY(M, hipEventSynchronize(p.second));
        float ms = 0.f;
        HIP_TRY(M, hipEventElapsedTime(&ms, p.first, p.second));
        out->count[k] += 1;
        out->ms[k] += ms;
      }
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    M->ev[k].clear();
  }
  M->prof = enable != 0;
  return MHDG_OK;
}

mhdg_status mhdg_query(const mhdg_mesh* M, int32_t precision, int32_t restart, mhdg_sizes* out) {
  if (!M || !out || restart < 1 ||
      (precision != MHDG_FP64 && precision != MHDG_FP32 && precision != MHDG_BF16 &&
       precision != MHDG_QELIM))
    return MHDG_ERR_INVALID_ARG;
  out->n_macro = M->n_macro;
  out->n_faces = M->n_faces;
  out->n_interior_faces = M->n_int;
  out->n_trace = M->n_trace;
  out->n_nodes = M->n_nodes;
  out->n_local = M->n_local;
  out->n_bnd_points = M->n_bnd_points;
  out->p = M->p;
  out->max_level = M->max_level;
  out->max_local = M->max_N;
  out->n_instances = M->n_inst;
  out->fold_ws_bytes = fold_layout(M).total;
  FactorLayout L = factor_layout(M, precision);
  out->factor_ws_bytes = L.total;
  out->solve_ws_bytes = solve_bytes(M, restart);
  return MHDG_OK;
}

mhdg_status mhdg_sample_points(const mhdg_mesh* M, double* node_xy, double* bnd_xy) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  const auto& one = M->one;
  if (node_xy) {
    int64_t o = 0;
    for (int64_t e = 0; e < one.n_macro; ++e) {
      const MacroInfo& mi = M->macros[e];
      const int32_t* t = &M->tri[3 * e];
      double x0 = M->xy[2 * t[0]], y0 = M->xy[2 * t[0] + 1];
      double e1x = M->xy[2 * t[1]] - x0, e1y = M->xy[2 * t[1] + 1] - y0;
      double e2x = M->xy[2 * t[2]] - x0, e2y = M->xy[2 * t[2] + 1] - y0;
      for (int j = 0; j <= mi.P; ++j)
        for (int i = 0; i <= mi.P - j; ++i) {
          double a = double(i) / mi.P, b = double(j) / mi.P;
          node_xy[2 * o] = x0 + a * e1x + b * e2x;
          node_xy[2 * o + 1] = y0 + a * e1y + b * e2y;
          ++o;
        }
    }
  }
  if (bnd_xy) {
    std::vector<double> t, w;
    gauss_legendre01(M->p + 2, t, w);
    // boundary faces in sorted order = order of bfaces
    std::vector<std::pair<int64_t, int64_t>> fv(one.n_faces);
    for (int64_t e = 0; e < one.n_macro; ++e)
      for (int k = 0; k < 3; ++k) {
        int64_t a = M->tri[3 * e + k], b = M->tri[3 * e + (k + 1) % 3];
        fv[one.macros[e].face[k]] = {std::min(a, b), std::max(a, b)};
      }
    std::vector<int32_t> bface_of(one.n_faces, -1);
    for (int64_t e = 0; e < one.n_macro; ++e)
      for (int k = 0; k < 3; ++k)
        if (one.macros[e].bnd_face[k] >= 0) bface_of[one.macros[e].face[k]] = one.macros[e].bnd_face[k];
    for (int64_t f = 0; f < one.n_faces; ++f) {
      if (bface_of[f] < 0) continue;
      const BndFaceInfo& b = one.bfaces[bface_of[f]];
      double ax = M->xy[2 * fv[f].first], ay = M->xy[2 * fv[f].first + 1];
      double bx = M->xy[2 * fv[f].second], by = M->xy[2 * fv[f].second + 1];
      int npc = 1 << b.level;
      int64_t o = b.g_off;
      for (int c = 0; c < npc; ++c)
        for (size_t q = 0; q < t.size(); ++q) {
          double s = (c + t[q]) / npc;
          bnd_xy[2 * o] = ax + s * (bx - ax);
          bnd_xy[2 * o + 1] = ay + s * (by - ay);
          ++o;
        }
    }
  }
  // every instance samples at the same points
  for (int32_t i = 1; i < M->n_inst; ++i) {
    if (node_xy)
      std::memcpy(node_xy + 2 * i * one.n_nodes, node_xy, 2 * one.n_nodes * sizeof(double));
    if (bnd_xy)
      std::memcpy(bnd_xy + 2 * i * one.n_bnd_points, bnd_xy, 2 * one.n_bnd_points * sizeof(double));
  }
  return MHDG_OK;
}

mhdg_status mhdg_factor_local(mhdg_mesh* M, const double* kappa, double beta_x, double beta_y,
                              double tau, int32_t precision, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  std::vector<double> beta(2 * size_t(M->n_inst));
  for (int32_t i = 0; i < M->n_inst; ++i) { beta[2 * i] = beta_x; beta[2 * i + 1] = beta_y; }
  return mhdg_factor_local_batched(M, kappa, beta.data(), tau, precision, ws, ws_bytes, stream);
}

mhdg_status mhdg_factor_local_batched(mhdg_mesh* M, const double* kappa, const double* beta,
                                      double tau, int32_t precision, void* ws, size_t ws_bytes,
                                      void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!kappa || !ws || !beta)
    return fail(M, MHDG_ERR_INVALID_ARG, "factor_local: null pointer");
  if (!(tau > 0.0) || !std::isfinite(tau))
    return fail(M, MHDG_ERR_INVALID_ARG, "factor_local: tau must be finite and > 0");
  for (int64_t i = 0; i < 2 * int64_t(M->n_inst); ++i)
    if (!std::isfinite(beta[i])) return fail(M, MHDG_ERR_INVALID_ARG, "factor_local: non-finite a");
  if (precision != MHDG_FP64 && precision != MHDG_FP32 && precision != MHDG_BF16 &&
      precision != MHDG_QELIM)
    return fail(M, MHDG_ERR_INVALID_ARG, "factor_local: unknown precision");
  if (precision == MHDG_BF16 && M->max_N > 1024)
    return fail(M, MHDG_ERR_INVALID_ARG, "factor_local: BF16 factors support N_K <= 1024");
  if (precision == MHDG_QELIM)
    for (auto& c : M->classes)
      if (c.N / 3 > 1237 || qelim_lds_bytes(c.N / 3, c.P) > 65536)
        return fail(M, MHDG_ERR_INVALID_ARG, "factor_local: flux elimination supports Q <= 1237");
  mhdg_sizes sz;
  mhdg_query(M, precision, 1, &sz);
  if (ws_bytes < sz.factor_ws_bytes)
    return fail(M, MHDG_ERR_WORKSPACE, "factor_local: workspace smaller than mhdg_query reports");
  hipStream_t s = (hipStream_t)stream;
  M->factored = false;
  M->have_rhs = false;
  M->folded = false;
  M->assembled = false;
  M->bcond = false;
  M->drop_graphs();
  M->precision = precision;
  M->tau = tau;
  M->ws = (char*)ws;
  M->ws_bytes = ws_bytes;
  for (auto& mi : M->macros) { mi.bx = beta[2 * mi.inst]; mi.by = beta[2 * mi.inst + 1]; }
  if (precision == MHDG_QELIM) {
    qelim_offsets(M->macros);
    build_qelim_templates(M);
  }
  M->L = factor_layout(M, precision);
  for (auto& c : M->classes)
    if (!c.lu_var && !c.solve_var) {
      std::pair<int, int> v;
      if (tune_lookup(tune_key(c, precision), &v)) { c.lu_var = v.first; c.solve_var = v.second; }
    }
  FactorLayout& L = M->L;
  char* w = M->ws;
  HIP_TRY(M, hipMemcpyAsync(w + L.meta, M->macros.data(), M->macros.size() * sizeof(MacroInfo),
                            hipMemcpyHostToDevice, s));
  if (!M->faces.empty())
    HIP_TRY(M, hipMemcpyAsync(w + L.faces, M->faces.data(), M->faces.size() * sizeof(FaceInfo),
                              hipMemcpyHostToDevice, s));
  if (!M->bfaces.empty())
    HIP_TRY(M, hipMemcpyAsync(w + L.bfaces, M->bfaces.data(), M->bfaces.size() * sizeof(BndFaceInfo),
                              hipMemcpyHostToDevice, s));
  HIP_TRY(M, hipMemcpyAsync(w + L.tmpl, M->tmpl.data(), M->tmpl.size() * sizeof(double),
                            hipMemcpyHostToDevice, s));
  HIP_TRY(M, hipMemcpyAsync(w + L.order, M->order.data(), M->order.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
  // the macro order lives after the permutation vector region: reuse status region size n_macro
  MacroInfo* info = (MacroInfo*)(w + L.meta);
  // kappa is read on the device; every value must be finite and > 0 before any
  // block is assembled or factored
  {
    HIP_TRY(M, launch_set_kappa(info, kappa, M->n_macro, (int32_t*)(w + L.status), s));
    std::vector<int32_t> bad(M->n_macro);
    HIP_TRY(M, hipMemcpyAsync(bad.data(), w + L.status, bad.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(M, hipStreamSynchronize(s));
    for (int64_t e = 0; e < M->n_macro; ++e)
      if (bad[e]) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "factor_local: kappa of macro %lld is not finite and > 0 (first such macro)",
                 (long long)e);
        return fail(M, MHDG_ERR_INVALID_ARG, buf);
      }
  }
  if (precision == MHDG_QELIM) {
    // the Schur block on u per macro, factored by the same LU kernels through a
    // table whose N / ld / offsets describe the Q x Q blocks
    HIP_TRY(M, hipMemcpyAsync(w + L.qtmpl, M->qtmpl.data(), M->qtmpl.size() * sizeof(double),
                              hipMemcpyHostToDevice, s));
    std::vector<MacroInfo> lu_info(M->macros);
    int maxQ = 0;
    for (auto& mi : lu_info) {
      maxQ = std::max(maxQ, mi.Q);
      mi.N = mi.Q;
      mi.ld = mi.sld;
      mi.fac_off = mi.sfac_off;
      mi.loc_off = mi.sperm_off;
    }
    std::vector<SizeClass> lu_classes(M->classes);
    for (auto& c : lu_classes) { c.N /= 3; c.lu_var = 0; c.solve_var = 0; }
    HIP_TRY(M, hipMemcpyAsync(w + L.info_lu, lu_info.data(), lu_info.size() * sizeof(MacroInfo),
                              hipMemcpyHostToDevice, s));
    {
      ProfScope ps(M, 0, s);
      HIP_TRY(M, launch_qelim_assemble((double*)(w + L.factors), info, M->n_macro, maxQ,
                                       (const double*)(w + L.tmpl), M->T,
                                       (const double*)(w + L.qtmpl), M->QT, tau, s));
    }
    {
      ProfScope ps(M, 1, s);
      HIP_TRY(M, launch_lu(w + L.factors, MHDG_FP64, (const MacroInfo*)(w + L.info_lu),
                           (const int32_t*)(w + L.order), lu_classes.data(),
                           (int)lu_classes.size(), (int32_t*)(w + L.perm),
                           (int32_t*)(w + L.status),
                           lu_scratch(M), lu_scratch_bytes(M), s));
    }
    // the host vectors above must outlive the copies
    HIP_TRY(M, hipStreamSynchronize(s));
  } else {
    {
      ProfScope ps(M, 0, s);
      HIP_TRY(M, launch_assemble(w + L.factors, lu_precision(precision), info, nullptr, M->n_macro,
                                 (const double*)(w + L.tmpl), M->T, tau, s));
    }
    {
      ProfScope ps(M, 1, s);
      HIP_TRY(M, launch_lu(w + L.factors, lu_precision(precision), info, (const int32_t*)(w + L.order),
                           M->classes.data(), (int)M->classes.size(), (int32_t*)(w + L.perm),
                           (int32_t*)(w + L.status),
                           lu_scratch(M), lu_scratch_bytes(M), s));
    }
  }
  if (precision == MHDG_BF16) {
    const MacroInfo& last = M->macros.back();
    const int64_t nf = last.fac_off + int64_t(last.N) * last.ld;
    HIP_TRY(M, launch_to_bf16((const float*)(w + L.factors), w + L.factors16, nf, s));
  }
  std::vector<int32_t> st(M->n_macro);
  HIP_TRY(M, hipMemcpyAsync(st.data(), w + L.status, st.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
  HIP_TRY(M, hipStreamSynchronize(s));
  for (int64_t e = 0; e < M->n_macro; ++e)
    if (st[e] != 0) {
      char buf[160];
      if (st[e] > 0) {
        snprintf(buf, sizeof buf, "factor_local: zero pivot in macro %lld at column %d",
                 (long long)e, st[e] - 1);
        return fail(M, MHDG_ERR_SINGULAR, buf);
      }
      snprintf(buf, sizeof buf, "factor_local: non-finite pivot in macro %lld at column %d",
               (long long)e, -st[e] - 1);
      return fail(M, MHDG_ERR_NONFINITE, buf);
    }
  M->factored = true;
  return MHDG_OK;
}

mhdg_status mhdg_fold_operator(mhdg_mesh* M, void* ws, size_t ws_bytes, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored || (M->precision != MHDG_FP64 && M->precision != MHDG_QELIM))
    return fail(M, MHDG_ERR_STATE, "fold_operator: needs FP64 factors (call factor_local first)");
  const FoldLayout F = fold_layout(M);
  if (!ws || ws_bytes < F.total)
    return fail(M, MHDG_ERR_WORKSPACE, "fold_operator: workspace smaller than mhdg_query reports");
  hipStream_t s = (hipStream_t)stream;
  char* fw = (char*)ws;
  // per-macro offsets of T_K
  std::vector<int64_t> toff(M->n_macro);
  int64_t o = 0;
  int maxL = 0;
  for (int64_t e = 0; e < M->n_macro; ++e) {
    toff[e] = o;
    const int L = fold_L(M, M->macros[e]);
    maxL = std::max(maxL, L);
    o += int64_t(L) * L;
  }
  if (maxL > kFoldMaxL) return fail(M, MHDG_ERR_INVALID_ARG, "fold_operator: macro trace too large");
  HIP_TRY(M, hipMemcpyAsync(fw + F.toff, toff.data(), toff.size() * 8, hipMemcpyHostToDevice, s));
  FactorLayout& L = M->L;
  char* w = M->ws;
  double* T = (double*)(fw + F.T);
  if (maxL > 0 && M->precision == MHDG_QELIM)
    HIP_TRY(M, launch_qelim_fold_build((const double*)(w + L.factors), (const MacroInfo*)(w + L.meta),
                                       (const int32_t*)(w + L.order), M->classes.data(),
                                       (int)M->classes.size(), (const int32_t*)(w + L.perm),
                                       (const double*)(w + L.tmpl), M->T,
                                       (const double*)(w + L.qtmpl), M->QT, M->tau, maxL,
                                       (const int64_t*)(fw + F.toff), T, s));
  else if (maxL > 0)
    HIP_TRY(M, launch_fold_build((const double*)(w + L.factors), (const MacroInfo*)(w + L.meta),
                                 (const int32_t*)(w + L.order), M->classes.data(),
                                 (int)M->classes.size(), (const int32_t*)(w + L.perm),
                                 (const double*)(w + L.tmpl), M->T, M->tau, maxL,
                                 (const int64_t*)(fw + F.toff), T, s));
  HIP_TRY(M, hipStreamSynchronize(s));
  M->fold_toff = (int64_t*)(fw + F.toff);
  M->fold_T = T;
  M->fold_maxL = maxL;
  M->folded = true;
  M->assembled = false;
  M->drop_graphs();
  return MHDG_OK;
}

size_t mhdg_trace_matrix_ws_bytes(const mhdg_mesh* M) {
  if (!M) return 0;
  return trace_plan_cached(M).total;
}

mhdg_status mhdg_assemble_trace_matrix(mhdg_mesh* M, void* ws, size_t ws_bytes, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->folded)
    return fail(M, MHDG_ERR_STATE, "assemble_trace_matrix: needs mhdg_fold_operator first");
  if (M->n_int > 0 && M->faces[0].nF > 0)
    for (const FaceInfo& f : M->faces)
      if (f.nF > (1 << kMaxLevel) * 4 + 1)
        return fail(M, MHDG_ERR_INVALID_ARG, "assemble_trace_matrix: face trace too large");
  const TracePlan& P = trace_plan_cached(M);
  for (size_t r = 0; r + 1 < P.row_ptr.size(); ++r)
    if (P.row_ptr[r + 1] - P.row_ptr[r] > 5)   // the product kernel gathers at most 5 blocks
      return fail(M, MHDG_ERR_INVALID_ARG, "assemble_trace_matrix: a face row with more than 5 blocks");
  if (!ws || ws_bytes < P.total)
    return fail(M, MHDG_ERR_WORKSPACE,
                "assemble_trace_matrix: workspace smaller than mhdg_trace_matrix_ws_bytes");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  HIP_TRY(M, hipMemcpyAsync(w + P.off_row, P.row_ptr.data(), P.row_ptr.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
  HIP_TRY(M, hipMemcpyAsync(w + P.off_blk, P.blocks.data(), P.blocks.size() * sizeof(TraceBlock),
                            hipMemcpyHostToDevice, s));
  FactorLayout& L = M->L;
  HIP_TRY(M, launch_trace_matrix_build((const TraceBlock*)(w + P.off_blk), int64_t(P.blocks.size()),
                                       (const FaceInfo*)(M->ws + L.faces),
                                       (const double*)(M->ws + L.tmpl), M->T, M->tau, M->fold_T,
                                       (double*)(w + P.off_val), (double*)(w + P.off_pval), s));
  HIP_TRY(M, hipStreamSynchronize(s));   // the one documented synchronisation
  M->tm_row_ptr = (const int32_t*)(w + P.off_row);
  M->tm_blocks = (const TraceBlock*)(w + P.off_blk);
  M->tm_values = (const double*)(w + P.off_val);
  M->tm_pvalues = (const double*)(w + P.off_pval);
  M->tm_n_blocks = int64_t(P.blocks.size());
  M->tm_n_values = P.n_values;
  M->tm_max_nF = 0;
  for (int64_t fi = 0; fi < M->n_int; ++fi) M->tm_max_nF = std::max(M->tm_max_nF, M->faces[fi].nF);
  M->assembled = true;
  M->drop_graphs();
  return MHDG_OK;
}

size_t mhdg_boundary_ws_bytes(const mhdg_mesh* M) {
  if (!M) return 0;
  return boundary_layout(M).total;
}

mhdg_status mhdg_condense_boundary(mhdg_mesh* M, void* ws, size_t ws_bytes, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored || (M->precision != MHDG_FP64 && M->precision != MHDG_QELIM))
    return fail(M, MHDG_ERR_STATE,
                "condense_boundary: needs MHDG_FP64 or MHDG_QELIM factors (call factor_local first)");
  const BoundaryLayout B = boundary_layout(M);
  if (!ws || ws_bytes < B.total)
    return fail(M, MHDG_ERR_WORKSPACE, "condense_boundary: workspace smaller than mhdg_boundary_ws_bytes");
  std::vector<int64_t> off(M->n_macro);
  int64_t o = 0;
  int maxP = 0;
  for (int64_t e = 0; e < M->n_macro; ++e) {
    off[e] = o;
    const int P = M->macros[e].P;
    maxP = std::max(maxP, P);
    o += 81 * int64_t(P) * P;
  }
  if (9 * maxP > 512)
    return fail(M, MHDG_ERR_INVALID_ARG, "condense_boundary: macro boundary larger than 512 unknowns");
  hipStream_t s = (hipStream_t)stream;
  char* bw = (char*)ws;
  HIP_TRY(M, hipMemcpyAsync(bw + B.off, off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
  FactorLayout& L = M->L;
  char* w = M->ws;
  double* W = (double*)(bw + B.W);
  if (M->n_macro > 0 && M->precision == MHDG_QELIM)
    HIP_TRY(M, launch_qelim_bc_build((const double*)(w + L.factors), (const MacroInfo*)(w + L.meta),
                                     (const int32_t*)(w + L.order), M->classes.data(),
                                     (int)M->classes.size(), (const int32_t*)(w + L.perm),
                                     (const double*)(w + L.tmpl), M->T,
                                     (const double*)(w + L.qtmpl), M->QT, M->tau,
                                     (const int64_t*)(bw + B.off), W, s));
  else if (M->n_macro > 0)
    HIP_TRY(M, launch_bc_build((const double*)(w + L.factors), (const MacroInfo*)(w + L.meta),
                               (const int32_t*)(w + L.order), M->classes.data(),
                               (int)M->classes.size(), (const int32_t*)(w + L.perm),
                               (const double*)(w + L.tmpl), M->T, (const int64_t*)(bw + B.off), W,
                               s));
  HIP_TRY(M, hipStreamSynchronize(s));   // the host offset table is freed on return
  M->bc_off = (const int64_t*)(bw + B.off);
  M->bc_W = W;
  M->bc_maxP = maxP;
  M->bcond = true;
  M->drop_graphs();
  return MHDG_OK;
}

mhdg_status mhdg_set_supg(mhdg_mesh* M, int32_t on) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (on != 0 && on != 1) return fail(M, MHDG_ERR_INVALID_ARG, "set_supg: on must be 0 or 1");
  if (on) build_supg_templates(M);
  auto mark = [&](std::vector<MacroInfo>& v) {
    for (auto& mi : v)
      mi.hsupg = on ? std::max(mi.len[0], std::max(mi.len[1], mi.len[2])) / double(1 << mi.level)
                    : 0.0;
  };
  mark(M->macros);
  mark(M->one.macros);
  M->supg = on != 0;
  M->factored = false;
  M->have_rhs = false;
  M->folded = false;
  M->assembled = false;
  M->bcond = false;
  M->drop_graphs();
  return MHDG_OK;
}

mhdg_status mhdg_set_kernel_variant(mhdg_mesh* M, int32_t N, int32_t lu_variant,
                                    int32_t solve_variant) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if ((lu_variant && !lu_variant_ok(lu_variant, N)) ||
      (solve_variant && !solve_variant_ok(solve_variant, N)))
    return fail(M, MHDG_ERR_INVALID_ARG, "set_kernel_variant: variant not available for this size");
  bool found = false;
  for (auto* cl : {&M->classes, &M->one.classes})
    for (auto& c : *cl)
      if (c.N == N) { c.lu_var = lu_variant; c.solve_var = solve_variant; found = true; }
  if (!found) return fail(M, MHDG_ERR_INVALID_ARG, "set_kernel_variant: no macros of that size");
  M->drop_graphs();
  return MHDG_OK;
}

mhdg_status mhdg_autotune(mhdg_mesh* M, int32_t flags, mhdg_tune_report* out, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored) return fail(M, MHDG_ERR_STATE, "autotune: call factor_local first");
  if (M->precision == MHDG_QELIM)
    return fail(M, MHDG_ERR_STATE, "autotune: not available for the flux-eliminated form");
  if (M->classes.size() > MHDG_MAX_CLASSES)
    return fail(M, MHDG_ERR_INVALID_ARG, "autotune: too many size classes");
  hipStream_t s = (hipStream_t)stream;
  FactorLayout& L = M->L;
  char* w = M->ws;
  MacroInfo* info = (MacroInfo*)(w + L.meta);
  const double* tm = (const double*)(w + L.tmpl);
  const int32_t* order = (const int32_t*)(w + L.order);
  hipEvent_t b, e;
  HIP_TRY(M, hipEventCreate(&b));
  HIP_TRY(M, hipEventCreate(&e));
  struct Ev {
    hipEvent_t b, e;
    ~Ev() { (void)hipEventDestroy(b); (void)hipEventDestroy(e); }
  } ev{b, e};
  mhdg_tune_report rep{};
  rep.n_classes = (int32_t)M->classes.size();
  auto elapsed = [&](float& ms) -> mhdg_status {
    HIP_TRY(M, hipEventSynchronize(e));
    HIP_TRY(M, hipEventElapsedTime(&ms, b, e));
    return MHDG_OK;
  };
  mhdg_status st;
  for (size_t ci = 0; ci < M->classes.size(); ++ci) {
    SizeClass& c = M->classes[ci];
    rep.N[ci] = c.N;
    rep.count[ci] = c.count;
    if (flags & MHDG_TUNE_LU) {
      // a subset of the class large enough to fill the device; the factors
      // it leaves are rebuilt below
      SizeClass sub = c;
      sub.count = std::min<int64_t>(c.count, 512);
      int best = 0;
      double best_ms = 0;
      for (int v = LU_PANEL; v <= LU_SPLIT; ++v) {
        if (!lu_variant_ok(v, c.N)) continue;
        sub.lu_var = v;
        SizeClass one_m = sub;
        one_m.count = 1;   // untimed: loads the kernel
        HIP_TRY(M, launch_lu(w + L.factors, lu_precision(M->precision), info, order, &one_m, 1,
                             (int32_t*)(w + L.perm), (int32_t*)(w + L.status),
                           lu_scratch(M), lu_scratch_bytes(M), s));
        HIP_TRY(M, launch_assemble(w + L.factors, lu_precision(M->precision), info, nullptr, M->n_macro, tm,
                                   M->T, M->tau, s));
        HIP_TRY(M, hipEventRecord(b, s));
        HIP_TRY(M, launch_lu(w + L.factors, lu_precision(M->precision), info, order, &sub, 1,
                             (int32_t*)(w + L.perm), (int32_t*)(w + L.status),
                           lu_scratch(M), lu_scratch_bytes(M), s));
        HIP_TRY(M, hipEventRecord(e, s));
        float ms = 0;
        if ((st = elapsed(ms))) return st;
        rep.lu_ms[ci][v] = ms;
        if (!best || ms < best_ms) { best = v; best_ms = ms; }
      }
      c.lu_var = best;
    }
    rep.lu_variant[ci] = c.lu_var ? c.lu_var : default_lu_variant(c.N);
  }
  // valid factors with the chosen LU variants
  HIP_TRY(M, launch_assemble(w + L.factors, lu_precision(M->precision), info, nullptr, M->n_macro,
                             tm, M->T, M->tau, s));
  HIP_TRY(M, launch_lu(w + L.factors, lu_precision(M->precision), info, order, M->classes.data(),
                       (int)M->classes.size(), (int32_t*)(w + L.perm), (int32_t*)(w + L.status),
                           lu_scratch(M), lu_scratch_bytes(M), s));
  if (M->precision == MHDG_BF16) {
    const MacroInfo& last = M->macros.back();
    HIP_TRY(M, launch_to_bf16((const float*)(w + L.factors), w + L.factors16,
                              last.fac_off + int64_t(last.N) * last.ld, s));
  }
  {
    std::vector<int32_t> stv(M->n_macro);
    HIP_TRY(M, hipMemcpyAsync(stv.data(), w + L.status, stv.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(M, hipStreamSynchronize(s));
    for (int32_t v : stv)
      if (v) return fail(M, MHDG_ERR_SINGULAR, "autotune: zero pivot while refactoring");
  }
  // apply solves: every class with each candidate, trace input zero (timing only)
  double* lam0 = (double*)(w + L.work1);
  HIP_TRY(M, hipMemsetAsync(lam0, 0, size_t(M->n_local) * sizeof(double), s));
  for (size_t ci = 0; ci < M->classes.size(); ++ci) {
    SizeClass& c = M->classes[ci];
    if (flags & MHDG_TUNE_SOLVE) {
      SizeClass sub = c;
      int best = 0;
      double best_ms = 0;
      for (int v = SOLVE_WAVE; v <= SOLVE_WAVE4_LG16; ++v) {
        if (!solve_variant_ok(v, c.N)) continue;
        if (M->precision == MHDG_BF16 && v != SOLVE_WAVE) continue;   // BF16: one wavefront
        sub.solve_var = v;
        HIP_TRY(M, launch_macro_solve(MODE_APPLY, 0, solve_factors(M), M->precision, info, order, &sub,
                                      1, (const int32_t*)(w + L.perm), tm, M->T, nullptr, M->tau,
                                      lam0, nullptr, nullptr, (double*)(w + L.slots), s));
        HIP_TRY(M, hipEventRecord(b, s));
        for (int r = 0; r < 3; ++r)
          HIP_TRY(M, launch_macro_solve(MODE_APPLY, 0, solve_factors(M), M->precision, info, order,
                                        &sub, 1, (const int32_t*)(w + L.perm), tm, M->T, nullptr,
                                        M->tau, lam0, nullptr, nullptr, (double*)(w + L.slots), s));
        HIP_TRY(M, hipEventRecord(e, s));
        float ms = 0;
        if ((st = elapsed(ms))) return st;
        rep.apply_ms[ci][v] = ms / 3;
        if (!best || ms < best_ms) { best = v; best_ms = ms; }
      }
      c.solve_var = best;
    }
    rep.solve_variant[ci] = c.solve_var ? c.solve_var : default_solve_variant(c.N);
    tune_store(tune_key(c, M->precision), {c.lu_var, c.solve_var});
    for (auto& oc : M->one.classes)
      if (oc.N == c.N) { oc.lu_var = c.lu_var; oc.solve_var = c.solve_var; }
  }
  M->drop_graphs();
  if (out) *out = rep;
  return MHDG_OK;
}

mhdg_status mhdg_local_matrix(mhdg_mesh* M, int64_t e, double* dst, void* stream) {
  if (!M || !dst || e < 0 || e >= M->n_macro) return MHDG_ERR_INVALID_ARG;
  if (!M->ws) return fail(M, MHDG_ERR_STATE, "local_matrix: call factor_local first");
  FactorLayout& L = M->L;
  HIP_TRY(M, launch_extract_matrix((const MacroInfo*)(M->ws + L.meta), e,
                                   (const double*)(M->ws + L.tmpl), M->T, M->tau, dst,
                                   (hipStream_t)stream));
  return MHDG_OK;
}

static mhdg_status run_macro_solve(mhdg_mesh* M, int mode, int transpose, const double* lam,
                                   const double* xin, double* yout, hipStream_t s,
                                   const int32_t* skip) {
  FactorLayout& L = M->L;
  char* w = M->ws;
  ProfScope ps(M, mode == MODE_APPLY ? 2 : 4, s);
  if (M->precision == MHDG_QELIM) {
    if (transpose)
      return fail(M, MHDG_ERR_STATE, "transposed solves need MHDG_FP64 factors");
    HIP_TRY(M, launch_qelim_solve(mode, (const double*)(w + L.factors), (const MacroInfo*)(w + L.meta),
                                  (const int32_t*)(w + L.order), M->classes.data(),
                                  (int)M->classes.size(), (const int32_t*)(w + L.perm),
                                  (const double*)(w + L.tmpl), M->T, (const double*)(w + L.qtmpl),
                                  M->QT, skip, M->tau, lam, xin, yout, (double*)(w + L.slots), s));
    return MHDG_OK;
  }
  HIP_TRY(M, launch_macro_solve(mode, transpose, solve_factors(M), M->precision,
                                (const MacroInfo*)(w + L.meta), (const int32_t*)(w + L.order),
                                M->classes.data(), (int)M->classes.size(),
                                (const int32_t*)(w + L.perm), (const double*)(w + L.tmpl), M->T,
                                skip, M->tau, lam, xin, yout, (double*)(w + L.slots), s));
  return MHDG_OK;
}

namespace {
mhdg_status apply_launches(mhdg_mesh* M, const double* lam, double* out, int32_t flags,
                           const int32_t* skip, hipStream_t s);
// applies that run through stored condensed operators (timed under index 5)
constexpr int32_t kCondensed = MHDG_FOLDED | MHDG_ASSEMBLED | MHDG_BOUNDARY;

// The trace operator with an optional per-instance mask (see gmres).  With
// MHDG_GRAPH the launches (one per size class, each covering every
// instance, then the face combine) are captured once per (lam, out, flags,
// skip) into a hipGraph and replayed as one launch.
mhdg_status apply_op(mhdg_mesh* M, const double* lam, double* out, int32_t flags,
                     const int32_t* skip, hipStream_t s) {
  if (!(flags & MHDG_GRAPH)) return apply_launches(M, lam, out, flags, skip, s);
  const int32_t f = flags & ~MHDG_GRAPH;
  for (auto& a : M->graphs)
    if (a.lam == lam && a.out == out && a.flags == f && a.skip == skip) {
      ProfScope ps(M, (f & kCondensed) ? 5 : 2, s);   // the whole replayed apply
      HIP_TRY(M, hipGraphLaunch(a.x, s));
      return MHDG_OK;
    }
  if (!M->cap) HIP_TRY(M, hipStreamCreateWithFlags(&M->cap, hipStreamNonBlocking));
  if (M->graphs.size() >= 16) {   // bounded cache: drop the oldest
    (void)hipGraphExecDestroy(M->graphs.front().x);
    (void)hipGraphDestroy(M->graphs.front().g);
    M->graphs.erase(M->graphs.begin());
  }
  // capture only records the launches; the graph runs on s when launched
  HIP_TRY(M, hipStreamBeginCapture(M->cap, hipStreamCaptureModeThreadLocal));
  const bool prof = M->prof;
  M->prof = false;   // no event records inside the graph
  mhdg_status st = apply_launches(M, lam, out, f, skip, M->cap);
  M->prof = prof;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(M->cap, &g);
  if (st) { if (g) (void)hipGraphDestroy(g); return st; }
  if (e != hipSuccess) return fail(M, MHDG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(M, MHDG_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  M->graphs.push_back({lam, out, f, skip, g, x});
  ProfScope ps(M, (f & kCondensed) ? 5 : 2, s);
  HIP_TRY(M, hipGraphLaunch(x, s));
  return MHDG_OK;
}

mhdg_status apply_launches(mhdg_mesh* M, const double* lam, double* out, int32_t flags,
                           const int32_t* skip, hipStream_t s) {
  const int tr = (flags & MHDG_TRANSPOSE) ? 1 : 0;
  if (flags & MHDG_ASSEMBLED) {
    FactorLayout& L = M->L;
    ProfScope ps(M, 5, s);
    HIP_TRY(M, launch_trace_matrix_apply(M->tm_row_ptr, M->tm_blocks,
                                         (const FaceInfo*)(M->ws + L.faces), M->n_int,
                                         M->tm_max_nF,
                                         (flags & MHDG_PRECONDITION) ? M->tm_pvalues
                                                                     : M->tm_values,
                                         skip, lam, out, s));
    return MHDG_OK;
  }
  if (flags & MHDG_BOUNDARY) {
    FactorLayout& L = M->L;
    {
      ProfScope ps(M, 5, s);
      HIP_TRY(M, launch_bc_apply((const MacroInfo*)(M->ws + L.meta), M->n_macro, M->bc_off,
                                 M->bc_W, M->bc_maxP, (const double*)(M->ws + L.tmpl), M->T,
                                 M->tau, skip, tr, lam, (double*)(M->ws + L.slots), s));
    }
    ProfScope ps(M, 3, s);
    HIP_TRY(M, launch_face_combine((flags & MHDG_PRECONDITION) ? FACE_PREC_S : FACE_S,
                                   (const FaceInfo*)(M->ws + L.faces), M->n_int,
                                   (const double*)(M->ws + L.tmpl), M->T, M->tau, lam,
                                   (const double*)(M->ws + L.slots), out, s, skip));
    return MHDG_OK;
  }
  if (flags & MHDG_FOLDED) {
    FactorLayout& L = M->L;
    {
      ProfScope ps(M, 5, s);
      HIP_TRY(M, launch_fold_apply((const MacroInfo*)(M->ws + L.meta), M->n_macro, M->fold_toff,
                                   M->fold_T, M->p, M->fold_maxL, skip, tr, lam,
                                   (double*)(M->ws + L.slots), s));
    }
    ProfScope ps(M, 3, s);
    HIP_TRY(M, launch_face_combine((flags & MHDG_PRECONDITION) ? FACE_PREC_S : FACE_S,
                                   (const FaceInfo*)(M->ws + L.faces), M->n_int,
                                   (const double*)(M->ws + L.tmpl), M->T, M->tau, lam,
                                   (const double*)(M->ws + L.slots), out, s, skip));
    return MHDG_OK;
  }
  mhdg_status st = run_macro_solve(M, MODE_APPLY, tr, lam, nullptr, nullptr, s, skip);
  if (st) return st;
  FactorLayout& L = M->L;
  ProfScope ps(M, 3, s);
  HIP_TRY(M, launch_face_combine((flags & MHDG_PRECONDITION) ? FACE_PREC_S : FACE_S,
                                 (const FaceInfo*)(M->ws + L.faces), M->n_int,
                                 (const double*)(M->ws + L.tmpl), M->T, M->tau, lam,
                                 (const double*)(M->ws + L.slots), out, s, skip));
  return MHDG_OK;
}
}  // namespace

mhdg_status mhdg_apply_trace_operator(mhdg_mesh* M, const double* lam, double* out, int32_t flags,
                                      void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored) return fail(M, MHDG_ERR_STATE, "apply: call factor_local first");
  if ((!lam || !out) && M->n_trace > 0) return fail(M, MHDG_ERR_INVALID_ARG, "apply: null vector");
  if (lam == out && M->n_trace > 0) return fail(M, MHDG_ERR_INVALID_ARG, "apply: lam and out alias");
  const int tr = (flags & MHDG_TRANSPOSE) ? 1 : 0;
  if (tr && M->precision != MHDG_FP64)
    return fail(M, MHDG_ERR_STATE, "apply: the transposed operator needs FP64 factors");
  if ((flags & MHDG_FOLDED) && !M->folded)
    return fail(M, MHDG_ERR_STATE, "apply: folded operators need mhdg_fold_operator");
  if (flags & MHDG_ASSEMBLED) {
    if (!M->assembled)
      return fail(M, MHDG_ERR_STATE, "apply: the assembled matrix needs mhdg_assemble_trace_matrix");
    if (tr || (flags & MHDG_FOLDED))
      return fail(M, MHDG_ERR_INVALID_ARG,
                  "apply: MHDG_ASSEMBLED takes no MHDG_TRANSPOSE or MHDG_FOLDED");
  }
  if (flags & MHDG_BOUNDARY) {
    if (!M->bcond)
      return fail(M, MHDG_ERR_STATE, "apply: the boundary-condensed blocks need mhdg_condense_boundary");
    if (flags & (MHDG_FOLDED | MHDG_ASSEMBLED))
      return fail(M, MHDG_ERR_INVALID_ARG,
                  "apply: MHDG_BOUNDARY takes no MHDG_FOLDED or MHDG_ASSEMBLED");
  }
  if (M->n_trace == 0) return MHDG_OK;
  return apply_op(M, lam, out, flags, nullptr, (hipStream_t)stream);
}

size_t mhdg_apply_many_ws_bytes(const mhdg_mesh* M, int32_t n_rhs) {
  if (!M || n_rhs < 0) return 0;
  return size_t(n_rhs) * size_t(M->n_slots) * sizeof(double);
}

}  // extern "C"

namespace {
// The many-vector apply with the contribution slots at `slots` (bytes of room
// given); shared by the workspace and the no-allocation entry points.
mhdg_status apply_many_impl(mhdg_mesh* M, int32_t n_rhs, const double* lam, double* out,
                            int32_t flags, void* ws, size_t ws_bytes, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (n_rhs < 0) return fail(M, MHDG_ERR_INVALID_ARG, "apply_many: n_rhs < 0");
  if (flags & ~(MHDG_PRECONDITION | MHDG_FOLDED))
    return fail(M, MHDG_ERR_INVALID_ARG,
                "apply_many: only MHDG_PRECONDITION and MHDG_FOLDED are accepted in flags");
  const bool folded = (flags & MHDG_FOLDED) != 0;
  if (!M->factored) return fail(M, MHDG_ERR_STATE, "apply_many: call factor_local first");
  if (folded && !M->folded)
    return fail(M, MHDG_ERR_STATE, "apply_many: folded operators need mhdg_fold_operator");
  if (!folded && M->precision != MHDG_FP64)
    return fail(M, MHDG_ERR_STATE, "apply_many: needs MHDG_FP64 factors (or MHDG_FOLDED)");
  if (n_rhs == 0 || M->n_trace == 0) return MHDG_OK;
  if (!lam || !out) return fail(M, MHDG_ERR_INVALID_ARG, "apply_many: null vector");
  const int64_t len = int64_t(n_rhs) * M->n_trace;
  if (lam < out + len && out < lam + len)
    return fail(M, MHDG_ERR_INVALID_ARG, "apply_many: lam and out overlap");
  if (!ws || ws_bytes < mhdg_apply_many_ws_bytes(M, n_rhs))
    return fail(M, MHDG_ERR_WORKSPACE, "apply_many: workspace smaller than mhdg_apply_many_ws_bytes");
  hipStream_t s = (hipStream_t)stream;
  FactorLayout& L = M->L;
  char* w = M->ws;
  double* slots = (double*)ws;
  if (folded) {
    ProfScope ps(M, 5, s);
    HIP_TRY(M, launch_fold_apply_many((const MacroInfo*)(w + L.meta), M->n_macro, M->fold_toff,
                                      M->fold_T, M->p, M->fold_maxL, n_rhs, lam, M->n_trace,
                                      slots, M->n_slots, s));
  } else {
    ProfScope ps(M, 2, s);
    HIP_TRY(M, launch_apply_many((const double*)(w + L.factors), (const MacroInfo*)(w + L.meta),
                                 (const int32_t*)(w + L.order), M->classes.data(),
                                 (int)M->classes.size(), (const int32_t*)(w + L.perm),
                                 (const double*)(w + L.tmpl), M->T, M->tau, n_rhs, lam,
                                 M->n_trace, slots, M->n_slots, s));
  }
  ProfScope ps(M, 3, s);
  for (int32_t v0 = 0; v0 < n_rhs; v0 += 65535)   // grid y limit
    HIP_TRY(M, launch_face_combine_many((flags & MHDG_PRECONDITION) ? 1 : 0,
                                        (const FaceInfo*)(w + L.faces), M->n_int,
                                        (const double*)(w + L.tmpl), M->T, M->tau,
                                        std::min<int32_t>(65535, n_rhs - v0),
                                        lam + int64_t(v0) * M->n_trace, M->n_trace,
                                        slots + int64_t(v0) * M->n_slots, M->n_slots,
                                        out + int64_t(v0) * M->n_trace, s));
  return MHDG_OK;
}

}  // namespace

// Contribution slots of mhdg_apply_trace_operator_many_noalloc: a fixed
// device array instead of a caller workspace.  Each GPU the library runs on
// holds its own copy (at its own address) until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device, never through the array's name.
static constexpr size_t kNoAllocBytes = size_t(MHDG_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex& scratch_mutex() {
  static std::mutex mu;
  return mu;
}
void* g_scratch[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on the first call
// on that device.
mhdg_status scratch_address(mhdg_mesh* M, void** out) {
  int dev = -1;
  HIP_TRY(M, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(M, MHDG_ERR_HIP, "apply_many_noalloc: device id out of range");
  std::lock_guard<std::mutex> lk(scratch_mutex());
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(M, MHDG_ERR_HIP, std::string("apply_many_noalloc: scratch address: ") +
                                       hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return MHDG_OK;
}
}  // namespace

extern "C" {

mhdg_status mhdg_apply_trace_operator_many(mhdg_mesh* M, int32_t n_rhs, const double* lam,
                                           double* out, int32_t flags, void* ws, size_t ws_bytes,
                                           void* stream) {
  return apply_many_impl(M, n_rhs, lam, out, flags, ws, ws_bytes, stream);
}

mhdg_status mhdg_apply_trace_operator_many_noalloc(mhdg_mesh* M, int32_t n_rhs, const double* lam,
                                                   double* out, int32_t flags, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (n_rhs < 0) return fail(M, MHDG_ERR_INVALID_ARG, "apply_many_noalloc: n_rhs < 0");
  const size_t need = mhdg_apply_many_ws_bytes(M, n_rhs);
  if (need > kNoAllocBytes)
    return fail(M, MHDG_ERR_INVALID_ARG,
                "apply_many_noalloc: n_rhs * n_slots * 8 = " + std::to_string(need) +
                    " bytes exceeds the fixed scratch of " + std::to_string(kNoAllocBytes) +
                    " bytes (use fewer vectors per call, or mhdg_apply_trace_operator_many)");
  if (n_rhs == 0 || M->n_trace == 0) return apply_many_impl(M, n_rhs, lam, out, flags, nullptr, 0, stream);
  void* ptr = nullptr;
  mhdg_status st = scratch_address(M, &ptr);
  if (st) return st;
  // no event records here (they would create events): timing stays off for this call
  const bool prof = M->prof;
  M->prof = false;
  st = apply_many_impl(M, n_rhs, lam, out, flags, ptr, kNoAllocBytes, stream);
  M->prof = prof;
  return st;
}

mhdg_status mhdg_local_solve(mhdg_mesh* M, const double* x, double* y, int32_t flags, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored) return fail(M, MHDG_ERR_STATE, "local_solve: call factor_local first");
  if (!x || !y) return fail(M, MHDG_ERR_INVALID_ARG, "local_solve: null vector");
  const int tr = (flags & MHDG_TRANSPOSE) ? 1 : 0;
  if (tr && M->precision != MHDG_FP64)
    return fail(M, MHDG_ERR_STATE, "local_solve: transposed solves need FP64 factors");
  return run_macro_solve(M, MODE_LOCAL, tr, nullptr, x, y, (hipStream_t)stream);
}

mhdg_status mhdg_rhs(mhdg_mesh* M, const double* f_nodes, const double* g_bnd, double* fhat,
                     int32_t flags, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored) return fail(M, MHDG_ERR_STATE, "rhs: call factor_local first");
  if (!f_nodes || (!g_bnd && M->n_bnd_points > 0) || (!fhat && M->n_trace > 0))
    return fail(M, MHDG_ERR_INVALID_ARG, "rhs: null vector");
  hipStream_t s = (hipStream_t)stream;
  FactorLayout& L = M->L;
  char* w = M->ws;
  const double* tm = (const double*)(w + L.tmpl);
  if (M->n_bnd > 0)
    HIP_TRY(M, launch_dirichlet((const BndFaceInfo*)(w + L.bfaces), M->n_bnd, tm, M->T, g_bnd,
                                (double*)(w + L.lamD), s));
  HIP_TRY(M, launch_local_rhs((const MacroInfo*)(w + L.meta), M->n_macro,
                              (const BndFaceInfo*)(w + L.bfaces), tm, M->T, f_nodes,
                              (const double*)(w + L.lamD), M->tau,
                              (double*)(w + L.R), s));
  M->have_rhs = true;
  if (M->n_trace == 0) return MHDG_OK;
  mhdg_status st = run_macro_solve(M, MODE_RHS, 0, nullptr, (const double*)(w + L.R), nullptr, s);
  if (st) return st;
  HIP_TRY(M, launch_face_combine((flags & MHDG_PRECONDITION) ? FACE_PREC_RHS : FACE_RHS,
                                 (const FaceInfo*)(w + L.faces), M->n_int, tm, M->T, M->tau,
                                 nullptr, (const double*)(w + L.slots), fhat, s));
  return MHDG_OK;
}

mhdg_status mhdg_flux_balance(mhdg_mesh* M, const double* lam, const double* qu,
                              const double* f_nodes, double* out, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored || !M->have_rhs)
    return fail(M, MHDG_ERR_STATE, "flux_balance: call factor_local and rhs/solve first");
  if (!qu || !f_nodes || !out || (!lam && M->n_trace > 0))
    return fail(M, MHDG_ERR_INVALID_ARG, "flux_balance: null vector");
  FactorLayout& L = M->L;
  char* w = M->ws;
  HIP_TRY(M, launch_flux_balance((const MacroInfo*)(w + L.meta), M->n_macro,
                                 (const BndFaceInfo*)(w + L.bfaces), (const double*)(w + L.tmpl),
                                 M->T, M->tau, lam, (const double*)(w + L.lamD), qu, f_nodes, out,
                                 (hipStream_t)stream));
  return MHDG_OK;
}

mhdg_status mhdg_recover_local(mhdg_mesh* M, const double* lam, double* qu, double* flux_res,
                               void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->factored || !M->have_rhs)
    return fail(M, MHDG_ERR_STATE, "recover_local: call factor_local and rhs/solve first");
  if (!qu || (!lam && M->n_trace > 0)) return fail(M, MHDG_ERR_INVALID_ARG, "recover_local: null vector");
  hipStream_t s = (hipStream_t)stream;
  FactorLayout& L = M->L;
  mhdg_status st = run_macro_solve(M, MODE_RECOVER, 0, lam, (const double*)(M->ws + L.R), qu, s);
  if (st) return st;
  if (M->precision == MHDG_FP32 || M->precision == MHDG_BF16) {
    // local iterative refinement: r = R - A U - B lam in FP64 (matrix-free),
    // U += A~^-1 r with the low-precision factors, until r stops decreasing
    char* fw = M->ws;
    const double* tm = (const double*)(fw + L.tmpl);
    const MacroInfo* info_d = (const MacroInfo*)(fw + L.meta);
    double* r = (double*)(fw + L.work1);
    double* d = (double*)(fw + L.work2);
    const int64_t nl = M->n_local;
    Gm G;
    G.n = nl;
    G.ld = nl;
    G.nblk = dots_nblk(nl);
    // scratch for the norms: the tail of work2 is not needed for them, use slots
    std::vector<double> hbuf(1);
    double prev = -1.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
      HIP_TRY(M, launch_local_residual(info_d, M->n_macro, tm, M->T, M->tau,
                                       (const double*)(fw + L.R), qu, lam, r, s));
      // ||r||: partial sums in d (nblk doubles), result in d[nblk]
      G.partial = d;
      G.hdev = d + G.nblk;
      double rn2;
      if ((st = dot(M, G, r, r, &rn2, s))) return st;
      const double rn = std::sqrt(rn2);
      if (rn == 0.0 || (prev >= 0.0 && rn > 0.5 * prev)) break;
      prev = rn;
      if ((st = run_macro_solve(M, MODE_LOCAL, 0, nullptr, r, d, s))) return st;
      HIP_TRY(M, launch_axpby(1.0, d, 1.0, qu, nl, s));
    }
    if (flux_res && M->n_trace > 0) {
      HIP_TRY(M, launch_boundary_C(info_d, M->n_macro, tm, M->T, M->tau, qu, (double*)(fw + L.slots), s));
      HIP_TRY(M, launch_face_combine(FACE_RESID, (const FaceInfo*)(fw + L.faces), M->n_int, tm,
                                     M->T, M->tau, lam, (const double*)(fw + L.slots), flux_res, s));
    }
    return MHDG_OK;
  }
  if (flux_res && M->n_trace > 0)
    HIP_TRY(M, launch_face_combine(FACE_RESID, (const FaceInfo*)(M->ws + L.faces), M->n_int,
                                   (const double*)(M->ws + L.tmpl), M->T, M->tau, lam,
                                   (const double*)(M->ws + L.slots), flux_res, s));
  return MHDG_OK;
}


static size_t solve_bytes_impl(const mhdg_mesh* M, int R) {
  const size_t ns = size_t(M->n_inst);
  const size_t vb = align_up(size_t(M->n_trace) * sizeof(double));
  const size_t nblk = size_t(dots_nblk(M->n_trace / M->n_inst));
  return align_up(vb * (R + 9)) + align_up(2 * nblk * ns * size_t(R + 2) * sizeof(double)) +
         align_up(2 * size_t(R + 2) * ns * 8) + align_up(size_t(R + 2) * ns * 8) +
         align_up((2 * size_t(R) + 3) * ns * 8) + align_up(size_t(R + 1) * R * ns * 8) +
         2 * align_up(size_t(R + 2) * ns * 8) + align_up(ns * 8) + align_up(ns * 4) +
         align_up(size_t(M->n_local) * sizeof(double)) + gm_dev_bytes(R, M->n_inst);
}

mhdg_status mhdg_solve(mhdg_mesh* M, const double* f_nodes, const double* g_bnd,
                       const mhdg_solve_opts* o, double* lam, void* ws, size_t ws_bytes,
                       mhdg_solve_info* info, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!o || !lam || !ws || o->restart < 1 || o->max_iter < 0 || !(o->rtol >= 0.0))
    return fail(M, MHDG_ERR_INVALID_ARG, "solve: bad options or null pointer");
  if (!M->factored) return fail(M, MHDG_ERR_STATE, "solve: call factor_local first");
  if (ws_bytes < solve_bytes_impl(M, o->restart))
    return fail(M, MHDG_ERR_WORKSPACE, "solve: workspace smaller than mhdg_query reports");
  if ((M->precision == MHDG_FP32 || M->precision == MHDG_BF16) && M->n_inst > 1)
    return fail(M, MHDG_ERR_STATE, "solve: reduced-precision factors need a single instance");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = M->n_trace;
  const int R = o->restart;
  const int ns = M->n_inst;
  auto t0 = std::chrono::steady_clock::now();
  Gm G;
  carve(M, ws, R, G);
  if (o->graph) G.op_flags |= MHDG_GRAPH;
  G.classic = o->classic_gs != 0;
  G.device = o->driver == MHDG_DRIVER_DEVICE && !G.classic && R <= kDeviceMaxRestart;
  if (o->folded) {
    if (!M->folded || (M->precision != MHDG_FP64 && M->precision != MHDG_QELIM))
      return fail(M, MHDG_ERR_STATE, "solve: folded applies need mhdg_fold_operator");
    G.op_flags |= MHDG_FOLDED;
  }
  if (o->assembled) {
    if (!M->assembled)
      return fail(M, MHDG_ERR_STATE, "solve: assembled applies need mhdg_assemble_trace_matrix");
    if (o->folded)
      return fail(M, MHDG_ERR_INVALID_ARG, "solve: folded and assembled are exclusive");
    G.op_flags |= MHDG_ASSEMBLED;
  }
  if (o->boundary) {
    if (!M->bcond)
      return fail(M, MHDG_ERR_STATE, "solve: boundary-condensed applies need mhdg_condense_boundary");
    if (o->folded || o->assembled)
      return fail(M, MHDG_ERR_INVALID_ARG,
                  "solve: boundary-condensed, folded and assembled applies are exclusive");
    G.op_flags |= MHDG_BOUNDARY;
  }
  const bool stop_true = o->stop_norm == MHDG_NORM_TRUE;
  if (stop_true && !(M->precision == MHDG_FP64 || M->precision == MHDG_QELIM))
    return fail(M, MHDG_ERR_INVALID_ARG,
                "solve: MHDG_NORM_TRUE needs FP64 or QELIM factors (reduced-precision factors "
                "stop on the refined system's residual)");
  if (stop_true && !G.device)
    return fail(M, MHDG_ERR_INVALID_ARG,
                "solve: MHDG_NORM_TRUE runs with the device driver only (classic_gs = 0, "
                "restart <= 2048)");
  mhdg_solve_info inf{};
  mhdg_status st;
  FactorLayout& L = M->L;
  char* fw = M->ws;
  const double* tm = (const double*)(fw + L.tmpl);
  const MacroInfo* info_d = (const MacroInfo*)(fw + L.meta);
  const FaceInfo* faces_d = (const FaceInfo*)(fw + L.faces);
  // f^ (and R_K, kept in the factor workspace) and D^-1 f^
  if ((st = mhdg_rhs(M, f_nodes, g_bnd, G.fh, 0, stream))) return st;
  if (n == 0) {
    if (info)
      for (int q = 0; q < ns; ++q) info[q] = inf;
    return MHDG_OK;
  }
  if ((st = mhdg_rhs(M, f_nodes, g_bnd, G.pf, MHDG_PRECONDITION, stream))) return st;
  inf.n_applies = 2;
  auto t1 = std::chrono::steady_clock::now();
  inf.t_rhs_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (o->zero_guess) HIP_TRY(M, hipMemsetAsync(lam, 0, n * sizeof(double), s));
  bool converged = false;
  double rel = 0.0;
  std::vector<mhdg_solve_info> per(ns);
  if (M->precision == MHDG_FP64 || M->precision == MHDG_QELIM) {
    // ---- plain form: GMRES on D^-1 S lam = D^-1 f^, one Krylov space per instance
    std::vector<double> bnorm(ns), tr2(ns), f2(ns), rels;
    std::vector<int> its;
    std::vector<char> done;
    if ((st = dot(M, G, G.pf, G.pf, bnorm.data(), s))) return st;
    for (auto& b : bnorm) b = std::sqrt(b);
    if (stop_true) G.fh_true = G.fh;
    std::vector<double> rtrue;
    if ((st = gmres(M, G, G.pf, bnorm.data(), lam, o->rtol, R, o->max_iter, its, rels,
                    inf.n_applies, done, s, &rtrue)))
      return st;
    if (!stop_true) {
      // true residual ||f^ - S lam|| / ||f^|| per instance (with MHDG_NORM_TRUE the
      // last cycle start measured it)
      if ((st = mhdg_apply_trace_operator(M, lam, G.tv, 0, stream))) return st;
      ++inf.n_applies;
      for (int q = 0; q < ns; ++q) ++G.seg_applies[q];
      HIP_TRY(M, launch_scale_copy(1.0, G.fh, G.rv, n, s));
      HIP_TRY(M, launch_axpby(-1.0, G.tv, 1.0, G.rv, n, s));
      if ((st = dot(M, G, G.rv, G.rv, tr2.data(), s))) return st;
      if ((st = dot(M, G, G.fh, G.fh, f2.data(), s))) return st;
      rtrue.assign(ns, 0.0);
      for (int q = 0; q < ns; ++q) rtrue[q] = f2[q] > 0 ? std::sqrt(tr2[q] / f2[q]) : 0.0;
    }
    converged = true;
    for (int q = 0; q < ns; ++q) {
      per[q].iterations = its[q];
      per[q].rel_res_prec = rels[q];
      per[q].rel_res_true = rtrue[q];
      per[q].status = done[q] ? MHDG_OK : MHDG_ERR_NOT_CONVERGED;
      converged &= done[q] != 0;
    }
  } else {
    // ---- reduced-precision factors: iterative refinement of the whole
    // hybridised system in FP64.  The residual (r_U, r_lam) = (R - A U - B lam,
    // -(C U + D lam)) is formed matrix-free in FP64; the correction solves the
    // condensed system with the stored low-precision factors (inner GMRES on
    // D^-1 S~ dlam = D^-1 (r_lam - sum C A~^-1 r_U), then dU = A~^-1 (r_U - B dlam)).
    double* rU = (double*)(fw + L.work1);
    const int64_t nl = M->n_local;
    HIP_TRY(M, hipMemsetAsync(G.U, 0, nl * sizeof(double), s));
    if (!o->zero_guess) {
      // start U from the low-precision local solve for the given lam
      HIP_TRY(M, launch_macro_solve(MODE_RECOVER, 0, solve_factors(M), M->precision, info_d, (const int32_t*)(fw + L.order),
                                    M->classes.data(), (int)M->classes.size(), (const int32_t*)(fw + L.perm), tm, M->T,
                                    nullptr, M->tau, lam, (const double*)(fw + L.R), G.U,
                                    (double*)(fw + L.slots), s));
    }
    const double inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : 1e-5;
    const int max_outer = o->max_outer > 0 ? o->max_outer : 30;
    double rho0 = 0.0;
    int outer = 0, it_total = 0;
    for (;; ++outer) {
      // FP64 residual of the full system
      HIP_TRY(M, launch_local_residual(info_d, M->n_macro, tm, M->T, M->tau,
                                       (const double*)(fw + L.R), G.U, lam, rU, s));
      HIP_TRY(M, launch_boundary_C(info_d, M->n_macro, tm, M->T, M->tau, G.U, (double*)(fw + L.slots), s));
      HIP_TRY(M, launch_face_combine(FACE_RESID, faces_d, M->n_int, tm, M->T, M->tau, lam,
                                     (const double*)(fw + L.slots), G.cl, s));      // C U + D lam
      // condensed right-hand side b = D^-1 (r_lam - sum C A~^-1 r_U)
      HIP_TRY(M, launch_macro_solve(MODE_RHS, 0, solve_factors(M), M->precision, info_d, (const int32_t*)(fw + L.order),
                                    M->classes.data(), (int)M->classes.size(), (const int32_t*)(fw + L.perm), tm, M->T,
                                    nullptr, M->tau, nullptr, rU, nullptr,
                                    (double*)(fw + L.slots), s));
      ++inf.n_applies;
      HIP_TRY(M, launch_face_combine(FACE_PREC_RHS, faces_d, M->n_int, tm, M->T, M->tau, nullptr,
                                     (const double*)(fw + L.slots), G.rv, s));      // -D^-1 sum C A~^-1 r_U
      HIP_TRY(M, launch_face_combine(FACE_DINV, faces_d, M->n_int, tm, M->T, M->tau, G.cl,
                                     nullptr, G.tv, s));                            // D^-1 (C U + D lam)
      HIP_TRY(M, launch_scale_copy(1.0, G.rv, G.wv, n, s));
      HIP_TRY(M, launch_axpby(-1.0, G.tv, 1.0, G.wv, n, s));                       // b in wv
      double b2;
      if ((st = dot(M, G, G.wv, G.wv, &b2, s))) return st;
      const double rho = std::sqrt(b2);
      if (!std::isfinite(rho))
        return fail(M, MHDG_ERR_NOT_CONVERGED, "solve: non-finite refinement residual");
      if (outer == 0) rho0 = rho;
      rel = rho0 > 0 ? rho / rho0 : 0.0;
      if (rho0 == 0.0 || rel <= o->rtol) { converged = true; break; }
      if (outer >= max_outer || it_total >= o->max_iter) break;
      // inner solve to a relative tolerance no tighter than needed for the target
      const double eta = std::max(inner_rtol, 0.3 * o->rtol / std::max(rel, 1e-300));
      HIP_TRY(M, launch_scale_copy(1.0, G.wv, G.fh, n, s));                        // keep b: GMRES uses V/wv
      HIP_TRY(M, hipMemsetAsync(G.dl, 0, n * sizeof(double), s));
      std::vector<int> it;
      std::vector<double> irel;
      std::vector<char> iconv;
      if ((st = gmres(M, G, G.fh, &rho, G.dl, eta, R, o->max_iter - it_total, it, irel,
                      inf.n_applies, iconv, s)))
        return st;
      it_total += it[0];
      // dU = A~^-1 (r_U - B dlam); U += dU; lam += dlam
      HIP_TRY(M, launch_macro_solve(MODE_RECOVER, 0, solve_factors(M), M->precision, info_d, (const int32_t*)(fw + L.order),
                                    M->classes.data(), (int)M->classes.size(), (const int32_t*)(fw + L.perm), tm, M->T,
                                    nullptr, M->tau, G.dl, rU, rU, (double*)(fw + L.slots), s));
      ++inf.n_applies;
      HIP_TRY(M, launch_axpby(1.0, rU, 1.0, G.U, nl, s));
      HIP_TRY(M, launch_axpby(1.0, G.dl, 1.0, lam, n, s));
    }
    per[0].iterations = it_total;
    per[0].outer_iterations = outer;
    per[0].rel_res_prec = rel;
    per[0].rel_res_true = -1.0;   // needs FP64 factors; see rel_res_prec (FP64 residual, condensed)
    per[0].status = converged ? MHDG_OK : MHDG_ERR_NOT_CONVERGED;
  }
  auto t2 = std::chrono::steady_clock::now();
  inf.t_gmres_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
  if (info)
    for (int q = 0; q < ns; ++q) {
      info[q] = per[q];
      info[q].t_rhs_ms = inf.t_rhs_ms;
      info[q].t_gmres_ms = inf.t_gmres_ms;
      // applies this instance took part in (rhs 2, GMRES, and for FP64 the
      // true residual unless the stopping test measured it)
      info[q].n_applies = ns == 1 ? inf.n_applies : 2 + G.seg_applies[q];
      info[q].reorth_passes = G.reorth;
      info[q].cycles = G.cycles;
      info[q].host_waits = G.waits;
    }
  if (!converged) return fail(M, MHDG_ERR_NOT_CONVERGED, "solve: max_iter reached");
  return MHDG_OK;
}

mhdg_status mhdg_mass_apply(mhdg_mesh* M, const double* v, double* out, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!M->ws) return fail(M, MHDG_ERR_STATE, "mass_apply: call factor_local first");
  if (!v || !out || v == out) return fail(M, MHDG_ERR_INVALID_ARG, "mass_apply: bad vectors");
  FactorLayout& L = M->L;
  HIP_TRY(M, launch_mass((const MacroInfo*)(M->ws + L.meta), M->n_macro,
                         (const double*)(M->ws + L.tmpl), M->T, v, out, (hipStream_t)stream));
  return MHDG_OK;
}

// Adjoint: K^T Psi = dJ/dX with X = (U, lam), condensed onto the trace:
// S^T psi_lam = -sum_K B_K^T A_K^-T g_K (GMRES left-preconditioned with
// D^-1; D is symmetric), psi_K = A_K^-T (g_K - C_K^T psi_lam), both with the
// stored LU factors; then dJ/dtheta = Psi^T (dF/dtheta - dK/dtheta X).
mhdg_status mhdg_adjoint(mhdg_mesh* M, const double* lam, const double* qu, const double* dJ_dU,
                         const mhdg_solve_opts* o, double* psi_lam, double* psi_U,
                         double* dJ_dkappa, double* dJ_dbeta, void* ws, size_t ws_bytes,
                         mhdg_solve_info* info, void* stream) {
  if (!M) return MHDG_ERR_INVALID_ARG;
  if (!o || !qu || !dJ_dU || !psi_U || !dJ_dkappa || !dJ_dbeta || !ws || o->restart < 1 ||
      (M->n_trace > 0 && (!lam || !psi_lam)))
    return fail(M, MHDG_ERR_INVALID_ARG, "adjoint: bad options or null pointer");
  if (M->supg)
    return fail(M, MHDG_ERR_STATE,
                "adjoint: the SUPG forms are not affine in kappa and a (call mhdg_set_supg(mesh, 0))");
  if (!M->factored || !M->have_rhs)
    return fail(M, MHDG_ERR_STATE, "adjoint: call factor_local and solve first");
  if (M->precision != MHDG_FP64)
    return fail(M, MHDG_ERR_STATE, "adjoint: needs FP64 factors");
  if (M->n_inst != 1)
    return fail(M, MHDG_ERR_STATE, "adjoint: needs a single coefficient instance");
  if (ws_bytes < solve_bytes_impl(M, o->restart))
    return fail(M, MHDG_ERR_WORKSPACE, "adjoint: workspace smaller than mhdg_query reports");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = M->n_trace;
  Gm G;
  carve(M, ws, o->restart, G);
  G.op_flags = MHDG_PRECONDITION | MHDG_TRANSPOSE | (o->graph ? MHDG_GRAPH : 0);
  G.classic = o->classic_gs != 0;
  G.device = o->driver == MHDG_DRIVER_DEVICE && !G.classic && o->restart <= kDeviceMaxRestart;
  if (o->stop_norm == MHDG_NORM_TRUE)
    return fail(M, MHDG_ERR_INVALID_ARG, "adjoint: stops on the preconditioned residual only");
  if (o->folded) {
    if (!M->folded) return fail(M, MHDG_ERR_STATE, "adjoint: folded applies need mhdg_fold_operator");
    G.op_flags |= MHDG_FOLDED;
  }
  if (o->boundary) {
    if (!M->bcond)
      return fail(M, MHDG_ERR_STATE, "adjoint: boundary-condensed applies need mhdg_condense_boundary");
    if (o->folded)
      return fail(M, MHDG_ERR_INVALID_ARG, "adjoint: boundary-condensed and folded are exclusive");
    G.op_flags |= MHDG_BOUNDARY;
  }
  FactorLayout& L = M->L;
  char* fw = M->ws;
  const double* tm = (const double*)(fw + L.tmpl);
  const MacroInfo* info_d = (const MacroInfo*)(fw + L.meta);
  const FaceInfo* faces_d = (const FaceInfo*)(fw + L.faces);
  mhdg_solve_info inf{};
  mhdg_status st;
  bool converged = true;
  if (n > 0) {
    // right-hand side D^-1 b, b = -sum B^T A^-T g
    if ((st = run_macro_solve(M, MODE_RHS, 1, nullptr, dJ_dU, nullptr, s))) return st;
    HIP_TRY(M, launch_face_combine(FACE_PREC_RHS, faces_d, M->n_int, tm, M->T, M->tau, nullptr,
                                   (const double*)(fw + L.slots), G.pf, s));
    inf.n_applies = 1;
    double b2;
    if ((st = dot(M, G, G.pf, G.pf, &b2, s))) return st;
    HIP_TRY(M, hipMemsetAsync(psi_lam, 0, n * sizeof(double), s));
    if (b2 > 0) {
      const double bn = std::sqrt(b2);
      std::vector<int> its;
      std::vector<double> rels;
      std::vector<char> done;
      if ((st = gmres(M, G, G.pf, &bn, psi_lam, o->rtol, o->restart, o->max_iter, its, rels,
                      inf.n_applies, done, s)))
        return st;
      inf.iterations = its[0];
      inf.rel_res_prec = rels[0];
      inf.cycles = G.cycles;
      inf.host_waits = G.waits;
      converged = done[0] != 0;
    }
  }
  // psi_U = A^-T (g - C^T psi_lam)
  if ((st = run_macro_solve(M, MODE_RECOVER, 1, psi_lam, dJ_dU, psi_U, s))) return st;
  ++inf.n_applies;
  HIP_TRY(M, launch_adjoint_contract(info_d, M->n_macro, (const BndFaceInfo*)(fw + L.bfaces), tm,
                                     M->T, qu, psi_U, lam, psi_lam, (const double*)(fw + L.lamD),
                                     dJ_dkappa, (double*)(fw + L.work1), dJ_dbeta, s));
  inf.status = converged ? MHDG_OK : MHDG_ERR_NOT_CONVERGED;
  if (info) *info = inf;
  if (!converged) return fail(M, MHDG_ERR_NOT_CONVERGED, "adjoint: max_iter reached");
  return MHDG_OK;
}

}  // extern "C"
