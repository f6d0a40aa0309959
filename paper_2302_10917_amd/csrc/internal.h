// Internal declarations shared by the host driver (host.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mhdg {

constexpr int kMaxLevel = 5;
constexpr int kFactorGuard = 64 * 64;  // elements of readable padding after the last factor block

// Pivot search of the LU kernels: the magnitude compared for a candidate,
// with NaN ranked above every number so that a column whose candidates are
// all NaN still picks a row inside the block (and is reported), and the
// status word of a macro: 0, col + 1 for an exactly zero pivot, or
// -(col + 1) for a non-finite one (the first failing column).
__device__ __forceinline__ double pivot_mag(double x) {
  const double v = fabs(x);
  return v == v ? v : __builtin_huge_val();
}
__device__ __forceinline__ int pivot_status(double best, int col) {
  if (best == 0.0) return col + 1;
  if (!(best < __builtin_huge_val())) return -(col + 1);
  return 0;
}

// Per-macro data, built on the host at setup and copied into the factor
// workspace by factor_local.  All doubles first so the layout has no holes.
struct MacroInfo {
  double G[4];        // inverse Jacobian of the macro map, G[k*2+d] = d xi_k / d x_d
  double dJ;          // |det J| (twice the area)
  double len[3];      // edge lengths, edge k from vertex k to vertex k+1
  double nrm[6];      // outward unit normals (nx, ny) per edge
  double kappa;       // filled on the device from the caller's kappa array
  double bx, by;      // advection a of this macro's coefficient instance
  double hsupg;       // SUPG: sub-triangle diameter, 0 when the forms are not stabilised
  int64_t fac_off;    // element offset of this macro's factor block
  int64_t loc_off;    // offset into n_local vectors
  int64_t node_off;   // offset into n_nodes vectors
  int64_t slot_off[3];// offset of the (macro, edge) contribution slot, -1 on boundary
  int32_t face[3];    // face id (sorted order)
  int32_t orient[3];  // +1 if the local edge runs like the canonical face direction
  int32_t tr_off[3];  // global trace offset of an interior face, else -1
  int32_t bnd_face[3];// index into BndFaceInfo for a boundary face, else -1
  int32_t flevel[3];  // face level
  int32_t level;      // macro level r
  int32_t N;          // local size 3Q
  int32_t Q;
  int32_t P;          // 2^r p
  int32_t inst;       // coefficient instance this macro belongs to
  int32_t ld;         // leading dimension of the stored block: N rounded up to 16
  // flux-eliminated form: the Q x Q Schur block on u
  int32_t sld;        // its leading dimension (Q rounded up to 16)
  int64_t sfac_off;   // element offset of its factor block
  int64_t sperm_off;  // offset of its pivot vector (Q entries)
};

struct FaceInfo {     // interior faces
  double len;
  int64_t slot[2];    // slots of the two macros (lower macro id first)
  int32_t tr_off;
  int32_t nF;
  int32_t level;
  int32_t inst;       // coefficient instance
};

struct BndFaceInfo {  // boundary (Dirichlet) faces
  double len;
  int64_t g_off;      // offset of its samples in the g_D array
  int64_t lam_off;    // offset of its projected trace in the Dirichlet trace array
  int32_t nF;
  int32_t level;
};

// Offsets (in doubles / ints, from the template blob base) per level.
struct LevelTemplates {
  int64_t Mhat, E0, E1;     // Q x Q reference macro mass and derivative matrices
  int64_t E0T, E1T;         // their transposes (coalesced column access)
  int64_t M1, M1inv;        // (P+1)^2 1D trace mass on [0,1] and its inverse
  int64_t edge_node;        // int32 [3][P+1]: lattice node at local edge position s
  int64_t node_epos;        // int32 [Q][3]: position along local edge k, or -1
  int64_t bnd_index;        // int32 [Q]: position b in the macro boundary loop (edge k,
                            // position s < P -> kP + s), or -1 for nodes off the boundary
  int64_t T1[kMaxLevel + 1];// (P+1) x (P_F+1): int phi_s mu_l over [0,1], face level F >= r
  int64_t supg;             // SUPG: 9 Q x Q blocks (reference macro), or -1: (d_k phi_i, d_l phi_j)
                            // for kl = 00, 11, then 01 + 10; (d_k phi_i, D_c phi_j) for
                            // k = 0, 1 and D_c = d_00, d_01, d_11
  int32_t present, Q, P, N;
};

// Per-level templates of the flux-eliminated form (row-major Q x Q, offsets
// into their own device blob): Minv = Mhat^-1, P_a = (Ehat^a)^T Minv and its
// transpose PT_a, L_ab = P_a Ehat^b (a, b = 0, 1; L_10 = L_01^T), and Mbb, the
// 3P x 3P block of Minv on the boundary nodes in boundary order (b = kP + s).
// PB0 / PB1: the boundary rows of PT_a transposed, PB_a[j * 3P + b] =
// PT_a[node of boundary position b][j]
struct QLevel { int64_t Minv, P0, P1, PT0, PT1, L00, L01, L11, Mbb, PB0, PB1; };
struct QTemplates { QLevel lev[kMaxLevel + 1]; };

struct Templates {
  LevelTemplates lev[kMaxLevel + 1];
  int64_t dir_basis;        // (p+1) x kb: trace basis at the Dirichlet points of a segment
  int64_t dir_w;            // kb weights on [0,1]
  int32_t p, kb;
};

// Device workspace layout for factor_local / apply / rhs / recover.
struct FactorLayout {
  size_t meta, faces, bfaces, tmpl, order, perm, status, R, slots, lamD, work1, work2, factors,
      factors16, total;   // factors16: BF16 copy of the FP32 factors (BF16 precision only)
  size_t qtmpl = 0, info_lu = 0;   // flux-eliminated form: templates, Schur-block LU table
  size_t lu_scr = 0, lu_scr_bytes = 0;   // scratch of the split LU
};

// Macros of one local size, contiguous in the processing order (largest first):
// the heavy per-macro kernels are launched once per class with a register and
// thread configuration sized for that class.
struct SizeClass {
  int N, P;
  int64_t start, count;
  int32_t lu_var = 0;      // LuVariant, 0 = default rule
  int32_t solve_var = 0;   // SolveVariant, 0 = default rule
};

// Kernel variants the autotuner chooses between, per size class.
// LU_BLOCKED_U2 / _U4: the blocked LU with the trailing update's U tiles
// shared through LDS by 2 or 4 row tiles per wavefront.  LU_SPLIT: one
// launch per step of each 128-column panel, the trailing update as a
// batched MFMA GEMM over 64 x 64 tiles (needs a row-move scratch).
enum LuVariant {
  LU_DEFAULT = 0, LU_PANEL = 1, LU_BLOCKED = 2, LU_BLOCKED_U2 = 3, LU_BLOCKED_U4 = 4, LU_SPLIT = 5
};
// SOLVE_WAVE6 / SOLVE_WAVE5: one wavefront per macro like SOLVE_WAVE, with
// the register budget of 6 or 5 resident wavefronts per SIMD (for N_K in
// (512, 1024], where the 8-wavefront budget spills); SOLVE_WAVE5_LG12 and
// SOLVE_WAVE4_LG16 also keep 12 or 16 column chunks in flight per load group
// instead of 8.
enum SolveVariant { SOLVE_DEFAULT = 0, SOLVE_WAVE = 1, SOLVE_MW4 = 2, SOLVE_MW8 = 3,
                    SOLVE_WAVE6 = 4, SOLVE_WAVE5 = 5, SOLVE_WAVE5_LG12 = 6,
                    SOLVE_WAVE4_LG16 = 7 };
int default_lu_variant(int N);
int default_solve_variant(int N);
bool lu_variant_ok(int v, int N);
bool solve_variant_ok(int v, int N);

template <typename T>
hipError_t lu_blocked_class(int variant, T* fac, const MacroInfo* info, const int32_t* order,
                            const SizeClass& c, int32_t* perm, int32_t* status, hipStream_t s);
// bytes of per-macro scratch LU_SPLIT needs for a class (row moves and
// inverse diagonal blocks of the current panel; 0 for N <= 128)
size_t lu_split_scratch_bytes(const SizeClass& c);
template <typename T>
hipError_t lu_split_class(T* fac, const MacroInfo* info, const int32_t* order, const SizeClass& c,
                          int32_t* perm, int32_t* status, char* scratch, size_t scratch_bytes,
                          hipStream_t s);

enum SolveMode { MODE_APPLY = 0, MODE_RHS = 1, MODE_RECOVER = 2, MODE_LOCAL = 3 };

hipError_t launch_local_residual(const MacroInfo* info, int64_t n, const double* tmpl,
                                 const Templates& T, double tau, const double* R, const double* U,
                                 const double* lam, double* out, hipStream_t s);
hipError_t launch_adjoint_contract(const MacroInfo* info, int64_t n, const BndFaceInfo* bf,
                                   const double* tmpl, const Templates& T, const double* U,
                                   const double* Psi, const double* lam, const double* psi_lam,
                                   const double* lamD, double* dkappa, double* dbeta_part,
                                   double* dbeta, hipStream_t s);
hipError_t launch_mass(const MacroInfo* info, int64_t n, const double* tmpl, const Templates& T,
                       const double* v, double* out, hipStream_t s);
hipError_t launch_boundary_C(const MacroInfo* info, int64_t n, const double* tmpl,
                             const Templates& T, double tau, const double* U, double* slots,
                             hipStream_t s);

// ---- kernel launchers (kernels.hip) ----
// kappa into the macro table; bad[e] = 1 where kappa[e] is not finite and > 0
hipError_t launch_set_kappa(MacroInfo* info, const double* kappa, int64_t n, int32_t* bad,
                            hipStream_t s);
hipError_t launch_assemble(void* fac, int precision, const MacroInfo* info, const int32_t* order,
                           int64_t n, const double* tmpl, const Templates& T, double tau,
                           hipStream_t s);
// scratch: per-macro scratch for classes factored with LU_SPLIT
// (lu_split_scratch_bytes per class)
hipError_t launch_lu(void* fac, int precision, const MacroInfo* info, const int32_t* order,
                     const SizeClass* classes, int n_classes, int32_t* perm, int32_t* status,
                     char* scratch, size_t scratch_bytes, hipStream_t s);
hipError_t launch_dirichlet(const BndFaceInfo* bf, int64_t nbf, const double* tmpl,
                            const Templates& T, const double* g, double* lamD, hipStream_t s);
hipError_t launch_local_rhs(const MacroInfo* info, int64_t n, const BndFaceInfo* bf,
                            const double* tmpl, const Templates& T, const double* f,
                            const double* lamD, double tau, double* R, hipStream_t s);
// skip: null, or per-instance flags; macros (faces) of an instance whose flag
// is non-zero are not processed and their outputs are left untouched (face
// outputs are written as zero).
hipError_t launch_macro_solve(int mode, int transpose, const void* fac, int precision,
                              const MacroInfo* info, const int32_t* order,
                              const SizeClass* classes, int n_classes, const int32_t* perm,
                              const double* tmpl, const Templates& T, const int32_t* skip,
                              double tau, const double* lam, const double* xin, double* yout,
                              double* slots, hipStream_t s);
hipError_t launch_face_combine(int mode, const FaceInfo* fi, int64_t nf, const double* tmpl,
                               const Templates& T, double tau, const double* lam,
                               const double* slots, double* out, hipStream_t s,
                               const int32_t* skip = nullptr);
// per macro <flux^.n, 1>_dK - (f_h, 1)_K (the local problem tested with w = 1)
hipError_t launch_flux_balance(const MacroInfo* info, int64_t n, const BndFaceInfo* bf,
                               const double* tmpl, const Templates& T, double tau,
                               const double* lam, const double* lamD, const double* U,
                               const double* f, double* out, hipStream_t s);
// step 4 for n_rhs vectors in one launch (FACE_S, or FACE_PREC_S with precondition = 1);
// vector v at lam / out + v * ld_lam, its slots at slots + v * ld_slots
hipError_t launch_face_combine_many(int precondition, const FaceInfo* fi, int64_t nf,
                                    const double* tmpl, const Templates& T, double tau,
                                    int n_rhs, const double* lam, int64_t ld_lam,
                                    const double* slots, int64_t ld_slots, double* out,
                                    hipStream_t s);
hipError_t launch_extract_matrix(const MacroInfo* info, int64_t e, const double* tmpl,
                                 const Templates& T, double tau, double* dst, hipStream_t s);
// face_combine modes
enum FaceMode { FACE_S = 0, FACE_PREC_S = 1, FACE_RHS = 2, FACE_PREC_RHS = 3, FACE_RESID = 4,
                FACE_DINV = 5 /* out = D_F^-1 lam (slots unused) */ };

// folded macro operators T_K = C_K A_K^-1 B_K (fold.hip)
constexpr int kFoldMaxL = 192;
// flux-eliminated form (qelim.hip, kernels.hip): Schur block assembly (row-major
// into the factor blocks at sfac_off) and the per-macro solves in every mode
hipError_t launch_qelim_assemble(double* fac, const MacroInfo* info, int64_t n, int maxQ,
                                 const double* tmpl, const Templates& T, const double* qtm,
                                 const QTemplates& QT, double tau, hipStream_t s);
hipError_t launch_qelim_solve(int mode, const double* fac, const MacroInfo* info,
                              const int32_t* order, const SizeClass* classes, int n_classes,
                              const int32_t* perm, const double* tmpl, const Templates& T,
                              const double* qtm, const QTemplates& QT, const int32_t* skip,
                              double tau, const double* lam, const double* xin, double* yout,
                              double* slots, hipStream_t s);
size_t qelim_lds_bytes(int Q, int P);
// T_K for every macro from the Schur-block factors (max_L: the largest L_K)
hipError_t launch_qelim_fold_build(const double* fac, const MacroInfo* info, const int32_t* order,
                                   const SizeClass* classes, int n_classes, const int32_t* perm,
                                   const double* tmpl, const Templates& T, const double* qtm,
                                   const QTemplates& QT, double tau, int max_L,
                                   const int64_t* toff, double* out, hipStream_t s);

// W_K = (A_K^-1)_bb for every macro from the Schur-block factors (boundary.hip
// layout: offsets woff, blocks W)
hipError_t launch_qelim_bc_build(const double* fac, const MacroInfo* info, const int32_t* order,
                                 const SizeClass* classes, int n_classes, const int32_t* perm,
                                 const double* tmpl, const Templates& T, const double* qtm,
                                 const QTemplates& QT, double tau, const int64_t* woff, double* W,
                                 hipStream_t s);

// T_K for every macro, from the FP64 factors (max_L: the largest L_K)
hipError_t launch_fold_build(const double* fac, const MacroInfo* info, const int32_t* order,
                             const SizeClass* classes, int n_classes, const int32_t* perm,
                             const double* tmpl, const Templates& T, double tau, int max_L,
                             const int64_t* toff, double* out, hipStream_t s);
hipError_t launch_fold_apply(const MacroInfo* info, int64_t n, const int64_t* toff, const double* T,
                             int p, int max_L, const int32_t* skip, int transpose,
                             const double* lam, double* slots, hipStream_t s);

// boundary-condensed blocks W_K = (A_K^-1)_bb (boundary.hip): the build from
// the FP64 factors, then steps 1-3 through W_K (W_K^T when transposed)
hipError_t launch_bc_build(const double* fac, const MacroInfo* info, const int32_t* order,
                           const SizeClass* classes, int n_classes, const int32_t* perm,
                           const double* tmpl, const Templates& T, const int64_t* woff,
                           double* W, hipStream_t s);
hipError_t launch_bc_apply(const MacroInfo* info, int64_t n, const int64_t* woff, const double* W,
                           int max_P, const double* tmpl, const Templates& T, double tau,
                           const int32_t* skip, int transpose, const double* lam, double* slots,
                           hipStream_t s);

// steps 1-3 for n_rhs trace vectors at once (many.hip): vector v reads
// lam + v * ld_lam and writes its slots at slots + v * ld_slots
hipError_t launch_apply_many(const double* fac, const MacroInfo* info, const int32_t* order,
                             const SizeClass* classes, int n_classes, const int32_t* perm,
                             const double* tmpl, const Templates& T, double tau, int n_rhs,
                             const double* lam, int64_t ld_lam, double* slots, int64_t ld_slots,
                             hipStream_t s);

// folded steps 1-3 for n_rhs trace vectors (T_K read once per group of 8)
hipError_t launch_fold_apply_many(const MacroInfo* info, int64_t n, const int64_t* toff,
                                  const double* T, int p, int max_L, int n_rhs, const double* lam,
                                  int64_t ld_lam, double* slots, int64_t ld_slots, hipStream_t s);

// GMRES vector kernels
// Vectors may hold nseg independent segments of length n (coefficient
// instances): dot products and updates are per segment; out / h are indexed
// [column * nseg + segment].
// skip (null, or per segment): segments with a nonzero flag are left out
// (their outputs are not written); ncol_seg (null, or per segment) limits the
// columns gemv_sub reads for each segment.
hipError_t launch_dots(const double* V, int64_t ld, int ncols, const double* w, int64_t n,
                       double* partial, int nblk, double* out, hipStream_t s, int nseg = 1,
                       const int32_t* skip = nullptr);
hipError_t launch_gemv_sub(const double* V, int64_t ld, int ncols, const double* h, double* w,
                           int64_t n, double sign, hipStream_t s, int nseg = 1,
                           const int32_t* ncol_seg = nullptr);
hipError_t launch_to_bf16(const float* src, void* dst, int64_t n, hipStream_t s);
hipError_t launch_seg_scale_copy(const double* alpha, const double* x, double* y, int64_t n, int nseg,
                                 hipStream_t s);
// delayed-reorthogonalisation Arnoldi (see host gmres): two products per
// column in one read of V, the Hessenberg correction, the fused two-output update
hipError_t launch_dots2(const double* V, int64_t ld, int ncols, const double* x, const double* y,
                        int64_t n, double* partial, int nblk, double* out, hipStream_t s,
                        int nseg, const int32_t* skip = nullptr);
// the chunk partial sums of launch_dots2 only (their sums left to the caller)
hipError_t launch_dots2_partial(const double* V, int64_t ld, int ncols, const double* x,
                                const double* y, int64_t n, double* partial, int nblk,
                                hipStream_t s, int nseg, const int32_t* skip = nullptr);
hipError_t launch_hbar_gemv(const double* Hb, int64_t ld, int nseg, int kmax, int rows,
                            const double* pq, double* out, hipStream_t s);
hipError_t launch_dual_update(double* V, int64_t ld, int j, int64_t n, int nseg, const double* ca,
                              const double* cd, const double* sc, const double* z, double* u2,
                              hipStream_t s, const int32_t* skip = nullptr);

// One block of the assembled trace matrix (assembled.hip): rows of interior
// face row_face, columns of interior face col_face (indices into the
// FaceInfo array), values column-major at S + voff; built from ncontrib
// (1 or 2) sub-blocks T_K[r0 + i, c0 + j] of folded operators (T_K at toff,
// leading dimension L), plus D_F when diag.
struct TraceBlock {
  int64_t voff;
  int64_t toff[2];
  int32_t row_face, col_face, nF, nC, ncontrib;
  int32_t col_off;   // trace offset of the column face (diagonal: col_face == row_face)
  int32_t L[2], r0[2], c0[2];
};
static_assert(sizeof(TraceBlock) == 72, "the block table's documented entry size");
// S's blocks, then those of D^-1 S (Pm, the same layout)
hipError_t launch_trace_matrix_build(const TraceBlock* blk, int64_t n_blocks, const FaceInfo* faces,
                                     const double* tmpl, const Templates& T, double tau,
                                     const double* Tk, double* S, double* Pm, hipStream_t s);
// out = S lam over the block rows (S: the values of S or of D^-1 S); max_nF:
// the largest face trace (picks the lane split of the product kernel)
hipError_t launch_trace_matrix_apply(const int32_t* row_ptr, const TraceBlock* blk,
                                     const FaceInfo* faces, int64_t n_faces, int max_nF,
                                     const double* S, const int32_t* skip, const double* lam,
                                     double* out, hipStream_t s);

// Device state of the GMRES whose per-segment recurrences run on the device
// (gmres_dev.hip); every pointer is into the solve workspace.  Per segment
// q of ns: H rotated Hessenberg ((R + 1) x R, column-major), cs / sn
// rotations [R], g rotated right side [R + 1], hprev [R + 1]; Hb finished
// unrotated columns ((k (R + 1) + i) ns + q); pq dual products and Hbar a,
// hy single products, coef update coefficients, y least-squares solution
// [R ns]; alpha, nrm, nrm_true, fref, bref, rel, rel_true, tgt, est [ns];
// prm = (rtol, max_iter); skip, active, done, jc (finished columns this
// cycle), iters (in all), flag (non-finite residual), napp (applies taken
// part in) [ns]; any [1].
struct GmDev {
  double *H, *cs, *sn, *g, *hprev, *Hb, *pq, *hy, *coef, *y;
  double *alpha, *nrm, *nrm_true, *fref, *bref, *rel, *rel_true, *tgt, *est, *prm;
  int32_t *skip, *active, *done, *jc, *iters, *flag, *napp, *any;
  int ns;
};
hipError_t launch_gm_start(const GmDev& d, int R, hipStream_t s);
hipError_t launch_gm_step(const GmDev& d, int R, int j, int last, hipStream_t s);
// dots2's final sums, the Hbar correction and gm_step of column j in one
// launch (the partial sums of launch_dots2_partial in; j + 1 <= kGmColumnMax)
constexpr int kGmColumnMax = 64;
hipError_t launch_gm_column(const GmDev& d, const double* partial, int nblk, int R, int j,
                            hipStream_t s);
hipError_t launch_gm_lsq(const GmDev& d, int R, hipStream_t s);
hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
hipError_t launch_scale_copy(double a, const double* x, double* y, int64_t n, hipStream_t s);
int dots_nblk(int64_t n);

}  // namespace mhdg
