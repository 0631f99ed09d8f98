// Host-side launchers of the HPS HIP kernels (gfx950).  Every launcher enqueues on the
// given stream and checks the launch; none synchronizes.
#pragma once

#include "common.hpp"

namespace hps {

// ------------------------------------------------------------------ batched GEMM
// C_b = beta * C_b + alpha * A_b * B_b   (b = 0..batch-1), column-major.
// A is M x K, B is K x N, C is M x N.  A and B may be real (double) or complex
// (interleaved double2); C is complex.  Leading dimensions and batch strides are in
// elements of the operand's own type.  Optional int32 maps scatter C: element (i, j)
// lives at C_b[crow[i] + ldc * ccol[j]] (identity where the map is null).
struct GemmDesc {
  int M = 0, N = 0, K = 0, batch = 1;
  const double* A = nullptr; long lda = 0, sA = 0; bool a_real = false;
  const double* B = nullptr; long ldb = 0, sB = 0; bool b_real = false;
  double* C = nullptr; long ldc = 0, sC = 0;
  double alpha = 1.0, beta = 0.0;
  const int* crow = nullptr;
  const int* ccol = nullptr;
  bool c64 = false;  // A, B and C are complex64 (interleaved float); FP32 accumulation
  // optional real addend of the (i, j) entry (before the row and column maps): C0r[b * s0
  // + i + ld0 * j] is added to the real part (complex128 only)
  const double* C0r = nullptr; long ld0 = 0, s0 = 0;
};
void zgemm(const GemmDesc& d, hipStream_t st);
// Autotuner: time every tile variant for d's shape and record the fastest (synchronizes
// st; a shape already recorded is skipped).  zgemm then launches the recorded variant.
void zgemm_tune(const GemmDesc& d, hipStream_t st);
int zgemm_tune_entries();
void zgemm_tune_clear();
std::string zgemm_tune_dump();               // "M N K batch flags variant" per line
int zgemm_tune_load(const std::string& text);  // merges; returns the lines read
// name of the kernel variant zgemm launches for d: tile "MxN" plus r/c for real or
// complex A and B (e.g. "64x64cc")
std::string zgemm_variant(const GemmDesc& d);

// ------------------------------------------------------------------ skinny GEMM (solve)
// out_b(i, r) = alpha * sum_k A_b(i, k) X_b(k, r)  +  addend(i, r),   r < nrhs,
// where addend is C0_b(i, r) if C0 is given, the current C_b value if accumulate is
// set, else 0.  A complex M x K (lda, sA).  X complex (ldx, sX); if xoff is given it
// replaces b*sX.  C complex with ldc, sC (or coff), optional row map crow.  C0
// complex with ld0, s0 (or c0off).  All offsets in complex elements.
struct SkinnyDesc {
  int M = 0, K = 0, nrhs = 1, batch = 1;
  const double* A = nullptr; long lda = 0, sA = 0;
  const double* X = nullptr; long ldx = 0, sX = 0; const long* xoff = nullptr;
  double* C = nullptr; long ldc = 0, sC = 0; const long* coff = nullptr;
  const int* crow = nullptr;
  const double* C0 = nullptr; long ld0 = 0, s0 = 0; const long* c0off = nullptr;
  bool accumulate = false;
  double alpha = 1.0;
  bool a_c64 = false;  // A is complex64 (FP32 products and accumulation)
  long xbase = 0, cbase = 0;  // subtracted from xoff[b] / coff[b]
  // workspace for the split-K partial sums (at least skinny_work_bytes(d) bytes)
  void* work = nullptr;
  // optional second operator of the same shape and strides, applied in the same launch
  // (its batch entries follow the first's): its own A, C, crow and C0, and its own X
  // (same strides and offsets) if X2 is set, else the first's X
  const double* A2 = nullptr;
  double* C2 = nullptr;
  const int* crow2 = nullptr;
  const double* C02 = nullptr;
  const double* X2 = nullptr;
  // Operators of several factors of one shape in one launch: when aper > 0, entry b
  // belongs to factor q = b / aper and its operator is Atab[q] + (b % aper) * sA (Atab2
  // for the second operator); A and A2 are then unused.  nrq[q] > 0 limits factor q to
  // its first nrq[q] right-hand sides: its entries skip the columns beyond (their
  // outputs are left unwritten).
  static constexpr int kMaxTab = 16;
  int aper = 0;
  const double* Atab[kMaxTab] = {};
  const double* Atab2[kMaxTab] = {};
  int nrq[kMaxTab] = {};
};
size_t skinny_work_bytes(const SkinnyDesc& d);

// One upward-sweep merge level in one launch, for levels whose interface is short
// (up_fused_fits): one workgroup per box gathers the children's outgoing data,
// forms t~3a = W^{-1} (R33b h3a - h3b), t~3b = -h3a - R33a t~3a and the parent's
// h = [h1a + R13a t~3a ; h2b + R23b t~3b] with the box's vectors in LDS, and writes
// t~3a, t~3b (kept for the downward sweep) and h.  Layouts as the separate launches
// use: hc [2 nbox][nrhs][nbc], hp [nbox][nrhs][nbp], tta/ttb [nbox][nrhs][n3]; jumps
// (optional) as for up_gather.  Box q's operators: factor f = q / per, box q % per of
// its level arrays R33b[f], Winv[f], R33a[f], R13a[f], R23b[f]; nrq[f] > 0 limits
// factor f to its first nrq[f] right-hand sides (the other columns are left unwritten).
struct UpLevelDesc {
  int nbox = 0, nbc = 0, n1 = 0, n2 = 0, n3 = 0, nbp = 0, nrhs = 0;
  const int *perm = nullptr, *i1a = nullptr, *i3a = nullptr, *i2b = nullptr, *i3b = nullptr;
  const double* hc = nullptr;
  double* hp = nullptr;
  double *tta = nullptr, *ttb = nullptr;
  const double* jmp = nullptr; long ldj = 0; const int *ja = nullptr, *jb = nullptr; long jbase = 0;
  bool c64 = false;  // the level's operators are complex64
  int per = 0;       // boxes per factor
  const double *R33b[SkinnyDesc::kMaxTab] = {}, *Winv[SkinnyDesc::kMaxTab] = {},
               *R33a[SkinnyDesc::kMaxTab] = {}, *R13a[SkinnyDesc::kMaxTab] = {},
               *R23b[SkinnyDesc::kMaxTab] = {};
  int nrq[SkinnyDesc::kMaxTab] = {};
};
bool up_fused_fits(int n1, int n2, int n3, int nbp);  // the level's box fits the kernel
void up_fused(const UpLevelDesc& d, hipStream_t st);

// One downward-sweep merge level in one launch, for the same short-interface levels:
// one workgroup per box stages the parent's incoming data t (tp [nbox][nrhs][nbp]),
// copies its I1 / I2 entries into the children's outer rows and writes the children's
// interface rows t3a = Phi^a t (+ t~3a), t3b = Phi^b t (+ t~3b) (tc [2 nbox][nrhs][nbc];
// tta/ttb optional [nbox][nrhs][n3]).  Operators and nrq as for UpLevelDesc.
struct DownLevelDesc {
  int nbox = 0, nbc = 0, n1 = 0, n2 = 0, n3 = 0, nbp = 0, nrhs = 0;
  const int *perm = nullptr, *i1a = nullptr, *i3a = nullptr, *i2b = nullptr, *i3b = nullptr;
  const double* tp = nullptr;
  double* tc = nullptr;
  const double *tta = nullptr, *ttb = nullptr;
  bool c64 = false;
  int per = 0;
  const double *PhiA[SkinnyDesc::kMaxTab] = {}, *PhiB[SkinnyDesc::kMaxTab] = {};
  int nrq[SkinnyDesc::kMaxTab] = {};
};
bool down_fused_fits(int n1, int n2, int n3, int nbp);  // the level's box fits the kernel
void down_fused(const DownLevelDesc& d, hipStream_t st);
void zgemm_skinny(const SkinnyDesc& d, hipStream_t st);

// ------------------------------------------------------------------ complex inversion
// Batched Gauss-Jordan inversion of n x n complex matrices.
// In: A_b (lda, sA).  Out: Inv_b (ldo, sO); Out may alias A (A is read completely before
// Out is written).  info[b] is set to (k+1) if the k-th pivot is exactly zero (info must
// be zeroed by the caller).  Workspace is allocated by the caller through
// zinv_workspace_bytes.  c64: A, Out and the arithmetic are complex64 (strides still in
// complex entries).  Up to 64, and with full_pivoting, partial pivoting over the whole
// column; otherwise (in place only) the diagonal blocks of 64 columns are the pivots,
// each inverted with partial pivoting inside it, and the block steps run on the GEMM.
size_t zinv_workspace_bytes(int n, int batch, bool c64 = false);
void zinv(int n, int batch, const double* A, long lda, long sA, double* Out, long ldo,
          long sO, int* info, void* work, hipStream_t st, bool c64 = false,
          bool full_pivoting = false);

// ------------------------------------------------------------------ leaf stage
struct LeafDesc {
  int p = 0, nleaf = 0;
  int nl1 = 1;                   // leaves per problem
  long h0 = 0;                   // index of the launch's first leaf in the factor
  const double* prm = nullptr;   // device [problem][4]: kappa, Re eta, Im eta, 0
  const double* c = nullptr;     // device [nleaf * ni] in user (grid) leaf order
  const int* leaf_grid = nullptr;  // device [nleaf]: grid index of tree-ordered leaf h
  const double* tab = nullptr;   // device complex line tables, leaf_table_len(p) per problem
  double* BI = nullptr;          // device [nleaf][n*n] complex: [Psi | Y]
  float* BI32 = nullptr;         // if set: [nleaf][n*n] complex64 copy of [Psi | Y], written
                                 // by the Psi / boundary-row kernel (whose outputs then go
                                 // only there)
  double* R = nullptr;           // device [nleaf][nb*nb] complex
  double* Mg = nullptr;          // scratch of the interior inverse (leaf_scratch_bytes)
  int* info = nullptr;           // device [nleaf]
  // Dirichlet-block route (leaf_dir.hip)
  const int* route = nullptr;    // device [problem]: 1 = Dirichlet-block route, 0 = impedance
                                 // route; each route's kernels skip the other's leaves
  const double* rtab = nullptr;  // device real line tables, leaf_rtable_len(p) per problem
  double* X = nullptr;           // scratch [nleaf][n_i x n_b] real: A^{-1} A_ib
  double* Z = nullptr;           // scratch [nleaf][n_b x n_i] real: N_i A^{-1}
  double* Ai = nullptr;          // scratch [nleaf][n_i x n_i] real: A^{-1} (column-major)
};
// scratch the leaf inverse needs for nleaf leaves (0 when it fits in registers)
size_t leaf_scratch_bytes(int p, long nleaf);
// complex entries of the line table: G_x, G_y (m x m), the F_bb^{-1} F_bi line
// coefficients sS, sN, oW, oE, the W = A_ib F_bb^{-1} coefficients wS, wN, wW, wE (m
// each) and the two 2 x 2 inverses of F_bb (S/N pair, W/E pair)
int leaf_table_len(int p);
void leaf_interior_inverse(const LeafDesc& d, hipStream_t st);  // S_i^{-1} -> Y_i block
// Psi_i = -Y_i W, the boundary rows [Psi_b | Y_b] and R, from the Y_i block
void leaf_psi_and_boundary(const LeafDesc& d, hipStream_t st);
// Dirichlet-block route: doubles of the real line table of one problem; the largest c of
// each problem (nprob problems of per_prob samples); A^{-1} into the Y_i block (real
// values); X, Z into scratch and S = F_bb - N_i X into the Psi_b block; R from Psi_b
int leaf_rtable_len(int p);
// leaf_cmax leaves each problem's largest c in cmax as an order-preserving 64-bit key
// (NaN counted as +infinity); leaf_cmax_value turns a key copied to the host back into
// the double
void leaf_cmax(const double* c, int nprob, long per_prob, double* cmax, hipStream_t st);
double leaf_cmax_value(unsigned long long key);
void leaf_dirichlet_inverse(const LeafDesc& d, hipStream_t st);
void leaf_dirichlet_xz(const LeafDesc& d, hipStream_t st);
void leaf_dirichlet_R(const LeafDesc& d, hipStream_t st);

// ------------------------------------------------------------------ merge helpers
struct MergeLevelDesc {
  int nbox = 0;          // number of merges on the level
  int nbc = 0;           // children's boundary size
  int n1 = 0, n2 = 0, n3 = 0, nbp = 0;
  const int* codeA = nullptr;  // device [nbc]: (cls << 16) | k, cls 0 = I1, 1 = I3
  const int* codeB = nullptr;  // device [nbc]: cls 0 = I2, 1 = I3
  const int* perm = nullptr;   // device [nbp]: [I1; I2] position -> parent canonical
  const int* i1a = nullptr;    // device [n1]: I1 positions in alpha's boundary
  const int* i3a = nullptr;    // device [n3]: I3 positions in alpha's boundary
  const int* i2b = nullptr;    // device [n2]: I2 positions in beta's boundary
  const int* i3b = nullptr;    // device [n3]: I3 positions in beta's boundary
  const double* Rc = nullptr;  // children's R, [2*nbox][nbc*nbc]
  double* Rp = nullptr;        // parent R [nbox][nbp*nbp] (may be null: not formed)
  double* R33a = nullptr; double* R33b = nullptr;
  double* R13a = nullptr; double* R23b = nullptr;
  double* R31a = nullptr;      // scratch [nbox][n3*n1]
  double* T = nullptr;         // scratch [nbox][n3*nbp]
  double* PhiB = nullptr;      // [nbox][n3*nbp]
  bool c64 = false;            // the level's blocks (and its parent R) are complex64
  bool child_c64 = false;      // the children's R is complex64
};
void fill_zero(double* p, long ndouble, hipStream_t st);
void fill_zero_int(int* p, long n, hipStream_t st);
void fill_identity(double* p, int n, long stride, int batch, hipStream_t st, bool c64 = false);
// round n doubles to floats (complex128 -> complex64 storage)
void to_c64(const double* src, float* dst, long n, hipStream_t st);
// dst[i] = (double)src[i], i < n
void to_c128(const float* src, double* dst, long n, hipStream_t st);
void merge_extract(const MergeLevelDesc& d, hipStream_t st);
// parent R (written whole by the R^tau products) += blockdiag(R11^a, R22^b)
void merge_add_diag(const MergeLevelDesc& d, hipStream_t st);

// ------------------------------------------------------------------ solve helpers
// h_b = -2 i eta * u_b[0:nb]  for every leaf (u_b is n x nrhs, h_b is nb x nrhs); eta of
// leaf b is that of problem b / nl1 in prm ([problem][4]: kappa, Re eta, Im eta, 0), or,
// when tab is given, in the row tab->p[b / nl1] (problems of several factors)
struct PrmTab { const double* p[SkinnyDesc::kMaxTab] = {}; };
void leaf_h_from_u(int nleaf, int n, int nb, int nrhs, const double* prm, int nl1,
                   const double* u, double* h, hipStream_t st, const PrmTab* tab = nullptr);
// Upward gather of one level: h3a, -h3a (into ttb), -h3b (into v), and the h1/h2 parts
// of the parent's h.  hc: children's h [2*nbox][nbc x nrhs]; hp: [nbox][nbp x nrhs].
// With right-hand sides on the shared-edge rows (jmp: [nrhs][ldj], ja/jb: per merge and
// interface node the index of alpha's / beta's row in jmp, minus jbase), h3a is replaced by
// h3a - j2 (beta's row) and h3b by h3b - j1 (alpha's row).
void up_gather(const MergeLevelDesc& d, int nrhs, const double* hc, double* h3a,
               double* v, double* ttb, double* hp, const double* jmp, long ldj,
               const int* ja, const int* jb, long jbase, hipStream_t st);
// Downward scatter of one level: children's t on I1 / I2 from the parent's t.
void down_scatter(const MergeLevelDesc& d, int nrhs, const double* tp, long ldp,
                  double* tc, hipStream_t st);

// ------------------------------------------------------------------ FP64 residual
// Residual of the global collocation system for nrhs vectors u (grid leaf order), written
// as interior rows rs[r*rs_rhs + l*rs_leaf + k] (k < n_i) and boundary rows
// rb[r*rb_rhs + l*rb_leaf + k] (k < n_b).  Rows on the outer boundary go to
// rt[r*rt_rhs + root position] when rt is given (rb then holds 0 there), else to rb.
// nprob problems of one shape: leaf l' of the launch belongs to problem l' / (nx*ny); u, s,
// jumps hold [nrhs][nprob * nx*ny * len], t and rt [nprob][nrhs][nt].
struct ResidualDesc {
  int p = 0, nx = 0, ny = 0, nprob = 1;
  const double* prm = nullptr;  // device [nprob][4]: kappa, Re eta, Im eta, 0
  const double* D = nullptr;    // [4][p*p] Dx1, Dy1, Dxx, Dyy (column-major, scaled)
  const double* c = nullptr;    // [nleaf * n_i] real
  const double* u = nullptr;    // complex [nrhs][nleaf * n]
  const double* s = nullptr;    // complex [nrhs][nleaf * n_i] or null (zero)
  const double* t = nullptr;    // complex [nrhs][nt] or null (zero)
  const double* jmp = nullptr;  // complex [nrhs][nleaf * n_b] or null (zero)
  double* rs = nullptr; long rs_rhs = 0, rs_leaf = 0;
  double* rb = nullptr; long rb_rhs = 0, rb_leaf = 0;
  double* rt = nullptr;
  int nrhs = 1;
};
void residual(const ResidualDesc& d, int nrhs, hipStream_t st);
// y += x (complex, n entries)
void axpy(long n, const double* x, double* y, hipStream_t st);
// per right-hand side r (vectors of len complex entries, r-major): partial sums of |x|^2
// and |y|^2 over norms_blocks() blocks, part[2*(r*blocks + b) + {0,1}]
int norms_blocks();
void norms_partial(long len, int nrhs, const double* x, const double* y, double* part,
                   hipStream_t st);

}  // namespace hps
