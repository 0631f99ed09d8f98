/*
 * hps.h -- C ABI of the MI355X (gfx950) HPS direct solver for the variable-coefficient
 * Helmholtz impedance problem
 *
 *     -Lap u - kappa^2 c(x) u = s   in Omega = [x0,x1] x [y0,y1]
 *     du/dnu + i eta u        = t   on dOmega,        Re(eta) != 0
 *
 * (eq. (basic) of Beams, Gillman, Hewett, arXiv 1812.07167).  The library implements
 * the precomputation stage (Algorithm 1: batched leaf operators of Sec. 2.1, then the
 * level-by-level merge of Sec. 2.2) and the solve stage (Algorithm 2: upward and
 * downward sweeps) with hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   - Every function returns an int status (HPS_OK = 0 on success).  On failure,
 *     hps_last_error() returns a thread-local message.  No C++ exception crosses the ABI.
 *   - Complex arrays are interleaved (re, im) pairs of double (the layout of C99
 *     double _Complex, std::complex<double> and torch.complex128).  A "complex
 *     pointer" below is a double* to the first real part.
 *   - "device" pointers are HIP device memory of the current device; "host" pointers
 *     are ordinary host memory.  The caller owns every buffer it passes; the library
 *     owns the factor's memory (freed by hps_free).
 *   - Work is ordered on the stream given in hps_opts (NULL = the null stream).
 *     hps_build returns after the factorization has finished (it checks pivots);
 *     hps_solve returns after enqueueing, so u is valid after the stream syncs.
 *
 * Node ordering contract (the paper fixes only I_b = [I_s, I_e, I_n, I_w] in Sec. 2.1
 * and I_b^tau = [I_1, I_2] in Sec. 2.2; the rest is fixed here):
 *   - 1D points on [a,b]: x_k = a + (b-a)(1 - cos(k pi/(p-1)))/2, k = 0..p-1 (ascending
 *     Chebyshev-Lobatto points).
 *   - Leaves: uniform nx x ny grid, leaf index l = iy*nx + ix.
 *   - Within a leaf (n = p^2 - 4 nodes, corners dropped): [S (x ascending), E (y
 *     ascending), N (x ascending), W (y ascending), interior (for j in 1..p-2, for i in
 *     1..p-2)], i.e. I = [I_b, I_i] with m = p-2 nodes per side, n_b = 4m, n_i = m^2.
 *   - Root boundary (nt = 2 (nx + ny) m nodes): [S side: leaves ix = 0..nx-1, each x
 *     ascending; E side: iy = 0..ny-1, y ascending; N side: ix ascending; W side: iy
 *     ascending].
 *   - A node on an edge shared by two leaves appears once per leaf in u; both copies
 *     agree to round-off.
 */
#ifndef HPS_H
#define HPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  HPS_OK = 0,
  HPS_E_INVALID = 1,       /* bad argument (sizes, NULL, NaN, Re(eta) == 0, ...)        */
  HPS_E_NOMEM = 2,         /* device allocation failed                                   */
  HPS_E_SINGULAR = 3,      /* a zero pivot in a leaf or interface inversion              */
  HPS_E_DEVICE = 4,        /* a HIP runtime call failed                                  */
  HPS_E_NOT_CONVERGED = 5, /* mixed-precision refinement did not reach its tolerance     */
  HPS_E_BUSY = 6           /* no capacity: a server refused the request (admission)      */
};

/* Problem geometry: Omega = [x0,x1] x [y0,y1] split into nx x ny equal leaves; nx and
 * ny are powers of two, 1 <= nx*ny <= 65536 (Sec. 2: uniform partition + binary tree). */
typedef struct {
  double x0, x1, y0, y1;
  int32_t nx, ny;
} hps_domain;

/* Arithmetic of the factorization and of the solve sweeps. */
enum {
  HPS_PREC_C128 = 0,  /* complex128 throughout                                            */
  HPS_PREC_MIXED = 1  /* leaves computed in complex128; every merge product, stored merge
                         operator and solve product in complex64 on the matrix cores with
                         FP32 accumulation; the interface inverses W^{-1} of the top
                         fp64_top_levels levels computed in complex128; each solve is then
                         corrected with the FP64 residual of the global collocation system
                         (not in the paper)                                                 */
};

/* Build options.  hps_default_opts() fills the defaults noted below. */
typedef struct {
  int32_t precision;      /* HPS_PREC_C128 (default) or HPS_PREC_MIXED                    */
  int32_t keep_all_R;     /* 1 = keep every box's ItI operator R for inspection (tests);
                             0 = free children's R after each merge, as Sec. 2.4 does     */
  int32_t store_root_R;   /* 1 = form the root's R (Algorithm 1 does; the solve does not
                             use it) (default 1)                                          */
  int32_t profile;        /* 1 = record HIP events around every kernel group of the build
                             and of each solve; read them with hps_stage_times (default 0) */
  void* stream;           /* hipStream_t the work is ordered on (default NULL)            */
  int32_t fp64_top_levels; /* HPS_PREC_MIXED: merge levels 0..fp64_top_levels-1 (the root
                             is level 0) invert W in complex128 (default 3)              */
  int32_t refine_max_iter; /* residual correction steps per solve; -1 = automatic: 10 for
                             HPS_PREC_MIXED, 0 for HPS_PREC_C128 (default -1)            */
  double refine_tol;       /* correction stops once, for every right-hand side r (of
                             every problem of a batched solve, each measured on its own),
                             ||delta_r|| <= refine_tol ||u_r||, or the corrections contract
                             (each below half the last) so that the next one, estimated as
                             ||delta_r||^2 / ||delta_r^prev||, is below that (default 1e-12) */
  int32_t autotune;        /* 1 = time every tile variant of each merge GEMM shape not yet
                             in the process's tuning table and record the fastest (the
                             build synchronizes its stream per new shape); builds launch
                             the recorded variant of a shape, else the default choice
                             (default 0).  Not in the paper: the analog of its per-level
                             calibration of thread counts (Sec. 3).                      */
  int32_t leaf_route;      /* how the leaf operators of Sec. 2.1 are formed (both give B^{-1}
                             of eqs. (homogeneous), (particular) to round-off):
                             0 = automatic (default): per problem, the interior Dirichlet
                             block A = Ahat(I_i, I_i) is inverted in real arithmetic and the
                             boundary unknowns eliminated after it when kappa^2 max(c) is at
                             most half of pi^2 (1/h_x^2 + 1/h_y^2), the smallest eigenvalue of
                             a leaf's Dirichlet Laplacian (A is then safely invertible);
                             otherwise the boundary unknowns are eliminated first through the
                             impedance rows and the complex interior Schur complement is
                             inverted.
                             1 = the impedance-row elimination for every problem.          */
  int32_t interface_pivoting; /* how W = I - R33^b R33^a is inverted (W^{-1} of eq. (talpha)):
                             0 = diagonal blocks of 64 columns as pivots, each inverted with
                             partial pivoting inside it, block steps on the matrix cores
                             (default; W is identity minus a product of two compressions of
                             ItI operators, which for real c and eta are contractions in the
                             boundary quadrature norm, so no exchanges between blocks are
                             needed -- a singular diagonal block repeats the build with 1);
                             1 = partial pivoting over whole columns (LAPACK's choice).     */
} hps_opts;

/* Outcome of the most recent solve on a factor (hps_last_solve_info). */
typedef struct {
  int32_t iterations;  /* residual correction steps taken (0 when correction is off)     */
  int32_t converged;   /* 1 when the last relative correction met refine_tol             */
  double correction;   /* max over right-hand sides (and problems of a batched solve) of
                          ||delta|| / ||u|| in the last step,
                          or of its contraction estimate of the next step where that is
                          what met the tolerance                                        */
} hps_solve_info;

/* Timing of one kernel group (profile = 1).  flops and bytes are the algorithmic work
 * of the group (dense-equivalent counts of the formulas it evaluates, not hardware
 * counters); ms is the summed HIP-event time of its launches on the factor's stream. */
typedef struct {
  char name[32];
  int32_t launches;
  int32_t reserved;
  double ms;
  double flops;
  double bytes;
} hps_stage_time;

typedef struct hps_factor hps_factor;

typedef struct {
  int32_t p, nx, ny, levels; /* levels = log2(nx*ny); level 0 is the root               */
  int64_t nleaf;             /* nx*ny                                                    */
  int64_t n_leaf_nodes;      /* nleaf * (p*p - 4): length of one u vector                */
  int64_t n_interior;        /* nleaf * (p-2)^2: length of one s vector                  */
  int64_t n_root;            /* 2 (nx + ny)(p - 2): length of one t vector               */
  int64_t device_bytes;      /* device memory held by the factor                         */
} hps_factor_info;

/* Which stored operator hps_factor_get copies out. */
enum {
  HPS_OP_PSI = 0,   /* leaf:  Psi (n x n_b), B Psi = [I; 0]      Sec. 2.1.1 eq. (hmgsolnopdef) */
  HPS_OP_Y = 1,     /* leaf:  Y (n x n_i),   B Y = [0; I]        Sec. 2.1.2 eq. (prtsolnopdef) */
  HPS_OP_R = 2,     /* any box with R kept: ItI operator, rows/cols in the box's [S,E,N,W]
                       boundary order (each side in ascending coordinate)                       */
  HPS_OP_WINV = 3,  /* merge: W^{-1}, W = I - R33^b R33^a        Sec. 2.2                       */
  HPS_OP_PHI_A = 4, /* merge: Phi^a (n3 x nb_parent), eq. (talpha); columns in the parent's
                       [S,E,N,W] order                                                          */
  HPS_OP_PHI_B = 5, /* merge: Phi^b (n3 x nb_parent), eq. (tbeta); same column order          */
  HPS_OP_R33A = 6,  /* merge: R33^a (n3 x n3)                                                   */
  HPS_OP_R33B = 7,  /* merge: R33^b (n3 x n3)                                                   */
  HPS_OP_R13A = 8,  /* merge: R13^a (n1 x n3); rows in alpha's boundary order restricted to I1 */
  HPS_OP_R23B = 9   /* merge: R23^b (n2 x n3); rows in beta's boundary order restricted to I2  */
};

/* Thread-local message describing the last failure on this thread ("" if none). */
const char* hps_last_error(void);

/* Library ABI version (major*10000 + minor*100 + patch). */
int32_t hps_version(void);

/* Fill *opts with the defaults. */
void hps_default_opts(hps_opts* opts);

/* Node coordinates in the ordering contract above (host pointers, caller-allocated,
 * each may be NULL):
 *   xy_leaf      [nx*ny*(p*p-4)][2]   all leaf nodes, leaf-major
 *   xy_interior  [nx*ny*(p-2)^2][2]   interior nodes only (where c and s are sampled)
 *   xy_root      [2(nx+ny)(p-2)][2]   root boundary nodes (where t is sampled)
 *   nrm_root     [2(nx+ny)(p-2)][2]   outward unit normals at xy_root
 * Sec. 2.1 (classic Chebyshev product grid with the corners removed). */
int hps_nodes(const hps_domain* dom, int32_t p, double* xy_leaf, double* xy_interior,
              double* xy_root, double* nrm_root);

/* Precomputation stage (Algorithm 1).
 *   dom         geometry (host)
 *   p           Chebyshev points per direction per leaf, 4 <= p <= 16
 *   kappa       wave number, finite and >= 0
 *   eta_re/im   impedance parameter eta (Re(eta) != 0, Definition 2.1)
 *   c_interior  device, [nx*ny*(p-2)^2] real samples of c at the interior nodes in the
 *               ordering contract (C only enters interior collocation rows, Sec. 2.1);
 *               read during the call only
 *   opts        NULL for defaults
 *   out         receives the factor handle; *out = NULL on failure (nothing leaks)
 * Errors: HPS_E_INVALID (arguments), HPS_E_NOMEM, HPS_E_SINGULAR (zero pivot in a leaf
 * or interface inversion), HPS_E_DEVICE. */
int hps_build(const hps_domain* dom, int32_t p, double kappa, double eta_re,
              double eta_im, const double* c_interior, const hps_opts* opts,
              hps_factor** out);

/* Solve stage (Algorithm 2) for nrhs right-hand sides at once.
 *   s   device complex, [nrhs][n_interior] body load at the interior nodes, or NULL for
 *       s = 0 (then only the downward sweep runs, as Sec. 2 notes)
 *   t   device complex, [nrhs][n_root] impedance data on the root boundary
 *   u   device complex, [nrhs][n_leaf_nodes] output, the solution at every leaf node
 * s, t and u must not overlap.  The factor is only read: several solves may use one
 * factor concurrently.  The call takes its workspace from the library's cache of
 * device buffers (see hps_release_cached).
 * Errors: HPS_E_INVALID (NULL factor/t/u, nrhs < 1), HPS_E_NOMEM, HPS_E_DEVICE. */
int hps_solve(hps_factor* f, int32_t nrhs, const double* s, const double* t, double* u);

/* Allocation-free solve, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments,
 * results and errors as hps_solve; in addition it calls no hipMalloc, hipFree or
 * allocating library routine.  Its workspace is carved from a fixed device array of
 * HPS_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on every GPU it runs on until
 * the process ends (the array's device address is looked up once per device, on the
 * first call there).  A call whose workspace exceeds that size (the upward sweep's
 * vectors grow with nrhs and the leaf count; mixed precision adds the correction's
 * residual) fails with HPS_E_INVALID and enqueues nothing.  Every call on one GPU uses
 * the same array, which keeps the last call's contents (nothing is read before it is
 * written): calls that overlap on one GPU -- several streams or host threads -- race, and
 * the caller must order them.  opts.profile records are not taken. */
#define HPS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hps_solve_noalloc(hps_factor* f, int32_t nrhs, const double* s, const double* t,
                      double* u);

/* Cross-problem batching (not in the paper; the paper's parallelism is over the boxes
 * of one problem).  Builds nprob independent problems; problems with the same domain,
 * leaf grid and p are factored together, every leaf and merge-level launch covering all
 * of them.  Groups of different shapes are built at the same time, each on a stream of
 * the library's own (up to 4 at once) that starts after the work queued on
 * opts.stream; the call returns when every group is built, and the handles then use
 * opts.stream.  Arguments are arrays of length nprob with the meaning of hps_build's
 * (c_interior[i] a device pointer); opts apply to all.  out[i] receives problem i's
 * handle; handles of one group share its device memory, which is released with the
 * last of them (hps_free).  Each handle works with every other entry point.  On failure
 * every out[i] is NULL and nothing leaks.  Errors: as hps_build. */
int hps_build_batch(int32_t nprob, const hps_domain* doms, const int32_t* p,
                    const double* kappa, const double* eta_re, const double* eta_im,
                    const double* const* c_interior, const hps_opts* opts, hps_factor** out);

/* Batched solve: for i < nprob, solve problem f[i] for nrhs[i] right-hand sides
 * (s[i] may be NULL, and s itself may be NULL for all-zero body loads; t[i], u[i] as for
 * hps_solve).  Requests on problems of one group run as one solve over all of them (the
 * right-hand sides padded with zeros to the largest nrhs[i] of the group), so every
 * per-level launch covers all those problems.  Requests on problems of different groups
 * that share the leaf grid, p, level precisions and stream, without residual
 * correction, also share every per-level launch, up to 16 problems per solve (each
 * problem's launches cover only its own nrhs[i] right-hand sides).  A problem may
 * appear once per call.  Runs on the stream of f[i]'s factor (the first of each
 * sharing set).  Synchronizes the stream when residual correction is on.  Errors: as
 * hps_solve. */
int hps_solve_batch(int32_t nprob, hps_factor* const* f, const int32_t* nrhs,
                    const double* const* s, const double* const* t, double* const* u);

/* Solve with right-hand sides on the shared-edge rows of the global collocation system
 * (not in the paper; the correction step of a reduced-precision solve).  As hps_solve,
 * plus
 *   jumps  device complex, [nrhs][nx*ny][n_b]: for a node on the edge shared by leaf l
 *          (position k of its boundary, order [S, E, N, W]) and leaf l', the row
 *          F_l u_l + G_l' u_l' = jumps[r][l][k] (F = N + i eta, G = N - i eta with N the
 *          outward normal derivative of each leaf's interpolant, Sec. 2.1); entries on
 *          the outer boundary are ignored.  NULL means zero.
 * At every merge the interface conditions of Sec. 2.2 become t3^a = -g3^b + j1 and
 * t3^b = -g3^a + j2, i.e. eqs. (talpha)/(tbeta) with h3^b - j1 and h3^a - j2 in place of
 * h3^b and h3^a in the particular parts.
 * Errors: as hps_solve. */
int hps_solve_jumps(hps_factor* f, int32_t nrhs, const double* s, const double* t,
                    const double* jumps, double* u);

/* FP64 residual b - A u of the global collocation system that the factorization
 * eliminates (rows: interior collocation rows Ahat(I_i, I) u_l = s of Sec. 2.1, impedance
 * rows F u_l = t on the outer boundary, and F_l u_l + G_l' u_l' = jumps on shared edges),
 * evaluated matrix-free from the differentiation matrices, c, kappa and eta.
 *   s, t, jumps  device complex as for hps_solve_jumps (NULL = zero)
 *   u            device complex, [nrhs][n_leaf_nodes]
 *   r            device complex, [nrhs][n_leaf_nodes] output in the layout of u: for each
 *                leaf the n_b boundary rows (order [S, E, N, W]) then the n_i interior
 *                rows
 * Stream-ordered on the factor's stream; no synchronization.
 * Errors: HPS_E_INVALID, HPS_E_DEVICE. */
int hps_residual(hps_factor* f, int32_t nrhs, const double* s, const double* t,
                 const double* jumps, const double* u, double* r);

/* Iterations and last relative correction of the factor's most recent hps_solve /
 * hps_solve_jumps.  With residual correction on, those calls synchronize the stream
 * once per step and return HPS_E_NOT_CONVERGED (u holding the last iterate) when the
 * tolerance is not met within refine_max_iter steps. */
int hps_last_solve_info(const hps_factor* f, hps_solve_info* info);

/* Sizes of a factor. */
int hps_factor_query(const hps_factor* f, hps_factor_info* info);

/* Copy one stored operator to a host buffer (column-major complex, ld = rows).
 *   what    one of HPS_OP_*
 *   level   tree level (0 = root, levels = leaves); merges live on levels 0..levels-1
 *   box     box index within the level, 0..2^level-1, in the level's tree order (the
 *           children of box q of level l are boxes 2q (alpha: left / bottom) and 2q+1
 *           (beta: right / top) of level l+1)
 *   dst     host, capacity dst_len complex entries; rows/cols receive the shape
 * Errors: HPS_E_INVALID if the operator is not stored (e.g. R freed) or too large. */
int hps_factor_get(const hps_factor* f, int32_t what, int32_t level, int32_t box,
                   double* dst, int64_t dst_len, int32_t* rows, int32_t* cols);

/* Leaf range [ix0,ix1) x [iy0,iy1) covered by box `box` of level `level`. */
int hps_factor_box(const hps_factor* f, int32_t level, int32_t box, int32_t* ix0,
                   int32_t* ix1, int32_t* iy0, int32_t* iy1);

/* Per-kernel-group timings of the factor's build (which = 0) or of its most recent
 * solve (which = 1), recorded when opts.profile = 1.  Writes up to cap records to out
 * (host) and the number of records to *n.  Waits for the recorded events.  Not
 * meaningful while several solves run concurrently on the factor. */
int hps_stage_times(const hps_factor* f, int32_t which, hps_stage_time* out, int32_t cap,
                    int32_t* n);

/* Release a factor (NULL is a no-op). */
void hps_free(hps_factor* f);

/* Tuning table of the merge GEMMs (filled by builds with opts.autotune = 1; shared by
 * every build in the process).  The file format is text, one line per GEMM shape:
 * "M N K batch flags variant" (flags: 1 real A, 2 real B, 4 complex64, 8 beta != 0,
 * 16 scattered output; variant: tile "MxN", e.g. 128x64).  load merges into the table.
 * Errors: HPS_E_INVALID (NULL, unreadable or malformed file). */
int hps_autotune_entries(int32_t* n);
int hps_autotune_clear(void);
int hps_autotune_save(const char* path);
int hps_autotune_load(const char* path);

/* Solve workspaces and staging come from a cache of device buffers that the library
 * keeps per device; a buffer freed by a finished call stays allocated for the next call
 * (reuse is ordered after the previous use with an event).  This frees the idle ones
 * after synchronizing the device, and drops the cached plans (tree and index maps of a
 * factor shape, reused by later builds of that shape) that no factor uses.
 * Errors: HPS_E_DEVICE. */
int hps_release_cached(void);

/* Allocator hook: route the library's device memory (factors, build scratch, solve
 * workspaces, staging) through the caller's allocator, e.g. a framework's caching
 * allocator, instead of hipMalloc and the library's buffer cache.
 *   alloc(bytes, stream, ctx)  returns device memory of at least bytes on the current
 *       device, usable by work on `stream` (a hipStream_t; NULL for buffers that live
 *       across calls), or NULL when it has none (the library call then fails with
 *       HPS_E_NOMEM).
 *   free(ptr, stream, ctx)  returns ptr.  Work queued on `stream` may still use it: a
 *       stream-ordered allocator reuses it after that work; for buffers handed out with
 *       stream NULL the library synchronizes the device first.
 * Every buffer goes back to the hook that provided it, also after the hook changes.
 * The index maps of a plan are shared by every factor of one shape (device, leaf grid,
 * p, problem count) and come from the allocator that was active when the shape was
 * first planned; hps_release_cached drops the cached plans no factor uses.
 * Both functions NULL restores the library's own allocator; one of them NULL is
 * HPS_E_INVALID.  Installing a hook releases the idle cached buffers.  The functions
 * may be called from the request loop's threads.  Errors: HPS_E_INVALID, HPS_E_DEVICE. */
typedef void* (*hps_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*hps_free_fn)(void* ptr, void* stream, void* ctx);
int hps_set_allocator(hps_alloc_fn alloc, hps_free_fn free, void* ctx);

/* Device bytes that hps_build of one problem of this shape would use, from the same plan
 * the build lays out (host arithmetic only; nothing is allocated):
 *   build_peak  the most held at once during the build (operators, ItI buffers, scratch)
 *   resident    what the factor holds afterwards (hps_factor_query's device_bytes, up to
 *               the rounding of small tables)
 * Either output may be NULL (not both).  Errors: HPS_E_INVALID. */
int hps_estimate_bytes(const hps_domain* dom, int32_t p, const hps_opts* opts,
                       int64_t* build_peak, int64_t* resident);

/* ---------------------------------------------------------------- request loop
 * Serving (not in the paper).  A server keeps factored problems resident in device
 * memory and runs build and solve requests on a pool of work slots, each a host thread
 * with its own stream, so that work of several requests overlaps on the device.
 *   - Admission by memory: every work item (a build, or one solve) starts
 *     only when the bytes it needs (hps_estimate_bytes' build_peak, or the solve's
 *     workspace and staging) fit under the budget beside what is already committed
 *     (resident factors, running items).  If it does not fit, factors of idle problems
 *     (no queued or running request) are freed, least recently used first (when
 *     evict_idle is set; a solve evicts only while no other solve runs, otherwise it
 *     waits for their memory to come back); an evicted problem is rebuilt from the
 *     server's copy of its data when its next solve request comes up.
 *   - Continuous batching: when a slot takes a problem's solve, it merges every queued
 *     request of that problem (up to max_batch_rhs right-hand sides) into one solve.
 *     With share_problems set, the same solve also takes the queued requests of other
 *     idle resident problems that can share its launches (same leaf grid, p and level
 *     precisions, no residual correction; oldest first, up to 16 problems, each up to
 *     max_batch_rhs), so every per-level launch covers all of them.  Requests that
 *     arrive while others run are taken as soon as a slot and memory free up.
 *   - Solve slots: the first solve_slots slots never take a build, so a solve does not
 *     wait for a slot behind long builds.
 *   - A solve or build whose allocation fails for want of device memory while other work
 *     runs is put back in the queue and retried once some of that work has ended
 *     (stats.retried); with nothing else running it fails with HPS_E_NOMEM.
 * A request's result does not depend on what it was batched with beyond round-off.
 * Inputs (c, s, t) must be complete on the device when submitted (the server's streams
 * do not wait on the caller's); u is complete when its completion is returned by
 * hps_server_poll.  Buffers passed to submit_solve must stay valid until then. */
typedef struct hps_server hps_server;

typedef struct {
  int32_t slots;              /* work slots: streams and host threads (default 4)           */
  int32_t max_batch_rhs;      /* right-hand sides merged into one solve (default 64)        */
  int32_t max_pending_builds; /* queued builds beyond which submit_build returns
                                 HPS_E_BUSY (default 64)                                   */
  int32_t evict_idle;         /* 1 = free idle factors, least recently used first, to admit
                                 work (default 1)                                          */
  int32_t solve_slots;        /* slots that take only solves (default 1; at most slots - 1) */
  int32_t share_problems;     /* 1 = one solve serves several shareable problems
                                 (default 1)                                               */
} hps_server_opts;

enum { HPS_REQ_BUILD = 0, HPS_REQ_SOLVE = 1 };

typedef struct {
  uint64_t req;        /* id returned by the submit call                                  */
  uint64_t problem;    /* problem id                                                       */
  int32_t kind;        /* HPS_REQ_BUILD or HPS_REQ_SOLVE                                   */
  int32_t status;      /* HPS_OK or the error code of the work item                       */
  int32_t nrhs;        /* right-hand sides of the request (0 for a build)                */
  int32_t batch_rhs;   /* right-hand sides of the solve that served it                   */
  int32_t iterations;  /* residual-correction steps of that solve                        */
  int32_t rebuilt;     /* 1 if the factor was rebuilt after an eviction to serve it       */
  double t_submit;     /* seconds since hps_server_create: submission,                    */
  double t_start;      /*   start of the work item that served it,                        */
  double t_end;        /*   and its end (results complete)                                */
} hps_completion;

typedef struct {
  int64_t builds, rebuilds, evictions;  /* factorizations done, of them after eviction   */
  int64_t solves, rhs, batches;         /* solve requests done, their RHS, solve calls    */
  int64_t rejected, failed;             /* submissions refused (HPS_E_BUSY), failed items */
  int32_t resident, pending;            /* problems with a factor; requests not returned  */
  int32_t max_concurrent;               /* most work items that ran at once               */
  int32_t slots;
  double p50_ms, p99_ms, max_ms;        /* solve latency, submission to completion        */
  double wall_s;                        /* first submission to last completion            */
  double rhs_per_s, solves_per_s;       /* over wall_s                                    */
  int64_t budget_bytes, committed_bytes, peak_committed_bytes;
  int64_t shared_batches;               /* solve calls that served several problems       */
  int64_t shared_problems;              /* problems those calls served, summed            */
  int64_t retried;                      /* solves and builds put back in the queue after
                                           running out of device memory beside other
                                           running work                                  */
} hps_stats;

/* Fill *opts with the defaults. */
void hps_server_default_opts(hps_server_opts* opts);

/* Start a server on the current device.  hbm_budget: bytes the server may commit (0 =
 * 90% of the device memory free at the call); opts NULL for defaults.
 * Errors: HPS_E_INVALID, HPS_E_DEVICE. */
int hps_server_create(size_t hbm_budget, const hps_server_opts* opts, hps_server** out);

/* Queue the factorization of a problem (arguments as for hps_build; opts.stream is
 * ignored, opts.profile must be 0).  c_interior is copied before the call returns.
 * *problem receives the id to solve with, *req the id of its completion.
 * Errors: HPS_E_INVALID; HPS_E_BUSY when the build alone exceeds the budget or too many
 * builds are queued (the request is rejected); HPS_E_NOMEM, HPS_E_DEVICE. */
int hps_server_submit_build(hps_server* srv, const hps_domain* dom, int32_t p, double kappa,
                            double eta_re, double eta_im, const double* c_interior,
                            const hps_opts* opts, uint64_t* problem, uint64_t* req);

/* Queue a solve of nrhs right-hand sides of a problem (s, t, u as for hps_solve; device
 * pointers owned by the caller, valid until the completion is returned).  Allowed as
 * soon as the problem's build is submitted.  Errors: HPS_E_INVALID (unknown or released
 * problem, arguments). */
int hps_server_submit_solve(hps_server* srv, uint64_t problem, int32_t nrhs, const double* s,
                            const double* t, double* u, uint64_t* req);

/* Drop a problem: its factor and data are freed once its queued requests are done;
 * later submissions for it fail with HPS_E_INVALID. */
int hps_server_release(hps_server* srv, uint64_t problem);

/* Return up to max completions (host array out) in completion order; *n receives the
 * count.  Waits up to timeout_ms for the first one (0 = do not wait). */
int hps_server_poll(hps_server* srv, hps_completion* out, int32_t max, int32_t timeout_ms,
                    int32_t* n);

/* Counters and solve-latency percentiles so far. */
int hps_server_stats(hps_server* srv, hps_stats* stats);

/* Stop the server: running work items finish, queued requests are dropped without a
 * completion, every factor is freed.  NULL is a no-op. */
void hps_server_destroy(hps_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* HPS_H */
