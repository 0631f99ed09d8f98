// C ABI of the HPS library: plan (tree, index maps, spectral matrices), the build
// driver (Algorithm 1 as one batched leaf stage plus one batched merge pass per tree
// level) and the solve driver (Algorithm 2 as one batched pass per level, upward then
// downward).  Host code; all arithmetic on the hot path runs in the HIP kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/hps.h"
#include "kernels.hpp"
#include "serve_hooks.hpp"

// Device memory of the allocation-free solve (hps_solve_noalloc): a fixed array that every
// GPU the library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch below).
constexpr size_t kNoAllocScratch = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratch];

namespace hps {
namespace {

thread_local std::string g_err;

// ------------------------------------------------------------------ device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  // Large buffers (operator arenas, ItI buffers, build scratch) come from the library's
  // buffer cache, so that repeated builds of one shape do not map fresh memory each
  // time; their release waits for the device, as hipFree does.
  static constexpr size_t kCached = size_t(64) << 20;
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    if (void* q = hook_alloc(b, nullptr)) {  // the caller's allocator, when installed
      p = q;
      bytes = b;
      return;
    }
    if (b >= kCached) {
      p = ws_alloc_idle(b);
      bytes = b;
      return;
    }
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(e == hipErrorOutOfMemory ? HPS_E_NOMEM : HPS_E_DEVICE,
                  "device allocation of " + std::to_string(b) + " bytes failed: " +
                      hipGetErrorString(e));
    }
    bytes = b;
  }
  void release() {
    if (p && !hook_free(p, nullptr, true)) {
      if (bytes >= kCached) ws_free_idle(p);
      else (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  double* d() const { return static_cast<double*>(p); }
  int* i() const { return static_cast<int*>(p); }
  long* l() const { return static_cast<long*>(p); }
};

// Non-owning slice of an arena.
struct View {
  void* p = nullptr;
  size_t bytes = 0;
  double* d() const { return static_cast<double*>(p); }
  int* i() const { return static_cast<int*>(p); }
};

// Carves 256-byte aligned slices out of one allocation; a first pass with base ==
// nullptr only measures.
struct Carver {
  char* base = nullptr;
  size_t used = 0;
  View take(size_t bytes) {
    View v;
    v.bytes = bytes;
    v.p = base ? base + used : nullptr;
    used += (bytes + 255) & ~size_t(255);
    return v;
  }
};

template <class T>
void upload(DevBuf& b, const std::vector<T>& v) {
  b.alloc(v.size() * sizeof(T));
  if (!v.empty()) HPS_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// ------------------------------------------------------------------ spectral matrices
// Chebyshev-Lobatto points (ascending) and the classic differentiation matrix
// (Sec. 2.1; Trefethen's construction): off-diagonal (c_i/c_j)(-1)^{i+j}/(x_i-x_j),
// diagonal = -(sum of the off-diagonal row).
void cheb(int p, std::vector<double>& x, std::vector<double>& D) {
  x.resize(p);
  for (int k = 0; k < p; ++k) x[k] = -std::cos(M_PI * k / (p - 1));
  D.assign((size_t)p * p, 0.0);
  for (int i = 0; i < p; ++i) {
    double ci = (i == 0 || i == p - 1) ? 2.0 : 1.0, rs = 0.0;
    for (int j = 0; j < p; ++j) {
      if (i == j) continue;
      double cj = (j == 0 || j == p - 1) ? 2.0 : 1.0;
      double v = (ci / cj) * (((i + j) & 1) ? -1.0 : 1.0) / (x[i] - x[j]);
      D[i + (size_t)p * j] = v;
      rs += v;
    }
    D[i + (size_t)p * i] = -rs;
  }
}

// ------------------------------------------------------------------ plan
struct LevelPlan {
  int nbox = 0;
  int wx = 0, wy = 0;     // parent box size in leaves
  bool split_x = true;
  int nbc = 0, nbp = 0, n1 = 0, n2 = 0, n3 = 0;
  std::vector<int> codeA, codeB, perm, i1a, i3a, i2b, i3b;
  // per merge and interface node: index of alpha's / beta's shared-edge row in an
  // [nleaf][nb] array of boundary rows (grid leaf order)
  std::vector<int> ja, jb;
  DevBuf dmaps;  // codeA | codeB | perm | i1a | i3a | i2b | i3b | ja | jb
  const int* dcodeA = nullptr; const int* dcodeB = nullptr; const int* dperm = nullptr;
  const int* di1a = nullptr; const int* di3a = nullptr; const int* di2b = nullptr;
  const int* di3b = nullptr; const int* dja = nullptr; const int* djb = nullptr;
  // stored operators of the level (Sec. 2.4), slices of the factor's arena
  View Winv, R33a, R33b, R13a, R23b, PhiA, PhiB;
  bool c64 = false;    // the level's operators (and its R) are complex64
  bool inv64 = false;  // complex64 level whose W is inverted in complex128
};

struct Geo { int ix0, iy0, wx, wy; };

// The part of a plan that depends only on the device, the leaf grid, p and the number of
// problems of a group: the tree, each level's sizes and index maps (host and device),
// and the device leaf maps.  Shared, read-only, by every group of that shape.
struct PlanShape {
  int L = 0;
  std::vector<std::vector<Geo>> geo;
  std::vector<int> nbl;
  std::vector<LevelPlan> lv;  // sizes, maps and their device copies (no operator views)
  DevBuf dleaf_grid, dxoff, duoff;
  size_t bytes = 0;           // device bytes of the maps
};
// The plan cache.  It lives until the process ends and is never destroyed (its device
// memory must not be freed during static destruction, when the runtime may be gone).
typedef std::tuple<int, int, int, int, int> PlanKey;  // device, nx, ny, p, problems
struct PlanCache {
  std::mutex mu;
  std::map<PlanKey, std::shared_ptr<const PlanShape>> shapes;
  std::deque<PlanKey> order;  // oldest first
};
PlanCache& plan_cache() {
  static PlanCache* c = new PlanCache;
  return *c;
}
constexpr size_t kPlanCache = 32;

// ------------------------------------------------------------------ stage timers
// HIP events around kernel groups on the factor's stream (opts.profile = 1).  The
// flops/bytes attached to a record are the algorithmic work of the launches it covers.
struct StageRec {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  double flops = 0, bytes = 0;
};

struct Profiler {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<StageRec> recs;
  Profiler() = default;
  Profiler(const Profiler&) = delete;
  Profiler& operator=(const Profiler&) = delete;
  ~Profiler() { clear(); }
  void clear() {
    for (auto& r : recs) {
      if (r.a) (void)hipEventDestroy(r.a);
      if (r.b) (void)hipEventDestroy(r.b);
    }
    recs.clear();
  }
  void reset(bool enable, hipStream_t s) {
    clear();
    on = enable;
    st = s;
  }
  int begin(const char* name, double flops, double bytes) {
    StageRec r;
    r.name = name;
    r.flops = flops;
    r.bytes = bytes;
    HPS_HIP(hipEventCreate(&r.a));
    HPS_HIP(hipEventCreate(&r.b));
    HPS_HIP(hipEventRecord(r.a, st));
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int i) { (void)hipEventRecord(recs[i].b, st); }
};

struct Stage {
  Profiler& p;
  int idx = -1;
  Stage(Profiler& pr, const char* name, double flops, double bytes) : p(pr) {
    if (p.on) idx = p.begin(name, flops, bytes);
  }
  ~Stage() {
    if (idx >= 0) p.end(idx);
  }
};

void timed_gemm(Profiler& pr, const char* name, const GemmDesc& g, hipStream_t st,
                bool tune) {
  // the autotuner measures the tile variants for a shape it has not seen yet; the launch
  // below then uses the winner
  if (tune) zgemm_tune(g, st);
  const double mnk = (double)g.M * g.N * g.K * g.batch;
  const double fl = (g.a_real || g.b_real) ? 4.0 * mnk : 8.0 * mnk;
  const double by = (double)g.batch * ((double)g.M * g.K * (g.a_real ? 8 : 16) +
                                       (double)g.K * g.N * (g.b_real ? 8 : 16) +
                                       (double)g.M * g.N * 16 * (g.beta != 0.0 ? 2 : 1) +
                                       (g.C0r ? (double)g.M * g.N * 8 : 0.0));
  // one record name per kernel variant, so that a record's launches are launches of one
  // kernel (what a profiler's per-kernel average refers to)
  const std::string nm = std::string(name) + "[" + zgemm_variant(g) + "]";
  Stage s(pr, nm.c_str(), fl, by);
  zgemm(g, st);
}

void timed_skinny(Profiler& pr, const char* name, const SkinnyDesc& k, hipStream_t st) {
  const double nb = k.A2 ? 2.0 * k.batch : k.batch;  // a second operator doubles the work
  const double fl = 8.0 * k.M * k.K * (double)k.nrhs * nb;
  const double by = nb * ((double)k.M * k.K * 16 + (double)(k.K + k.M) * k.nrhs * 16);
  Stage s(pr, name, fl, by);
  zgemm_skinny(k, st);
}

bool split_x_rule(int wx, int wy) {
  if (wy == 1) return true;
  if (wx == 1) return false;
  return wx >= wy;  // longer side; ties split x
}

}  // namespace
}  // namespace hps

// Factorizations of nprob problems of one shape (domain, leaf grid, p) held together:
// every level's launches cover all of them (cross-problem batching).  Problem b owns
// leaves [b nl1, (b+1) nl1) and, on level l, boxes [b 2^l, (b+1) 2^l) in tree order.
struct hps_group {
  int p = 0, m = 0, n = 0, nb = 0, ni = 0;
  int nx = 0, ny = 0, L = 0;
  int nprob = 1;                           // problems in the group
  int nl1 = 0;                             // leaves per problem (nx * ny)
  int nleaf = 0;                           // leaves of all problems
  double x0 = 0, x1 = 0, y0 = 0, y1 = 0;
  std::vector<double> prm_h;               // [nprob][4]: kappa, Re eta, Im eta, 0
  hps::DevBuf dprm;
  hipStream_t stream = nullptr;
  hps_opts opts{};
  std::vector<std::vector<hps::Geo>> geo;  // per level, tree order
  std::vector<hps::LevelPlan> lv;          // merges producing level l (l = 0..L-1)
  std::vector<int> leaf_grid;              // tree-ordered leaf -> grid index
  // the tree and index maps, shared by every group of the same shape (plan cache), and
  // the device copies of the leaf maps it holds
  std::shared_ptr<const hps::PlanShape> shape;
  const int* pleaf_grid = nullptr;  // tree-ordered leaf -> grid index
  const long* pxoff = nullptr;      // leaf -> offset of its interior nodes in s
  const long* puoff = nullptr;      // leaf -> offset of its nodes in u
  hps::DevBuf dD, dLT;
  hps::DevBuf dRT;                         // [nprob] real line tables of the Dirichlet route
  hps::DevBuf droute;                      // [nprob] int: 1 = Dirichlet-block leaf route
  hps::DevBuf dcmax;                       // [nprob] largest c of each problem (route test)
  std::vector<int> route_h;                // host copy of droute
  hps::DevBuf ops;                         // arena: [Psi | Y] of every leaf + merge operators
  hps::View BI;                            // [nleaf][n*n] complex128 [Psi | Y] (complex128
                                           // precision only)
  hps::View BI32;                          // mixed precision: complex64 copy of [Psi | Y]
  bool mixed = false;                      // opts.precision == HPS_PREC_MIXED
  bool full_pivoting = false;              // interface inverses pivot over whole columns
                                           // (set when the block-pivot form broke down)
  hps::DevBuf rbuf[2];                     // ping-pong ItI operators (level l uses l % 2)
  std::vector<hps::DevBuf> rkeep;          // every level's R when opts.keep_all_R
  std::vector<hps::View> R;                // per level ItI operators (L+1 entries)
  std::vector<char> R_valid;               // R of the level still holds its operator
  std::vector<int> nbl;                    // boundary size per level
  hps::Profiler build_prof, solve_prof;
  hps::DevBuf dc;                          // c at the interior nodes (for the FP64 residual)
  hps_solve_info last_info{};              // of the most recent solve
  size_t bytes() const {
    size_t t = ops.bytes + (shape ? shape->bytes : 0) + dD.bytes + dLT.bytes + dRT.bytes +
               droute.bytes + dcmax.bytes + rbuf[0].bytes +
               rbuf[1].bytes + dc.bytes;
    for (auto& r : rkeep) t += r.bytes;
    return t + dprm.bytes;
  }
};

// Public handle: problem b0 of a group (the group lives while any handle does).
struct hps_factor {
  std::shared_ptr<hps_group> g;
  int b0 = 0;
};

namespace hps {
namespace {

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

void make_plan(hps_group& f) {
  const int m = f.m;
  f.L = ilog2(f.nl1);
  f.geo.assign(f.L + 1, {});
  f.geo[0].push_back({0, 0, f.nx, f.ny});
  f.lv.clear();
  f.lv.resize(f.L);
  f.nbl.assign(f.L + 1, 0);
  for (int l = 0; l <= f.L; ++l) {
    const Geo& g0 = f.geo[l][0];
    f.nbl[l] = 2 * (g0.wx + g0.wy) * m;
    if (l == f.L) break;
    const bool sx = split_x_rule(g0.wx, g0.wy);
    for (const Geo& g : f.geo[l]) {
      if (sx) {
        int w = g.wx / 2;
        f.geo[l + 1].push_back({g.ix0, g.iy0, w, g.wy});
        f.geo[l + 1].push_back({g.ix0 + w, g.iy0, w, g.wy});
      } else {
        int h = g.wy / 2;
        f.geo[l + 1].push_back({g.ix0, g.iy0, g.wx, h});
        f.geo[l + 1].push_back({g.ix0, g.iy0 + h, g.wx, h});
      }
    }
    LevelPlan& P = f.lv[l];
    P.nbox = (1 << l) * f.nprob;
    P.wx = g0.wx;
    P.wy = g0.wy;
    P.split_x = sx;
    const int wx = g0.wx, wy = g0.wy;
    if (sx) {
      const int wc = wx / 2;
      P.nbc = 2 * (wc + wy) * m;
      P.n3 = wy * m;
      P.n1 = P.n2 = 2 * wc * m + wy * m;
      P.codeA.resize(P.nbc);
      P.codeB.resize(P.nbc);
      const int S = wc * m, E = wy * m;  // child side lengths (S = N, E = W)
      for (int t = 0; t < S; ++t) {
        P.codeA[t] = t;                                   // S_a -> I1
        P.codeA[S + E + t] = S + t;                       // N_a -> I1
        P.codeB[t] = t;                                   // S_b -> I2
        P.codeB[S + E + t] = S + E + t;                   // N_b -> I2
      }
      for (int t = 0; t < E; ++t) {
        P.codeA[S + t] = (1 << 16) | t;                   // E_a -> I3
        P.codeA[2 * S + E + t] = 2 * S + t;               // W_a -> I1
        P.codeB[S + t] = S + t;                           // E_b -> I2
        P.codeB[2 * S + E + t] = (1 << 16) | t;           // W_b -> I3
      }
      P.nbp = 2 * (wx + wy) * m;
      P.perm.resize(P.nbp);
      const int pS = 0, pE = wx * m, pN = wx * m + wy * m, pW = 2 * wx * m + wy * m;
      for (int t = 0; t < S; ++t) {
        P.perm[t] = pS + t;                               // S_a
        P.perm[S + t] = pN + t;                           // N_a
        P.perm[P.n1 + t] = pS + S + t;                    // S_b
        P.perm[P.n1 + S + E + t] = pN + S + t;            // N_b
      }
      for (int t = 0; t < E; ++t) {
        P.perm[2 * S + t] = pW + t;                       // W_a
        P.perm[P.n1 + S + t] = pE + t;                    // E_b
      }
    } else {
      const int hc = wy / 2;
      P.nbc = 2 * (wx + hc) * m;
      P.n3 = wx * m;
      P.n1 = P.n2 = wx * m + 2 * hc * m;
      P.codeA.resize(P.nbc);
      P.codeB.resize(P.nbc);
      const int S = wx * m, E = hc * m;
      for (int t = 0; t < S; ++t) {
        P.codeA[t] = t;                                   // S_a -> I1
        P.codeA[S + E + t] = (1 << 16) | t;               // N_a -> I3
        P.codeB[t] = (1 << 16) | t;                       // S_b -> I3
        P.codeB[S + E + t] = E + t;                       // N_b -> I2
      }
      for (int t = 0; t < E; ++t) {
        P.codeA[S + t] = S + t;                           // E_a -> I1
        P.codeA[2 * S + E + t] = S + E + t;               // W_a -> I1
        P.codeB[S + t] = t;                               // E_b -> I2
        P.codeB[2 * S + E + t] = E + S + t;               // W_b -> I2
      }
      P.nbp = 2 * (wx + wy) * m;
      P.perm.resize(P.nbp);
      const int pS = 0, pE = wx * m, pN = wx * m + wy * m, pW = 2 * wx * m + wy * m;
      for (int t = 0; t < S; ++t) {
        P.perm[t] = pS + t;                               // S_a
        P.perm[P.n1 + E + t] = pN + t;                    // N_b
      }
      for (int t = 0; t < E; ++t) {
        P.perm[S + t] = pE + t;                           // E_a
        P.perm[S + E + t] = pW + t;                       // W_a
        P.perm[P.n1 + t] = pE + E + t;                    // E_b
        P.perm[P.n1 + E + S + t] = pW + E + t;            // W_b
      }
    }
    P.i1a.assign(P.n1, -1);
    P.i3a.assign(P.n3, -1);
    P.i2b.assign(P.n2, -1);
    P.i3b.assign(P.n3, -1);
    for (int pos = 0; pos < P.nbc; ++pos) {
      int ca = P.codeA[pos], cb = P.codeB[pos];
      if (ca >> 16) P.i3a[ca & 0xffff] = pos; else P.i1a[ca] = pos;
      if (cb >> 16) P.i3b[cb & 0xffff] = pos; else P.i2b[cb] = pos;
    }
    for (int v : P.i1a) if (v < 0) throw Error(HPS_E_INVALID, "plan: I1 map incomplete");
    for (int v : P.i3a) if (v < 0) throw Error(HPS_E_INVALID, "plan: I3 map incomplete");
    for (int v : P.i2b) if (v < 0) throw Error(HPS_E_INVALID, "plan: I2 map incomplete");
    for (int v : P.i3b) if (v < 0) throw Error(HPS_E_INVALID, "plan: I3 map incomplete");
    std::vector<int> seen(P.nbp, 0);
    for (int v : P.perm) {
      if (v < 0 || v >= P.nbp || seen[v]) throw Error(HPS_E_INVALID, "plan: perm not bijective");
      seen[v] = 1;
    }
    // I3 runs along alpha's E side (x split) or N side (y split) in ascending coordinate,
    // m nodes per leaf edge; beta sees the same nodes on its W / S side
    P.ja.resize((size_t)P.nbox * P.n3);
    P.jb.resize((size_t)P.nbox * P.n3);
    for (int b = 0; b < P.nbox; ++b) {
      const int prob = b >> l;  // boxes of problem prob: [prob 2^l, (prob+1) 2^l)
      const Geo& g = f.geo[l][b & ((1 << l) - 1)];
      for (int t = 0; t < P.n3; ++t) {
        const int blk = t / m, q = t % m;
        int la, lb, pa, pb;
        if (sx) {
          const int iy = g.iy0 + blk, ixa = g.ix0 + g.wx / 2 - 1;
          la = iy * f.nx + ixa; lb = la + 1; pa = m + q; pb = 3 * m + q;
        } else {
          const int ix = g.ix0 + blk, iya = g.iy0 + g.wy / 2 - 1;
          la = iya * f.nx + ix; lb = la + f.nx; pa = 2 * m + q; pb = q;
        }
        P.ja[(size_t)b * P.n3 + t] = (prob * f.nl1 + la) * f.nb + pa;
        P.jb[(size_t)b * P.n3 + t] = (prob * f.nl1 + lb) * f.nb + pb;
      }
    }
  }
  f.leaf_grid.resize(f.nleaf);
  for (int h = 0; h < f.nleaf; ++h) {
    const Geo& g = f.geo[f.L][h % f.nl1];
    f.leaf_grid[h] = (h / f.nl1) * f.nl1 + g.iy0 * f.nx + g.ix0;
  }
}

// ------------------------------------------------------------------ leaf line tables
void leaf_table_one(const hps_group& f, const double* all, double er, double ei, double* out);
void leaf_rtables(hps_group& f, const double* all);
// The leaf stage eliminates the boundary nodes through the impedance rows F = N + i eta
// (Sec. 2.1).  F_bb couples only the two end nodes of a grid line: (S_i, N_i) through
// the first and last rows of D_y, (W_j, E_j) through those of D_x.  With their 2 x 2
// inverses B (S/N) and C (W/E):
//   (F_bb^{-1} F_bi) rows:  S_i: sS[l] = -B11 Dy(0,l) + B12 Dy(p-1,l) on nodes (i, l),
//                           N_i: sN[l] = -B21 Dy(0,l) + B22 Dy(p-1,l), and W_j / E_j
//                           likewise with C and D_x on nodes (k, j): oW[k], oE[k];
//   S_i = A_ii - A_ib F_bb^{-1} F_bi = -(G_x (x) I) - (I (x) G_y) - kappa^2 diag(c),
//     G_x(i,k) = Dxx(i,k) - Dxx(i,0) oW[k] - Dxx(i,p-1) oE[k],
//     G_y(j,l) = Dyy(j,l) - Dyy(j,0) sS[l] - Dyy(j,p-1) sN[l];
//   W = A_ib F_bb^{-1}: row (i, j) has wS[j] = -Dyy(j,0) B11 - Dyy(j,p-1) B21 in column
//     S_i, wN[j] = -Dyy(j,0) B12 - Dyy(j,p-1) B22 in N_i, wW[i] = -Dxx(i,0) C11 -
//     Dxx(i,p-1) C21 in W_j and wE[i] = -Dxx(i,0) C12 - Dxx(i,p-1) C22 in E_j.
// (A = -Dxx - Dyy - kappa^2 c, so A_ib holds -Dxx(i,0), -Dxx(i,p-1), -Dyy(j,0),
// -Dyy(j,p-1).)  Indices i, j, k, l run over the interior points 1..p-2.
void leaf_tables(hps_group& f, const double* all) {
  const int len = leaf_table_len(f.p);
  std::vector<double> flat((size_t)2 * len * f.nprob);
  for (int b = 0; b < f.nprob; ++b)
    leaf_table_one(f, all, f.prm_h[4 * b + 1], f.prm_h[4 * b + 2], flat.data() + (size_t)2 * len * b);
  upload(f.dLT, flat);
}

// Real line tables of the Dirichlet-block leaf route (leaf_dir.hip), the same for every
// problem of a group (they depend on p and the leaf size only): the interior parts of
// D_xx, D_yy; the A_ib coefficients -D_yy(j, 0), -D_yy(j, p-1), -D_xx(i, 0), -D_xx(i, p-1);
// the N_i coefficients -D_y(0, j), D_y(p-1, j), -D_x(0, i), D_x(p-1, i) (interior j, i);
// and N_bb on the two ends of a line, rows and columns (S, N), then (W, E).
void leaf_rtables(hps_group& f, const double* all) {
  const int p = f.p, m = f.m;
  const double* Dx1 = all;
  const double* Dy1 = all + p * p;
  const double* Dxx = all + 2 * p * p;
  const double* Dyy = all + 3 * p * p;
  auto at = [p](const double* A, int i, int k) { return A[i + p * k]; };
  std::vector<double> one((size_t)leaf_rtable_len(p));
  double* Lx = one.data();
  double* Ly = Lx + m * m;
  double* t = Ly + m * m;
  for (int i = 1; i <= m; ++i)
    for (int k = 1; k <= m; ++k) {
      Lx[(i - 1) + m * (k - 1)] = at(Dxx, i, k);
      Ly[(i - 1) + m * (k - 1)] = at(Dyy, i, k);
    }
  for (int j = 1; j <= m; ++j) {
    t[0 * m + j - 1] = -at(Dyy, j, 0);
    t[1 * m + j - 1] = -at(Dyy, j, p - 1);
    t[2 * m + j - 1] = -at(Dxx, j, 0);
    t[3 * m + j - 1] = -at(Dxx, j, p - 1);
    t[4 * m + j - 1] = -at(Dy1, 0, j);
    t[5 * m + j - 1] = at(Dy1, p - 1, j);
    t[6 * m + j - 1] = -at(Dx1, 0, j);
    t[7 * m + j - 1] = at(Dx1, p - 1, j);
  }
  double* fy = t + 8 * m;
  double* fx = fy + 4;
  fy[0] = -at(Dy1, 0, 0); fy[1] = -at(Dy1, 0, p - 1);
  fy[2] = at(Dy1, p - 1, 0); fy[3] = at(Dy1, p - 1, p - 1);
  fx[0] = -at(Dx1, 0, 0); fx[1] = -at(Dx1, 0, p - 1);
  fx[2] = at(Dx1, p - 1, 0); fx[3] = at(Dx1, p - 1, p - 1);
  std::vector<double> flat;
  flat.reserve(one.size() * f.nprob);
  for (int b = 0; b < f.nprob; ++b) flat.insert(flat.end(), one.begin(), one.end());
  upload(f.dRT, flat);
}

// the line table of one problem (eta = er + i ei) into out (2 * leaf_table_len doubles)
void leaf_table_one(const hps_group& f, const double* all, double er, double ei, double* out) {
  using cd = std::complex<double>;
  const int p = f.p, m = f.m;
  const double* Dx1 = all;
  const double* Dy1 = all + p * p;
  const double* Dxx = all + 2 * p * p;
  const double* Dyy = all + 3 * p * p;
  auto at = [p](const double* A, int i, int k) { return A[i + p * k]; };
  const cd ie(-ei, er);  // i eta
  auto inv2 = [](cd a11, cd a12, cd a21, cd a22, cd* o) {
    const cd det = a11 * a22 - a12 * a21;
    if (!(std::abs(det) > 0.0))
      throw Error(HPS_E_SINGULAR, "leaf: singular end-node impedance block");
    o[0] = a22 / det; o[1] = -a12 / det; o[2] = -a21 / det; o[3] = a11 / det;
  };
  cd B[4], Cm[4];
  inv2(-at(Dy1, 0, 0) + ie, -at(Dy1, 0, p - 1), at(Dy1, p - 1, 0), at(Dy1, p - 1, p - 1) + ie, B);
  inv2(-at(Dx1, 0, 0) + ie, -at(Dx1, 0, p - 1), at(Dx1, p - 1, 0), at(Dx1, p - 1, p - 1) + ie, Cm);
  std::vector<cd> tab((size_t)leaf_table_len(p));
  cd* Gx = tab.data();
  cd* Gy = Gx + m * m;
  cd* sS = Gy + m * m;
  cd* sN = sS + m;
  cd* oW = sN + m;
  cd* oE = oW + m;
  cd* wS = oE + m;
  cd* wN = wS + m;
  cd* wW = wN + m;
  cd* wE = wW + m;
  cd* by = wE + m;
  cd* bx = by + 4;
  for (int l = 1; l <= m; ++l) {
    sS[l - 1] = -B[0] * at(Dy1, 0, l) + B[1] * at(Dy1, p - 1, l);
    sN[l - 1] = -B[2] * at(Dy1, 0, l) + B[3] * at(Dy1, p - 1, l);
    oW[l - 1] = -Cm[0] * at(Dx1, 0, l) + Cm[1] * at(Dx1, p - 1, l);
    oE[l - 1] = -Cm[2] * at(Dx1, 0, l) + Cm[3] * at(Dx1, p - 1, l);
  }
  for (int i = 1; i <= m; ++i)
    for (int k = 1; k <= m; ++k) {
      Gx[(i - 1) + m * (k - 1)] =
          at(Dxx, i, k) - at(Dxx, i, 0) * oW[k - 1] - at(Dxx, i, p - 1) * oE[k - 1];
      Gy[(i - 1) + m * (k - 1)] =
          at(Dyy, i, k) - at(Dyy, i, 0) * sS[k - 1] - at(Dyy, i, p - 1) * sN[k - 1];
    }
  for (int j = 1; j <= m; ++j) {
    wS[j - 1] = -at(Dyy, j, 0) * B[0] - at(Dyy, j, p - 1) * B[2];
    wN[j - 1] = -at(Dyy, j, 0) * B[1] - at(Dyy, j, p - 1) * B[3];
    wW[j - 1] = -at(Dxx, j, 0) * Cm[0] - at(Dxx, j, p - 1) * Cm[2];
    wE[j - 1] = -at(Dxx, j, 0) * Cm[1] - at(Dxx, j, p - 1) * Cm[3];
  }
  for (int q = 0; q < 4; ++q) {
    by[q] = B[q];
    bx[q] = Cm[q];
  }
  for (size_t e = 0; e < tab.size(); ++e) {
    out[2 * e] = tab[e].real();
    out[2 * e + 1] = tab[e].imag();
  }
}

// The shape part of a plan (hps::PlanShape): make_plan's tree and maps, uploaded once
// per device, leaf grid, p and problem count, and shared by every group of that shape
// (a build of a shape seen before skips planning and these uploads).
std::shared_ptr<const PlanShape> plan_for(const hps_group& f) {
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  const PlanKey key = std::make_tuple(dev, f.nx, f.ny, f.p, f.nprob);
  PlanCache& pc = plan_cache();
  {
    std::lock_guard<std::mutex> lk(pc.mu);
    auto it = pc.shapes.find(key);
    if (it != pc.shapes.end()) return it->second;
  }
  hps_group t;  // planned on the side; only the shape is kept
  t.p = f.p; t.m = f.m; t.n = f.n; t.nb = f.nb; t.ni = f.ni;
  t.nx = f.nx; t.ny = f.ny; t.nprob = f.nprob; t.nl1 = f.nl1; t.nleaf = f.nleaf;
  make_plan(t);
  auto sh = std::make_shared<PlanShape>();
  sh->L = t.L;
  sh->geo = std::move(t.geo);
  sh->nbl = std::move(t.nbl);
  sh->lv = std::move(t.lv);
  for (auto& P : sh->lv) {
    std::vector<int> all;
    auto app = [&](const std::vector<int>& v) { all.insert(all.end(), v.begin(), v.end()); };
    app(P.codeA); app(P.codeB); app(P.perm); app(P.i1a); app(P.i3a); app(P.i2b); app(P.i3b);
    app(P.ja); app(P.jb);
    upload(P.dmaps, all);
    sh->bytes += P.dmaps.bytes;
    const int* base = P.dmaps.i();
    P.dcodeA = base; base += P.codeA.size();
    P.dcodeB = base; base += P.codeB.size();
    P.dperm = base; base += P.perm.size();
    P.di1a = base; base += P.i1a.size();
    P.di3a = base; base += P.i3a.size();
    P.di2b = base; base += P.i2b.size();
    P.di3b = base; base += P.i3b.size();
    P.dja = base; base += P.ja.size();
    P.djb = base;
  }
  upload(sh->dleaf_grid, t.leaf_grid);
  std::vector<long> xoff(f.nleaf), uoff(f.nleaf);
  for (int h = 0; h < f.nleaf; ++h) {
    xoff[h] = (long)t.leaf_grid[h] * f.ni;
    uoff[h] = (long)t.leaf_grid[h] * f.n;
  }
  upload(sh->dxoff, xoff);
  upload(sh->duoff, uoff);
  sh->bytes += sh->dleaf_grid.bytes + sh->dxoff.bytes + sh->duoff.bytes;
  std::lock_guard<std::mutex> lk(pc.mu);
  auto ins = pc.shapes.emplace(key, sh);
  if (!ins.second) return ins.first->second;  // another thread planned it meanwhile
  pc.order.push_back(key);
  while (pc.order.size() > kPlanCache) {  // groups hold their shape alive themselves
    pc.shapes.erase(pc.order.front());
    pc.order.pop_front();
  }
  return sh;
}

// Forget the cached plans (a factor keeps its own shape alive).
void drop_plans() {
  PlanCache& pc = plan_cache();
  std::map<PlanKey, std::shared_ptr<const PlanShape>> gone;
  {
    std::lock_guard<std::mutex> lk(pc.mu);
    gone.swap(pc.shapes);
    pc.order.clear();
  }
}  // the unused shapes are freed here, outside the lock

// A group takes its shape's tree and level sizes, and device pointers into its maps.
void attach_plan(hps_group& f, std::shared_ptr<const PlanShape> sh) {
  f.L = sh->L;
  f.geo = sh->geo;
  f.nbl = sh->nbl;
  f.lv.clear();
  f.lv.resize(sh->lv.size());
  for (size_t l = 0; l < sh->lv.size(); ++l) {
    const LevelPlan& S = sh->lv[l];
    LevelPlan& P = f.lv[l];
    P.nbox = S.nbox; P.wx = S.wx; P.wy = S.wy; P.split_x = S.split_x;
    P.nbc = S.nbc; P.nbp = S.nbp; P.n1 = S.n1; P.n2 = S.n2; P.n3 = S.n3;
    P.dcodeA = S.dcodeA; P.dcodeB = S.dcodeB; P.dperm = S.dperm;
    P.di1a = S.di1a; P.di3a = S.di3a; P.di2b = S.di2b; P.di3b = S.di3b;
    P.dja = S.dja; P.djb = S.djb;
  }
  f.pleaf_grid = sh->dleaf_grid.i();
  f.pxoff = sh->dxoff.l();
  f.puoff = sh->duoff.l();
  f.shape = std::move(sh);
}

// The per-group tables: the scaled differentiation matrices (they depend on the leaf
// size), the line tables of the leaf stage and the problems' kappa and eta.
void upload_tables(hps_group& f) {
  std::vector<double> x, D;
  cheb(f.p, x, D);
  const int p = f.p;
  const double hx = (f.x1 - f.x0) / f.nx, hy = (f.y1 - f.y0) / f.ny;
  std::vector<double> all(4 * (size_t)p * p, 0.0);
  for (int e = 0; e < p * p; ++e) {
    all[e] = D[e] * 2.0 / hx;
    all[p * p + e] = D[e] * 2.0 / hy;
  }
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double sx = 0, sy = 0;
      for (int k = 0; k < p; ++k) {
        sx += all[i + p * k] * all[k + p * j];
        sy += all[p * p + i + p * k] * all[p * p + k + p * j];
      }
      all[2 * p * p + i + p * j] = sx;
      all[3 * p * p + i + p * j] = sy;
    }
  upload(f.dD, all);
  leaf_tables(f, all.data());
  leaf_rtables(f, all.data());
  upload(f.dprm, f.prm_h);
}

MergeLevelDesc level_desc(const hps_group& f, const LevelPlan& P) {
  MergeLevelDesc d;
  d.nbox = P.nbox; d.nbc = P.nbc; d.n1 = P.n1; d.n2 = P.n2; d.n3 = P.n3; d.nbp = P.nbp;
  d.codeA = P.dcodeA; d.codeB = P.dcodeB; d.perm = P.dperm;
  d.i1a = P.di1a; d.i3a = P.di3a; d.i2b = P.di2b; d.i3b = P.di3b;
  return d;
}

void check_info(const std::vector<int>& h, long off, long cnt, const char* what) {
  for (long i = 0; i < cnt; ++i)
    if (h[off + i])
      throw Error(HPS_E_SINGULAR, std::string(what) + ": zero pivot at step " +
                                      std::to_string(h[off + i] - 1) + " of matrix " +
                                      std::to_string(i));
}

// ------------------------------------------------------------------ build memory
// One arena holds every stored operator ([Psi | Y] of the leaves, then per level
// W^{-1}, R33a, R33b, R13a, R23b, Phi^a, Phi^b); the ItI operators R ping-pong between
// two buffers (level l in buffer l % 2), or get one buffer per level when every R is
// kept; one scratch arena serves the leaf stage and then each merge level in turn.
struct BuildScratch {
  DevBuf buf;
  View R31a, T, work;      // merge level (sized for the largest level)
  View w64;                // complex128 copy of a complex64 level's W (inverted in FP64)
  View info;               // [2 * nleaf] leaf infos, then one int per merge
  std::vector<long> info_off;  // per level offset into info
};

// bytes of one complex entry of level l's operators and R (the leaves' R is complex128)
size_t cbytes(const hps_group& f, int l) { return (l < f.L && f.lv[l].c64) ? 8 : 16; }

// leaves per launch of the leaf stage (bounds its scratch); in mixed precision the
// scratch also holds the chunk's complex128 [Psi | Y] (1 MB per leaf at p = 16), so the
// chunks are smaller
constexpr long kLeafChunk = 4096;
constexpr long kLeafChunkMixed = 1024;
long leaf_chunk(const hps_group& f) {
  return std::min<long>(f.nleaf, f.mixed ? kLeafChunkMixed : kLeafChunk);
}

bool level_forms_R(const hps_group& f, int l) {
  return l == f.L || l > 0 || f.opts.store_root_R;
}

size_t level_R_bytes(const hps_group& f, int l) {
  if (l == f.L) return (size_t)f.nleaf * f.nb * f.nb * 16;
  const LevelPlan& P = f.lv[l];
  return (size_t)P.nbox * P.nbp * P.nbp * cbytes(f, l);
}

// Layout of the operator arena (base = nullptr only sizes it); returns its bytes.
size_t arena_layout(hps_group& f, char* base) {
  const long nl = f.nleaf, n = f.n;
  Carver c;
  c.base = base;
  if (f.mixed) f.BI32 = c.take((size_t)nl * n * n * 8);
  else f.BI = c.take((size_t)nl * n * n * 16);
  for (auto& P : f.lv) {
    const size_t nbox = P.nbox, n1 = P.n1, n2 = P.n2, n3 = P.n3, nbp = P.nbp;
    const size_t e = P.c64 ? 8 : 16;
    P.Winv = c.take(nbox * n3 * n3 * e);
    P.R33a = c.take(nbox * n3 * n3 * e);
    P.R33b = c.take(nbox * n3 * n3 * e);
    P.R13a = c.take(nbox * n1 * n3 * e);
    P.R23b = c.take(nbox * n2 * n3 * e);
    P.PhiA = c.take(nbox * n3 * nbp * e);
    P.PhiB = c.take(nbox * n3 * nbp * e);
  }
  return c.used;
}

// Leaf-stage scratch of one chunk of leaves (byte offsets): the impedance route's
// inverse copies (mg), in mixed precision the chunk's complex128 [Psi | Y] (bi), then the
// Dirichlet route's X (n_i x n_b), Z (n_b x n_i) and real A^{-1} (n_i x n_i) per leaf.  Both routes may run on
// one chunk (problems of one group can take different routes), so both are laid out.
struct LeafScratch {
  size_t mg = 0, bi = 0, x = 0, z = 0, ai = 0, total = 0;
};
LeafScratch leaf_scratch(const hps_group& f) {
  auto r256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t lch = (size_t)leaf_chunk(f), n = f.n, ni = f.ni, nb = f.nb;
  LeafScratch L;
  L.mg = 0;
  L.bi = r256(leaf_scratch_bytes(f.p, (long)lch));
  L.x = L.bi + (f.mixed ? r256(lch * n * n * 16) : 0);
  L.z = L.x + r256(lch * ni * nb * 8);
  L.ai = L.z + r256(lch * nb * ni * 8);
  L.total = L.ai + r256(lch * ni * ni * 8);
  return L;
}

// Bytes of the build scratch (leaf chunks and merge levels; the info words follow).
size_t scratch_bytes(const hps_group& f) {
  size_t level_bytes = leaf_scratch(f).total;
  for (auto& P : f.lv) {
    Carver c;
    const size_t e = P.c64 ? 8 : 16;
    c.take((size_t)P.nbox * P.n3 * P.n1 * e);
    c.take((size_t)P.nbox * P.n3 * P.nbp * e);
    if (P.inv64) c.take((size_t)P.nbox * P.n3 * P.n3 * 16);
    c.take(zinv_workspace_bytes(P.n3, P.nbox, P.c64 && !P.inv64));
    level_bytes = std::max(level_bytes, c.used);
  }
  return (level_bytes + 255) & ~size_t(255);
}

// Device bytes of a planned group (make_plan done, nothing allocated): the peak during
// the build and what stays resident afterwards, from the same sizes the build allocates.
void estimate_bytes(hps_group& f, size_t* peak, size_t* resident) {
  const size_t arena = arena_layout(f, nullptr);
  size_t rb[2] = {0, 0}, kept = 0, keep_all = 0;
  for (int l = 0; l <= f.L; ++l)
    if (level_forms_R(f, l)) {
      rb[l % 2] = std::max(rb[l % 2], level_R_bytes(f, l));
      keep_all += level_R_bytes(f, l);
    }
  if (f.opts.keep_all_R) kept = keep_all;
  else if (level_forms_R(f, 0)) kept = rb[0];
  const size_t rbufs = f.opts.keep_all_R ? keep_all : rb[0] + rb[1];
  // leaf maps (int grid index, long x/u offsets), c, the four p x p differentiation
  // matrices, per-problem parameters and line tables, then the level maps
  size_t small = (size_t)f.nleaf * (4 + 16) + (size_t)f.nleaf * f.ni * 8 + (size_t)32 * f.p * f.p +
                 (size_t)32 * f.nprob + (size_t)f.nprob * leaf_table_len(f.p) * 16 +
                 (size_t)f.nprob * (leaf_rtable_len(f.p) * 8 + sizeof(int) + sizeof(double));
  for (auto& P : f.lv)
    small += 4 * (P.codeA.size() + P.codeB.size() + P.perm.size() + P.i1a.size() +
                  P.i3a.size() + P.i2b.size() + P.i3b.size() + P.ja.size() + P.jb.size());
  const size_t ninfo = 4 * (2 * (size_t)f.nleaf + (size_t)f.nleaf);
  *resident = arena + kept + small;
  *peak = arena + rbufs + small + scratch_bytes(f) + ninfo;
}

void plan_memory(hps_group& f, BuildScratch& sc) {
  const long nl = f.nleaf;
  f.ops.alloc(arena_layout(f, nullptr));
  arena_layout(f, static_cast<char*>(f.ops.p));
  f.R.assign(f.L + 1, View());
  f.R_valid.assign(f.L + 1, 0);
  if (f.opts.keep_all_R) {
    f.rkeep.clear();
    f.rkeep.resize(f.L + 1);
    for (int l = 0; l <= f.L; ++l)
      if (level_forms_R(f, l)) {
        f.rkeep[l].alloc(level_R_bytes(f, l));
        f.R[l].p = f.rkeep[l].p;
        f.R[l].bytes = f.rkeep[l].bytes;
      }
  } else {
    size_t need[2] = {0, 0};
    for (int l = 0; l <= f.L; ++l)
      if (level_forms_R(f, l)) need[l % 2] = std::max(need[l % 2], level_R_bytes(f, l));
    for (int b = 0; b < 2; ++b) f.rbuf[b].alloc(need[b]);
    for (int l = 0; l <= f.L; ++l)
      if (level_forms_R(f, l)) {
        f.R[l].p = f.rbuf[l % 2].p;
        f.R[l].bytes = level_R_bytes(f, l);
      }
  }
  // scratch: the leaf stage (per chunk of leaves: the inverse's copies and, in mixed
  // precision, the complex128 [Psi | Y] before its complex64 copy) and the merge levels
  // share the same bytes; infos follow
  long ninfo = 2 * nl;
  sc.info_off.assign(f.L, 0);
  for (int l = 0; l < f.L; ++l) {
    sc.info_off[l] = ninfo;
    ninfo += f.lv[l].nbox;
  }
  const size_t shared = scratch_bytes(f);
  sc.buf.alloc(shared + (size_t)ninfo * sizeof(int) + 256);
  char* base = static_cast<char*>(sc.buf.p);
  sc.info.p = base + shared;
  sc.info.bytes = (size_t)ninfo * sizeof(int);
}

void level_scratch(const LevelPlan& P, BuildScratch& sc) {
  Carver c;
  c.base = static_cast<char*>(sc.buf.p);
  const size_t e = P.c64 ? 8 : 16;
  sc.R31a = c.take((size_t)P.nbox * P.n3 * P.n1 * e);
  sc.T = c.take((size_t)P.nbox * P.n3 * P.nbp * e);
  sc.w64 = P.inv64 ? c.take((size_t)P.nbox * P.n3 * P.n3 * 16) : View();
  sc.work = c.take(zinv_workspace_bytes(P.n3, P.nbox, P.c64 && !P.inv64));
}

// ------------------------------------------------------------------ build
// Route of each problem's leaves.  The Dirichlet-block route (leaf_dir.hip: real A^{-1},
// a quarter of the complex inversion) needs the interior block A = -Lap_h - kappa^2 c to
// be safely invertible: -Lap - kappa^2 c is coercive on a leaf when kappa^2 c stays below
// the smallest eigenvalue pi^2 (1/h_x^2 + 1/h_y^2) of the leaf's Dirichlet Laplacian, and
// the route is taken when kappa^2 max(c) is at most half of it.  Otherwise (leaves of a
// wavelength or more, where kappa^2 c can meet a Dirichlet eigenvalue) the impedance
// route eliminates through the impedance rows, which stay well posed for Re eta != 0.
// opts.leaf_route = 1 takes the impedance route for every problem.
void choose_routes(hps_group& f, const double* c) {
  f.route_h.assign(f.nprob, 0);
  if (!f.dcmax.p) f.dcmax.alloc((size_t)f.nprob * sizeof(double));
  if (f.opts.leaf_route != 1) {
    leaf_cmax(c, f.nprob, (long)f.nl1 * f.ni, f.dcmax.d(), f.stream);
    std::vector<unsigned long long> key(f.nprob);
    HPS_HIP(hipMemcpyAsync(key.data(), f.dcmax.p, key.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, f.stream));
    HPS_HIP(hipStreamSynchronize(f.stream));
    std::vector<double> cm(f.nprob);
    for (int b = 0; b < f.nprob; ++b) cm[b] = leaf_cmax_value(key[b]);
    const double hx = (f.x1 - f.x0) / f.nx, hy = (f.y1 - f.y0) / f.ny;
    const double lam1 = M_PI * M_PI * (1.0 / (hx * hx) + 1.0 / (hy * hy));
    for (int b = 0; b < f.nprob; ++b) {
      const double k = f.prm_h[4 * b];
      f.route_h[b] = (std::isfinite(cm[b]) && k * k * cm[b] <= 0.5 * lam1) ? 1 : 0;
    }
  }
  upload(f.droute, f.route_h);
}

void build_leaves(hps_group& f, const double* c, BuildScratch& sc) {
  hipStream_t st = f.stream;
  const long nl = f.nleaf;
  const long n = f.n, nb = f.nb, ni = f.ni;
  LeafDesc d;
  d.p = f.p; d.nleaf = f.nleaf; d.nl1 = f.nl1; d.prm = f.dprm.d();
  d.c = c; d.leaf_grid = f.pleaf_grid; d.tab = f.dLT.d();
  d.R = f.R[f.L].d(); d.info = sc.info.i();
  d.route = f.droute.i(); d.rtab = f.dRT.d();
  // scratch per chunk (leaf_scratch): the impedance route's per-leaf copies, (mixed
  // precision) the complex128 [Psi | Y] of the chunk, rounded into the complex64 arena
  // at the end, and the Dirichlet route's X and Z
  char* scr = static_cast<char*>(sc.buf.p);
  const LeafScratch LS = leaf_scratch(f);
  const long lch = leaf_chunk(f);
  const size_t mg_bytes = leaf_scratch_bytes(f.p, lch);
  double* bi64 = f.mixed ? reinterpret_cast<double*>(scr + LS.bi) : nullptr;
  Profiler& pr = f.build_prof;
  for (long h0 = 0; h0 < nl; h0 += lch) {
    const int cnt = (int)std::min<long>(lch, nl - h0);
    LeafDesc dc = d;
    dc.nleaf = cnt;
    dc.h0 = h0;
    dc.leaf_grid = d.leaf_grid + h0;
    dc.BI = f.mixed ? bi64 : f.BI.d() + 2 * h0 * n * n;
    dc.R = d.R + 2 * h0 * nb * nb;
    dc.info = d.info + h0;
    dc.Mg = mg_bytes ? reinterpret_cast<double*>(scr) : nullptr;
    dc.X = reinterpret_cast<double*>(scr + LS.x);
    dc.Z = reinterpret_cast<double*>(scr + LS.z);
    dc.Ai = reinterpret_cast<double*>(scr + LS.ai);
    long nR = 0;  // leaves of the chunk on the Dirichlet route
    for (long hh = h0; hh < h0 + cnt; ++hh) nR += f.route_h[hh / f.nl1];
    const long nC = cnt - nR;
    const double r_ = nR, c_ = nC;
    if (nR > 0) {
      {
        // A^{-1}: real Gauss-Jordan, 2 n_i^3 flops
        Stage s(pr, "leaf_ainv", r_ * 2.0 * ni * ni * ni, r_ * (ni * 8.0 + ni * ni * 8.0));
        leaf_dirichlet_inverse(dc, st);
      }
      {
        // X = A^{-1} A_ib and Z = N_i A^{-1} (2 n_i^2 n_b each as dense products),
        // S = F_bb - N_i X (2 n_b^2 n_i)
        Stage s(pr, "leaf_xz", r_ * (4.0 * ni * ni * nb + 2.0 * nb * nb * ni),
                r_ * (ni * ni * 8.0 + 2.0 * ni * nb * 8.0 + nb * nb * 16.0));
        leaf_dirichlet_xz(dc, st);
      }
      {
        // S^{-1} (8 n_b^3), R = I - 2 i eta S^{-1}
        Stage s(pr, "leaf_sbinv", r_ * 8.0 * nb * nb * nb, r_ * 3.0 * nb * nb * 16.0);
        zinv((int)nb, cnt, dc.BI, n, n * n, dc.BI, n, n * n, d.info + nl + h0, nullptr, st,
             false);
        leaf_dirichlet_R(dc, st);
      }
      // Psi_i = -X Psi_b, Y_b = -Psi_b Z, Y_i = A^{-1} - X Y_b   (4 n_i n_b^2, 4 n_b^2 n_i,
      // 4 n_i^2 n_b flops: real times complex)
      GemmDesc g;
      g.M = ni; g.N = nb; g.K = nb; g.batch = cnt;
      g.A = dc.X; g.lda = ni; g.sA = ni * nb; g.a_real = true;
      g.B = dc.BI; g.ldb = n; g.sB = n * n;
      g.C = dc.BI + 2 * nb; g.ldc = n; g.sC = n * n;
      g.alpha = -1.0; g.beta = 0.0;
      timed_gemm(pr, "leaf_gemm", g, st, f.opts.autotune != 0);
      g = GemmDesc();
      g.M = nb; g.N = ni; g.K = nb; g.batch = cnt;
      g.A = dc.BI; g.lda = n; g.sA = n * n;
      g.B = dc.Z; g.ldb = nb; g.sB = nb * ni; g.b_real = true;
      g.C = dc.BI + 2 * n * nb; g.ldc = n; g.sC = n * n;
      g.alpha = -1.0; g.beta = 0.0;
      timed_gemm(pr, "leaf_gemm", g, st, f.opts.autotune != 0);
      g = GemmDesc();
      g.M = ni; g.N = ni; g.K = nb; g.batch = cnt;
      g.A = dc.X; g.lda = ni; g.sA = ni * nb; g.a_real = true;
      g.B = dc.BI + 2 * n * nb; g.ldb = n; g.sB = n * n;
      g.C = dc.BI + 2 * (n * nb + nb); g.ldc = n; g.sC = n * n;
      g.alpha = -1.0; g.beta = 0.0;
      g.C0r = dc.Ai; g.ld0 = ni; g.s0 = ni * ni;  // + A^{-1} (real)
      timed_gemm(pr, "leaf_gemm", g, st, f.opts.autotune != 0);
      if (f.mixed) {
        Stage s(pr, "leaf_round", 0.0, cnt * (double)n * n * 24.0);
        to_c64(dc.BI, reinterpret_cast<float*>(f.BI32.p) + 2 * h0 * n * n, 2L * cnt * n * n, st);
      }
    }
    if (nC > 0) {
      // mixed precision: the Psi / boundary-row kernel writes the complex64 [Psi | Y]
      dc.BI32 = f.mixed ? reinterpret_cast<float*>(f.BI32.p) + 2 * h0 * n * n : nullptr;
      {
        // S_i^{-1}: complex Gauss-Jordan, n_i^3 complex multiply-adds
        Stage s(pr, "leaf_sinv", c_ * 8.0 * ni * ni * ni, c_ * (ni * 8.0 + ni * ni * 16.0));
        leaf_interior_inverse(dc, st);
      }
      {
        // Y_i read once; Psi_i and the boundary rows written (complex64 in mixed precision,
        // with the interior Y rows), R written
        const double out = f.mixed ? n * n * 8.0 : (ni * nb + nb * n) * 16.0;
        Stage s(pr, "leaf_psi_bnd", c_ * (32.0 * ni * ni + 8.0 * nb * n * f.m),
                c_ * (ni * ni * 16.0 + out + nb * nb * 16.0));
        leaf_psi_and_boundary(dc, st);
      }
    }
  }
  f.R_valid[f.L] = 1;
}

void build_level(hps_group& f, int l, BuildScratch& sc) {
  hipStream_t st = f.stream;
  LevelPlan& P = f.lv[l];
  const long nbox = P.nbox, n1 = P.n1, n2 = P.n2, n3 = P.n3, nbp = P.nbp;
  const bool form_R = level_forms_R(f, l);
  level_scratch(P, sc);
  int* info = sc.info.i() + sc.info_off[l];

  MergeLevelDesc d = level_desc(f, P);
  d.c64 = P.c64;
  d.child_c64 = (l + 1 < f.L) && f.lv[l + 1].c64;
  const double ez = P.c64 ? 0.5 : 1.0;  // doubles per complex entry / 2
  d.Rc = f.R[l + 1].d();
  d.Rp = form_R ? f.R[l].d() : nullptr;
  d.R33a = P.R33a.d(); d.R33b = P.R33b.d(); d.R13a = P.R13a.d(); d.R23b = P.R23b.d();
  d.R31a = sc.R31a.d(); d.T = sc.T.d(); d.PhiB = P.PhiB.d();
  // profile = 2 names the merge groups per level (for tuning); 1 aggregates them
  const bool per_level = f.opts.profile == 2;
  const std::string sfx = per_level ? "@" + std::to_string(l) : std::string();
  const std::string gname_s = "merge_gemm" + sfx, ename = "merge_extract" + sfx,
                    iname = "merge_inv" + sfx;
  const char* gname = gname_s.c_str();
  {
    const double nbc = P.nbc;
    Stage s(f.build_prof, ename.c_str(), 0.0,
            nbox * (2.0 * nbc * nbc * 16 + 2.0 * n3 * nbp * 16 + n3 * n3 * 16.0));
    fill_zero(d.PhiB, (long)(2 * ez * nbox * n3 * nbp), st);
    merge_extract(d, st);
    // W = I - R33b R33a   (into the Winv buffer, inverted in place below)
    fill_identity(P.Winv.d(), (int)n3, n3 * n3, (int)nbox, st, P.c64);
  }
  GemmDesc g;
  g.M = n3; g.N = n3; g.K = n3; g.batch = nbox;
  g.A = P.R33b.d(); g.lda = n3; g.sA = n3 * n3;
  g.B = P.R33a.d(); g.ldb = n3; g.sB = n3 * n3;
  g.C = P.Winv.d(); g.ldc = n3; g.sC = n3 * n3;
  g.alpha = -1.0; g.beta = 1.0;
  g.c64 = P.c64;
  timed_gemm(f.build_prof, gname, g, st, f.opts.autotune != 0);
  // T[:, perm(I1)] = R33b R31a  (T[:, perm(I2)] = -R32b was written by the extract)
  g = GemmDesc();
  g.M = n3; g.N = n1; g.K = n3; g.batch = nbox;
  g.A = P.R33b.d(); g.lda = n3; g.sA = n3 * n3;
  g.B = sc.R31a.d(); g.ldb = n3; g.sB = n3 * n1;
  g.C = sc.T.d(); g.ldc = n3; g.sC = n3 * nbp; g.ccol = P.dperm;
  g.alpha = 1.0; g.beta = 0.0;
  g.c64 = P.c64;
  timed_gemm(f.build_prof, gname, g, st, f.opts.autotune != 0);
  // W^{-1}
  {
    Stage s(f.build_prof, iname.c_str(), nbox * 8.0 * n3 * n3 * n3, nbox * 2.0 * n3 * n3 * 16);
    if (P.inv64) {
      // complex64 level, W inverted in complex128 (the pivoting of large interface
      // matrices stays in double precision); the inverse is rounded back for storage
      const long cnt = 2L * nbox * n3 * n3;
      to_c128(reinterpret_cast<const float*>(P.Winv.p), sc.w64.d(), cnt, st);
      zinv((int)n3, (int)nbox, sc.w64.d(), n3, n3 * n3, sc.w64.d(), n3, n3 * n3, info,
           sc.work.p, st, false, f.full_pivoting);
      to_c64(sc.w64.d(), reinterpret_cast<float*>(P.Winv.p), cnt, st);
    } else {
      zinv((int)n3, (int)nbox, P.Winv.d(), n3, n3 * n3, P.Winv.d(), n3, n3 * n3, info,
           sc.work.p, st, P.c64, f.full_pivoting);
    }
  }
  // Phi^a = W^{-1} T   (eq. (talpha))
  g = GemmDesc();
  g.M = n3; g.N = nbp; g.K = n3; g.batch = nbox;
  g.A = P.Winv.d(); g.lda = n3; g.sA = n3 * n3;
  g.B = sc.T.d(); g.ldb = n3; g.sB = n3 * nbp;
  g.C = P.PhiA.d(); g.ldc = n3; g.sC = n3 * nbp;
  g.alpha = 1.0; g.beta = 0.0;
  g.c64 = P.c64;
  timed_gemm(f.build_prof, gname, g, st, f.opts.autotune != 0);
  // Phi^b = [-R31a, 0] - R33a Phi^a   (eq. (tbeta), short form)
  g = GemmDesc();
  g.M = n3; g.N = nbp; g.K = n3; g.batch = nbox;
  g.A = P.R33a.d(); g.lda = n3; g.sA = n3 * n3;
  g.B = P.PhiA.d(); g.ldb = n3; g.sB = n3 * nbp;
  g.C = P.PhiB.d(); g.ldc = n3; g.sC = n3 * nbp;
  g.alpha = -1.0; g.beta = 1.0;
  g.c64 = P.c64;
  timed_gemm(f.build_prof, gname, g, st, f.opts.autotune != 0);
  if (form_R) {
    // R^tau = blockdiag(R11a, R22b) + blockdiag(R13a, R23b) [Phi^a; Phi^b]   (eq. (out)):
    // the two products write every row (I1, then I2) and column of R^tau, then the
    // children's diagonal blocks are added
    g = GemmDesc();
    g.M = n1; g.N = nbp; g.K = n3; g.batch = nbox;
    g.A = P.R13a.d(); g.lda = n1; g.sA = n1 * n3;
    g.B = P.PhiA.d(); g.ldb = n3; g.sB = n3 * nbp;
    g.C = f.R[l].d(); g.ldc = nbp; g.sC = nbp * nbp; g.crow = P.dperm;
    g.alpha = 1.0; g.beta = 0.0;
    g.c64 = P.c64;
    timed_gemm(f.build_prof, gname, g, st, f.opts.autotune != 0);
    g.M = n2;
    g.A = P.R23b.d(); g.lda = n2; g.sA = n2 * n3;
    g.B = P.PhiB.d();
    g.crow = P.dperm + n1;
    g.c64 = P.c64;
    timed_gemm(f.build_prof, gname, g, st, f.opts.autotune != 0);
    {
      Stage s(f.build_prof, ename.c_str(), 0.0,
              nbox * ((double)n1 * n1 + (double)n2 * n2) * (16.0 + 2.0 * 16.0 * ez));
      merge_add_diag(d, st);
    }
    f.R_valid[l] = 1;
  }
  // children's R: overwritten two levels up (ping-pong) unless every R is kept
  if (!f.opts.keep_all_R) f.R_valid[l + 1] = 0;
}

void build_all(hps_group& f, const double* c) {
  BuildScratch sc;
  std::vector<int> h;
  for (int attempt = 0;; ++attempt) {
    plan_memory(f, sc);
    fill_zero_int(sc.info.i(), (long)(sc.info.bytes / sizeof(int)), f.stream);
    choose_routes(f, c);
    build_leaves(f, c, sc);
    for (int l = f.L - 1; l >= 0; --l) build_level(f, l, sc);
    // one synchronization for the whole build, then the pivot checks
    HPS_HIP(hipStreamSynchronize(f.stream));
    h.assign(sc.info.bytes / sizeof(int), 0);
    HPS_HIP(hipMemcpy(h.data(), sc.info.p, sc.info.bytes, hipMemcpyDeviceToHost));
    // An elimination without row exchanges that broke down is not an error of the
    // problem: a leaf of the Dirichlet-block route (a zero pivot block or growth past
    // the check) repeats the build with every leaf eliminated through its impedance rows,
    // an interface matrix whose diagonal block was singular repeats it with pivoting over
    // whole columns.  A failure of the fully pivoted forms is reported.
    bool dir_failed = false, w_failed = false;
    for (long i = 0; i < f.nleaf && !dir_failed; ++i)
      dir_failed = (h[i] || h[f.nleaf + i]) && f.route_h[i / f.nl1];
    for (int l = 0; l < f.L && !w_failed; ++l)
      for (long i = 0; i < f.lv[l].nbox && !w_failed; ++i)
        w_failed = h[sc.info_off[l] + i] != 0 && f.lv[l].n3 > 64 && !f.full_pivoting;
    if ((!dir_failed && !w_failed) || attempt > 0) break;
    if (dir_failed) f.opts.leaf_route = 1;
    if (w_failed) f.full_pivoting = true;
    f.build_prof.reset(f.opts.profile != 0, f.stream);
  }
  check_info(h, 0, f.nleaf, "leaf interior block");
  check_info(h, f.nleaf, f.nleaf, "leaf boundary Schur complement");
  for (int l = 0; l < f.L; ++l) check_info(h, sc.info_off[l], f.lv[l].nbox, "interface matrix W");
  // release the ItI buffer that no longer holds a kept operator
  if (!f.opts.keep_all_R) {
    for (int b = 0; b < 2; ++b) {
      bool holds = false;
      for (int l = 0; l <= f.L; ++l)
        if (f.R_valid[l] && l % 2 == b) holds = true;
      if (!holds) f.rbuf[b].release();
    }
  }
}

// ------------------------------------------------------------------ solve
// Workspace of one solve call: a single stream-ordered allocation carved into the
// per-level vectors.  A dry pass over the same code sizes it (no launches).
struct Arena {
  bool dry = true;
  hipStream_t st = nullptr;
  char* base = nullptr;
  size_t used = 0, split_need = 0, peak = 0, cap = 0;
  void* split = nullptr;
  void* block = nullptr;
  // caller-provided memory of fixed_cap bytes (the allocation-free solve): allocate()
  // carves the workspace from it and allocates nothing
  char* fixed = nullptr;
  size_t fixed_cap = 0;
  double* get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    size_t off = used;
    used += bytes;
    peak = std::max(peak, used);
    // a pass that needs more than the sizing pass measured is a planning error
    if (!dry && used > cap) throw Error(HPS_E_INVALID, "solve workspace exceeded its plan");
    // in the dry pass the pointer is a placeholder that is never dereferenced
    return reinterpret_cast<double*>((dry ? reinterpret_cast<char*>(4096) : base) + off);
  }
  void skinny(Profiler& pr, const char* name, SkinnyDesc k) {
    if (dry) {
      split_need = std::max(split_need, skinny_work_bytes(k));
      return;
    }
    k.work = split;
    timed_skinny(pr, name, k, st);
  }
  void allocate() {
    used = std::max(used, peak);
    cap = used;
    size_t total = used + split_need + 256;
    if (fixed) {
      if (total > fixed_cap)
        throw Error(HPS_E_INVALID, "solve workspace of " + std::to_string(total) +
                                       " bytes exceeds the allocation-free scratch of " +
                                       std::to_string(fixed_cap) + " bytes");
      base = fixed;
    } else {
      block = ws_alloc(total, st);
      base = static_cast<char*>(block);
    }
    split = base + ((used + 255) & ~size_t(255));
    used = 0;
    dry = false;
  }
  ~Arena() {
    if (block) ws_free(block, st);
  }
};

// Solve sweeps of Algorithm 2 for problems [pb, pb + np) of the group, nrhs right-hand
// sides each.  Layouts (complex128): s [nrhs][np nl1 ni], jmp [nrhs][np nl1 nb],
// t [np][nrhs][nt], u [nrhs][np nl1 n].
// Problems of several factors of one shape, solved together: their right-hand sides are
// laid out as for one group of np problems (problem q's leaves [q nl1, (q+1) nl1)), each
// operator launch takes the factors' operator bases from tables, and the leaf maps come
// from the plan of an np-problem group.
struct Across {
  static constexpr int kMax = SkinnyDesc::kMaxTab;
  int np = 0;
  std::shared_ptr<const PlanShape> sh;  // leaf maps of an np-problem group
  int nrq[kMax] = {};                   // right-hand sides of each problem
  const double* leaf[kMax] = {};        // [Psi | Y] of the problem's first leaf
  PrmTab prm;                           // kappa, Re eta, Im eta of each problem
  struct Level {
    const double *R33b[kMax], *Winv[kMax], *R33a[kMax], *R13a[kMax], *R23b[kMax],
        *PhiA[kMax], *PhiB[kMax];
  };
  std::vector<Level> lv;
  // route launch k through the tables: entry b of factor b / per, operator tab (and tab2)
  void put(SkinnyDesc& k, int per, const double* const* tab, const double* const* tab2 = nullptr,
           long add = 0) const {
    k.aper = per;
    for (int q = 0; q < np; ++q) {
      k.Atab[q] = tab[q] + add;
      if (tab2) k.Atab2[q] = tab2[q] + add;
      k.nrq[q] = nrq[q];
    }
  }
};

void solve_pass(hps_group& f, int pb, int np, int nrhs, const double* s, const double* t,
                const double* jmp, double* u, Arena& ws, const Across* ax = nullptr) {
  hipStream_t st = ws.st;
  Profiler& pr = f.solve_prof;
  pr.reset(!ws.dry && !ws.fixed && f.opts.profile != 0, st);
  const char* nm = "solve_leaf_up";
  const long nl = (long)np * f.nl1, n = f.n, nb = f.nb, ni = f.ni;
  const long h0 = (long)pb * f.nl1;  // first leaf of the range
  const int le = f.mixed ? 1 : 2;    // doubles per complex entry of the leaf operators
  const double* leafops = ax ? nullptr : (f.mixed ? f.BI32.d() : f.BI.d()) + le * h0 * n * n;
  const long* xoff = ax ? ax->sh->dxoff.l() : f.pxoff + h0;
  const long* uoff = ax ? ax->sh->duoff.l() : f.puoff + h0;
  const long lbase = ax ? 0 : h0;  // leaf index the offset tables start from
  // the upward pass runs for a body load or for right-hand sides on shared-edge rows
  const bool up = (s != nullptr) || (jmp != nullptr);
  std::vector<double*> h(f.L + 1, nullptr), tt(f.L + 1, nullptr), tta(f.L, nullptr),
      ttb(f.L, nullptr);
  double* ut = nullptr;
  if (up) {
    ut = ws.get((size_t)nl * n * nrhs * 16);
    h[f.L] = ws.get((size_t)nl * nb * nrhs * 16);
    if (s) {
      // leaf: u~ = Y s   (Algorithm 2 step (3))
      SkinnyDesc k;
      k.M = n; k.K = ni; k.nrhs = nrhs; k.batch = (int)nl;
      k.a_c64 = f.mixed;
      if (ax) ax->put(k, f.nl1, ax->leaf, nullptr, le * n * nb);
      else k.A = leafops + le * n * nb;
      k.lda = n; k.sA = n * n;
      k.X = s; k.ldx = nl * ni; k.xoff = xoff; k.xbase = lbase * ni;
      k.C = ut; k.ldc = n; k.sC = n * nrhs;
      ws.skinny(pr, nm, k);
      Stage sg(pr, "solve_gather", 0.0, nl * nb * nrhs * 32.0);
      if (!ws.dry)
        leaf_h_from_u((int)nl, f.n, f.nb, nrhs, f.dprm.d() + 4 * pb, f.nl1, ut, h[f.L], st,
                      ax ? &ax->prm : nullptr);
    } else if (!ws.dry) {
      fill_zero(ut, 2 * nl * n * nrhs, st);
      fill_zero(h[f.L], 2 * nl * nb * nrhs, st);
    }
    // merges, bottom-up   (steps (5)-(7))
    nm = "solve_merge_up";
    for (int l = f.L - 1; l >= 0; --l) {
      LevelPlan& P = f.lv[l];
      MergeLevelDesc d = level_desc(f, P);
      const long nbox = (long)np << l, box0 = (long)pb << l;
      d.nbox = (int)nbox;
      const long n1 = P.n1, n2 = P.n2, n3 = P.n3, nbp = P.nbp;
      const int e = P.c64 ? 1 : 2;
      auto op = [&](const View& v, long per) { return v.d() + box0 * per * e; };
      const Across::Level* tl = ax ? &ax->lv[l] : nullptr;
      const int per = 1 << l;  // boxes of one problem on the level
      if (l > 0 && up_fused_fits((int)n1, (int)n2, (int)n3, (int)nbp)) {
        // a short interface: gather, the three interface products and h^tau of each box
        // in one launch, the box's vectors in LDS
        tta[l] = ws.get((size_t)nbox * n3 * nrhs * 16);
        ttb[l] = ws.get((size_t)nbox * n3 * nrhs * 16);
        h[l] = ws.get((size_t)nbox * nbp * nrhs * 16);
        UpLevelDesc u;
        u.nbox = (int)nbox; u.nbc = P.nbc; u.n1 = (int)n1; u.n2 = (int)n2; u.n3 = (int)n3;
        u.nbp = (int)nbp; u.nrhs = nrhs;
        u.perm = P.dperm; u.i1a = P.di1a; u.i3a = P.di3a; u.i2b = P.di2b; u.i3b = P.di3b;
        u.hc = h[l + 1]; u.hp = h[l]; u.tta = tta[l]; u.ttb = ttb[l];
        if (jmp) {
          u.jmp = jmp; u.ldj = nl * nb; u.ja = P.dja + box0 * n3; u.jb = P.djb + box0 * n3;
          u.jbase = h0 * nb;
        }
        u.c64 = P.c64;
        if (tl) {
          u.per = per;
          for (int q = 0; q < ax->np; ++q) {
            u.R33b[q] = tl->R33b[q]; u.Winv[q] = tl->Winv[q]; u.R33a[q] = tl->R33a[q];
            u.R13a[q] = tl->R13a[q]; u.R23b[q] = tl->R23b[q]; u.nrq[q] = ax->nrq[q];
          }
        } else {
          u.per = (int)nbox;
          u.R33b[0] = op(P.R33b, n3 * n3); u.Winv[0] = op(P.Winv, n3 * n3);
          u.R33a[0] = op(P.R33a, n3 * n3); u.R13a[0] = op(P.R13a, n1 * n3);
          u.R23b[0] = op(P.R23b, n2 * n3);
        }
        const double fl = 8.0 * nbox * nrhs * (3.0 * n3 * n3 + (double)(n1 + n2) * n3);
        // operators once; children's h in, t~3a, t~3b and h out
        const double by = nbox * ((3.0 * n3 * n3 + (double)(n1 + n2) * n3) * 8.0 * e +
                                  (2.0 * P.nbc + 2.0 * n3 + nbp) * nrhs * 16.0);
        Stage sg(pr, nm, fl, by);
        if (!ws.dry) up_fused(u, st);
        continue;
      }
      double* h3a = ws.get((size_t)nbox * n3 * nrhs * 16);
      double* v = ws.get((size_t)nbox * n3 * nrhs * 16);
      tta[l] = ws.get((size_t)nbox * n3 * nrhs * 16);
      ttb[l] = ws.get((size_t)nbox * n3 * nrhs * 16);
      h[l] = ws.get((size_t)nbox * nbp * nrhs * 16);
      {
        Stage sg(pr, "solve_gather", 0.0, nbox * (2.0 * P.nbc + 3.0 * n3 + nbp) * nrhs * 16);
        if (!ws.dry)
          up_gather(d, nrhs, h[l + 1], h3a, v, ttb[l], h[l], jmp, nl * nb,
                    jmp ? P.dja + box0 * n3 : nullptr, jmp ? P.djb + box0 * n3 : nullptr,
                    h0 * nb, st);
      }
      // v = R33b h3a - h3b
      SkinnyDesc k;
      k.M = n3; k.K = n3; k.nrhs = nrhs; k.batch = (int)nbox; k.a_c64 = P.c64;
      k.A = op(P.R33b, n3 * n3); k.lda = n3; k.sA = n3 * n3;
      if (tl) ax->put(k, per, tl->R33b);
      k.X = h3a; k.ldx = n3; k.sX = n3 * nrhs;
      k.C = v; k.ldc = n3; k.sC = n3 * nrhs; k.accumulate = true;
      ws.skinny(pr, nm, k);
      // t~3a = W^{-1} v
      k = SkinnyDesc();
      k.M = n3; k.K = n3; k.nrhs = nrhs; k.batch = (int)nbox; k.a_c64 = P.c64;
      k.A = op(P.Winv, n3 * n3); k.lda = n3; k.sA = n3 * n3;
      if (tl) ax->put(k, per, tl->Winv);
      k.X = v; k.ldx = n3; k.sX = n3 * nrhs;
      k.C = tta[l]; k.ldc = n3; k.sC = n3 * nrhs;
      ws.skinny(pr, nm, k);
      // t~3b = -h3a - R33a t~3a
      k = SkinnyDesc();
      k.M = n3; k.K = n3; k.nrhs = nrhs; k.batch = (int)nbox; k.a_c64 = P.c64;
      k.A = op(P.R33a, n3 * n3); k.lda = n3; k.sA = n3 * n3;
      if (tl) ax->put(k, per, tl->R33a);
      k.X = tta[l]; k.ldx = n3; k.sX = n3 * nrhs;
      k.C = ttb[l]; k.ldc = n3; k.sC = n3 * nrhs; k.accumulate = true; k.alpha = -1.0;
      ws.skinny(pr, nm, k);
      if (l > 0) {
        // h^tau = [h1a + R13a t~3a ; h2b + R23b t~3b]   (eq. (flux_part)); the two halves
        // write disjoint rows of h^tau and share a launch when the children are alike
        k = SkinnyDesc();
        k.M = n1; k.K = n3; k.nrhs = nrhs; k.batch = (int)nbox; k.a_c64 = P.c64;
        k.A = op(P.R13a, n1 * n3); k.lda = n1; k.sA = n1 * n3;
        k.X = tta[l]; k.ldx = n3; k.sX = n3 * nrhs;
        k.C = h[l]; k.ldc = nbp; k.sC = nbp * nrhs; k.crow = P.dperm; k.accumulate = true;
        if (n1 == n2) {
          k.A2 = op(P.R23b, n2 * n3); k.X2 = ttb[l]; k.C2 = h[l]; k.crow2 = P.dperm + n1;
          if (tl) ax->put(k, per, tl->R13a, tl->R23b);
          ws.skinny(pr, nm, k);
        } else {
          if (tl) ax->put(k, per, tl->R13a);
          ws.skinny(pr, nm, k);
          k.M = n2;
          k.A = op(P.R23b, n2 * n3); k.lda = n2; k.sA = n2 * n3;
          if (tl) ax->put(k, per, tl->R23b);
          k.X = ttb[l];
          k.crow = P.dperm + n1;
          ws.skinny(pr, nm, k);
        }
      }
    }
  }
  // downward pass   (steps (10)-(18))
  nm = "solve_merge_down";
  for (int l = 0; l < f.L; ++l) {
    LevelPlan& P = f.lv[l];
    MergeLevelDesc d = level_desc(f, P);
    const long nbox = (long)np << l, box0 = (long)pb << l;
    d.nbox = (int)nbox;
    const long n3 = P.n3, nbp = P.nbp, nbc = P.nbc;
    const int e = P.c64 ? 1 : 2;
    const double* tp = (l == 0) ? t : tt[l];
    const long sp = nbp * nrhs;
    tt[l + 1] = ws.get((size_t)2 * nbox * nbc * nrhs * 16);
    if (l > 0 && down_fused_fits(P.n1, P.n2, (int)n3, (int)nbp)) {
      // a short interface: the children's outer rows and both Phi products of each box in
      // one launch, the parent's t in LDS
      DownLevelDesc dd;
      dd.nbox = (int)nbox; dd.nbc = (int)nbc; dd.n1 = P.n1; dd.n2 = P.n2; dd.n3 = (int)n3;
      dd.nbp = (int)nbp; dd.nrhs = nrhs;
      dd.perm = P.dperm; dd.i1a = P.di1a; dd.i3a = P.di3a; dd.i2b = P.di2b; dd.i3b = P.di3b;
      dd.tp = tp; dd.tc = tt[l + 1];
      if (up) {
        dd.tta = tta[l];
        dd.ttb = ttb[l];
      }
      dd.c64 = P.c64;
      if (ax) {
        dd.per = 1 << l;
        for (int q = 0; q < ax->np; ++q) {
          dd.PhiA[q] = ax->lv[l].PhiA[q]; dd.PhiB[q] = ax->lv[l].PhiB[q]; dd.nrq[q] = ax->nrq[q];
        }
      } else {
        dd.per = (int)nbox;
        dd.PhiA[0] = P.PhiA.d() + box0 * n3 * nbp * e;
        dd.PhiB[0] = P.PhiB.d() + box0 * n3 * nbp * e;
      }
      const double fl = 16.0 * nbox * nrhs * (double)n3 * nbp;
      const double by = nbox * (2.0 * n3 * nbp * 8.0 * e +
                                (nbp + 2.0 * nbc + (up ? 2.0 * n3 : 0.0)) * nrhs * 16.0);
      Stage sg(pr, nm, fl, by);
      if (!ws.dry) down_fused(dd, st);
      continue;
    }
    {
      Stage sg(pr, "solve_gather", 0.0, nbox * 2.0 * (P.n1 + P.n2) * nrhs * 16);
      if (!ws.dry) down_scatter(d, nrhs, tp, nbp, tt[l + 1], st);
    }
    // both children's interface values in one launch: t3 = Phi^a t (+ t~3a) into child
    // a's slot, Phi^b t (+ t~3b) into child b's
    SkinnyDesc k;
    k.M = n3; k.K = nbp; k.nrhs = nrhs; k.batch = (int)nbox; k.a_c64 = P.c64;
    k.A = P.PhiA.d() + box0 * n3 * nbp * e;
    k.A2 = P.PhiB.d() + box0 * n3 * nbp * e;
    if (ax) ax->put(k, 1 << l, ax->lv[l].PhiA, ax->lv[l].PhiB);
    k.lda = n3; k.sA = n3 * nbp;
    k.X = tp; k.ldx = nbp; k.sX = sp;
    k.C = tt[l + 1]; k.C2 = tt[l + 1] + 2 * nbc * nrhs; k.ldc = nbc; k.sC = 2 * nbc * nrhs;
    k.crow = P.di3a; k.crow2 = P.di3b;
    if (up) {
      k.C0 = tta[l]; k.C02 = ttb[l]; k.ld0 = n3; k.s0 = n3 * nrhs;
    }
    ws.skinny(pr, nm, k);
  }
  // leaves: u = Psi t + u~   (step (13))
  {
    nm = "solve_leaf_down";
    SkinnyDesc k;
    k.M = n; k.K = nb; k.nrhs = nrhs; k.batch = (int)nl; k.a_c64 = f.mixed;
    k.A = leafops; k.lda = n; k.sA = n * n;
    if (ax) ax->put(k, f.nl1, ax->leaf);
    k.X = (f.L == 0) ? t : tt[f.L]; k.ldx = nb; k.sX = nb * nrhs;
    k.C = u; k.ldc = nl * n; k.coff = uoff; k.cbase = lbase * n;
    if (up) {
      k.C0 = ut; k.ld0 = n; k.s0 = n * nrhs;
    }
    ws.skinny(pr, nm, k);
  }
}

template <class F>
int guard(F&& fn) {
  try {
    g_err.clear();
    fn();
    return HPS_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return HPS_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return HPS_E_DEVICE;
  }
}

void validate_domain(const hps_domain* dom, int p) {
  if (!dom) throw Error(HPS_E_INVALID, "domain is NULL");
  if (p < 4 || p > 16) throw Error(HPS_E_INVALID, "p must be in [4, 16]");
  if (!is_pow2(dom->nx) || !is_pow2(dom->ny))
    throw Error(HPS_E_INVALID, "nx and ny must be powers of two");
  if ((long)dom->nx * dom->ny > 65536) throw Error(HPS_E_INVALID, "nx*ny must be <= 65536");
  if (!(std::isfinite(dom->x0) && std::isfinite(dom->x1) && std::isfinite(dom->y0) &&
        std::isfinite(dom->y1)) ||
      !(dom->x1 > dom->x0) || !(dom->y1 > dom->y0))
    throw Error(HPS_E_INVALID, "domain bounds must be finite with x1 > x0, y1 > y0");
}

}  // namespace
}  // namespace hps

using namespace hps;

extern "C" {

const char* hps_last_error(void) { return g_err.c_str(); }

int32_t hps_version(void) { return 10000; }

void hps_default_opts(hps_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = HPS_PREC_C128;
  o->keep_all_R = 0;
  o->store_root_R = 1;
  o->stream = nullptr;
  o->fp64_top_levels = 3;
  o->refine_max_iter = -1;
  o->refine_tol = 1e-12;
  o->autotune = 0;
}

int hps_nodes(const hps_domain* dom, int32_t p, double* xy_leaf, double* xy_interior,
              double* xy_root, double* nrm_root) {
  return guard([&] {
    validate_domain(dom, p);
    std::vector<double> x, D;
    cheb(p, x, D);
    const int m = p - 2, n = p * p - 4, nb = 4 * m, nx = dom->nx, ny = dom->ny;
    const double hx = (dom->x1 - dom->x0) / nx, hy = (dom->y1 - dom->y0) / ny;
    auto X = [&](int ix, int i) { return dom->x0 + ix * hx + hx * (1.0 + x[i]) / 2.0; };
    auto Y = [&](int iy, int j) { return dom->y0 + iy * hy + hy * (1.0 + x[j]) / 2.0; };
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix) {
        const long l = (long)iy * nx + ix;
        std::vector<double> pts;
        pts.reserve(2 * n);
        for (int i = 1; i <= m; ++i) { pts.push_back(X(ix, i)); pts.push_back(Y(iy, 0)); }
        for (int j = 1; j <= m; ++j) { pts.push_back(X(ix, p - 1)); pts.push_back(Y(iy, j)); }
        for (int i = 1; i <= m; ++i) { pts.push_back(X(ix, i)); pts.push_back(Y(iy, p - 1)); }
        for (int j = 1; j <= m; ++j) { pts.push_back(X(ix, 0)); pts.push_back(Y(iy, j)); }
        for (int j = 1; j <= m; ++j)
          for (int i = 1; i <= m; ++i) { pts.push_back(X(ix, i)); pts.push_back(Y(iy, j)); }
        if (xy_leaf) std::memcpy(xy_leaf + 2 * l * n, pts.data(), 2 * n * sizeof(double));
        if (xy_interior)
          std::memcpy(xy_interior + 2 * l * m * m, pts.data() + 2 * nb, 2 * m * m * sizeof(double));
      }
    long k = 0;
    auto put = [&](double px, double py, double nxv, double nyv) {
      if (xy_root) { xy_root[2 * k] = px; xy_root[2 * k + 1] = py; }
      if (nrm_root) { nrm_root[2 * k] = nxv; nrm_root[2 * k + 1] = nyv; }
      ++k;
    };
    for (int ix = 0; ix < nx; ++ix)
      for (int i = 1; i <= m; ++i) put(X(ix, i), Y(0, 0), 0.0, -1.0);
    for (int iy = 0; iy < ny; ++iy)
      for (int j = 1; j <= m; ++j) put(X(nx - 1, p - 1), Y(iy, j), 1.0, 0.0);
    for (int ix = 0; ix < nx; ++ix)
      for (int i = 1; i <= m; ++i) put(X(ix, i), Y(ny - 1, p - 1), 0.0, 1.0);
    for (int iy = 0; iy < ny; ++iy)
      for (int j = 1; j <= m; ++j) put(X(0, 0), Y(iy, j), -1.0, 0.0);
  });
}

}  // extern "C"

namespace hps {
namespace {

void check_problem(const hps_domain* dom, int p, double kappa, double er, double ei,
                   const double* c) {
  validate_domain(dom, p);
  if (!c) throw Error(HPS_E_INVALID, "c_interior is NULL");
  if (!std::isfinite(kappa) || kappa < 0) throw Error(HPS_E_INVALID, "kappa must be finite, >= 0");
  if (!std::isfinite(er) || !std::isfinite(ei) || er == 0.0)
    throw Error(HPS_E_INVALID, "eta must be finite with Re(eta) != 0");
}

// Build the factorizations of nprob problems that share domain, leaf grid and p.
// shape groups of one hps_build_batch call built at the same time
constexpr size_t kBatchStreams = 4;

std::shared_ptr<hps_group> build_group(const hps_domain& dom, int p, int nprob,
                                       const double* kappa, const double* er, const double* ei,
                                       const double* const* c, const hps_opts* opts) {
  auto f = std::make_shared<hps_group>();
  if (opts) f->opts = *opts; else hps_default_opts(&f->opts);
  if (f->opts.precision != HPS_PREC_C128 && f->opts.precision != HPS_PREC_MIXED)
    throw Error(HPS_E_INVALID, "unsupported precision mode");
  if (f->opts.fp64_top_levels < 0) throw Error(HPS_E_INVALID, "fp64_top_levels must be >= 0");
  if (!(f->opts.refine_tol > 0.0)) throw Error(HPS_E_INVALID, "refine_tol must be > 0");
  f->mixed = f->opts.precision == HPS_PREC_MIXED;
  f->full_pivoting = f->opts.interface_pivoting == 1;
  f->p = p; f->m = p - 2; f->n = p * p - 4; f->nb = 4 * (p - 2); f->ni = (p - 2) * (p - 2);
  f->nx = dom.nx; f->ny = dom.ny;
  f->nprob = nprob; f->nl1 = dom.nx * dom.ny; f->nleaf = f->nl1 * nprob;
  f->x0 = dom.x0; f->x1 = dom.x1; f->y0 = dom.y0; f->y1 = dom.y1;
  f->prm_h.assign((size_t)4 * nprob, 0.0);
  for (int b = 0; b < nprob; ++b) {
    f->prm_h[4 * b] = kappa[b];
    f->prm_h[4 * b + 1] = er[b];
    f->prm_h[4 * b + 2] = ei[b];
  }
  f->stream = static_cast<hipStream_t>(f->opts.stream);
  attach_plan(*f, plan_for(*f));
  for (int l = 0; l < f->L; ++l) {
    f->lv[l].c64 = f->mixed;
    f->lv[l].inv64 = f->mixed && l < f->opts.fp64_top_levels;
  }
  upload_tables(*f);
  // the group's own copy of c (problem-major), read by the leaf stage and the residual
  const size_t per = (size_t)f->nl1 * f->ni * sizeof(double);
  f->dc.alloc(per * nprob);
  for (int b = 0; b < nprob; ++b)
    HPS_HIP(hipMemcpyAsync(static_cast<char*>(f->dc.p) + per * b, c[b], per,
                           hipMemcpyDeviceToDevice, f->stream));
  f->build_prof.reset(f->opts.profile != 0, f->stream);
  build_all(*f, f->dc.d());
  return f;
}

}  // namespace
}  // namespace hps

extern "C" {

int hps_build(const hps_domain* dom, int32_t p, double kappa, double eta_re, double eta_im,
              const double* c_interior, const hps_opts* opts, hps_factor** out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!out) throw Error(HPS_E_INVALID, "out is NULL");
    check_problem(dom, p, kappa, eta_re, eta_im, c_interior);
    std::unique_ptr<hps_factor> h(new hps_factor);
    h->g = build_group(*dom, p, 1, &kappa, &eta_re, &eta_im, &c_interior, opts);
    h->b0 = 0;
    *out = h.release();
  });
}

int hps_build_batch(int32_t nprob, const hps_domain* doms, const int32_t* p,
                    const double* kappa, const double* eta_re, const double* eta_im,
                    const double* const* c_interior, const hps_opts* opts, hps_factor** out) {
  if (out && nprob > 0)
    for (int i = 0; i < nprob; ++i) out[i] = nullptr;
  std::vector<std::unique_ptr<hps_factor>> made;
  int rc = guard([&] {
    if (nprob < 1) throw Error(HPS_E_INVALID, "nprob must be >= 1");
    if (!out || !doms || !p || !kappa || !eta_re || !eta_im || !c_interior)
      throw Error(HPS_E_INVALID, "NULL argument");
    for (int i = 0; i < nprob; ++i)
      check_problem(&doms[i], p[i], kappa[i], eta_re[i], eta_im[i], c_interior[i]);
    made.resize(nprob);
    // problems of one shape (domain, leaf grid, p) share a group, in first-seen order
    std::vector<char> done(nprob, 0);
    std::vector<std::vector<int>> groups;
    for (int i = 0; i < nprob; ++i) {
      if (done[i]) continue;
      std::vector<int> mem;
      for (int j = i; j < nprob; ++j) {
        const hps_domain &a = doms[i], &b = doms[j];
        if (!done[j] && p[j] == p[i] && a.nx == b.nx && a.ny == b.ny && a.x0 == b.x0 &&
            a.x1 == b.x1 && a.y0 == b.y0 && a.y1 == b.y1) {
          mem.push_back(j);
          done[j] = 1;
        }
      }
      groups.push_back(std::move(mem));
    }
    auto build_one = [&](const std::vector<int>& mem, const hps_opts* o) {
      std::vector<double> k(mem.size()), er(mem.size()), ei(mem.size());
      std::vector<const double*> cs(mem.size());
      for (size_t q = 0; q < mem.size(); ++q) {
        k[q] = kappa[mem[q]]; er[q] = eta_re[mem[q]]; ei[q] = eta_im[mem[q]];
        cs[q] = c_interior[mem[q]];
      }
      return build_group(doms[mem[0]], p[mem[0]], (int)mem.size(), k.data(), er.data(),
                         ei.data(), cs.data(), o);
    };
    std::vector<std::shared_ptr<hps_group>> gs(groups.size());
    if (groups.size() == 1) {
      gs[0] = build_one(groups[0], opts);
    } else {
      // Groups are built concurrently, each on a stream of its own (up to kBatchStreams
      // at a time), so that the launches of different shapes overlap on the device.  The
      // streams start after the caller's queued work (the inputs) and are synchronized
      // before returning; the groups then keep the caller's stream for later calls.
      hps_opts base;
      if (opts) base = *opts; else hps_default_opts(&base);
      hipStream_t caller = static_cast<hipStream_t>(base.stream);
      int dev = 0;
      HPS_HIP(hipGetDevice(&dev));
      hipEvent_t ready = nullptr;
      HPS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      struct EvFree {
        hipEvent_t e;
        ~EvFree() { (void)hipEventDestroy(e); }
      } evf{ready};
      HPS_HIP(hipEventRecord(ready, caller));
      std::atomic<size_t> next{0};
      std::mutex emu;
      std::exception_ptr err;
      auto worker = [&]() {
        hipStream_t st = nullptr;
        try {
          HPS_HIP(hipSetDevice(dev));
          // default priority, like every stream of the library
          HPS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
          HPS_HIP(hipStreamWaitEvent(st, ready, 0));
          hps_opts o = base;
          o.stream = st;
          for (size_t i = next++; i < groups.size(); i = next++) {
            {
              std::lock_guard<std::mutex> lk(emu);
              if (err) break;
            }
            gs[i] = build_one(groups[i], &o);
          }
          HPS_HIP(hipStreamSynchronize(st));
        } catch (...) {
          std::lock_guard<std::mutex> lk(emu);
          if (!err) err = std::current_exception();
        }
        if (st) {
          (void)hipStreamSynchronize(st);
          (void)hipStreamDestroy(st);
        }
      };
      const int nw = (int)std::min<size_t>(groups.size(), kBatchStreams);
      std::vector<std::thread> th;
      for (int w = 0; w < nw; ++w) th.emplace_back(worker);
      for (auto& t : th) t.join();
      if (err) std::rethrow_exception(err);
      for (auto& g : gs) {
        g->stream = caller;
        g->opts.stream = caller;
      }
    }
    for (size_t gi = 0; gi < groups.size(); ++gi)
      for (size_t q = 0; q < groups[gi].size(); ++q) {
        const int i = groups[gi][q];
        made[i].reset(new hps_factor);
        made[i]->g = gs[gi];
        made[i]->b0 = (int)q;
      }
  });
  if (rc == HPS_OK)
    for (int i = 0; i < nprob; ++i) out[i] = made[i].release();
  return rc;
}

}  // extern "C"

namespace hps {
namespace {

// Device address of the scratch array on the current device, looked up once per device
// (each GPU holds its own copy of the array, at its own address).
char* noalloc_scratch() {
  static std::mutex mu;
  static std::vector<char*> addr;
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    HPS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(HPS_E_DEVICE, "no device address for the allocation-free scratch");
    addr[dev] = static_cast<char*>(p);
  }
  return addr[dev];
}

ResidualDesc residual_desc(const hps_group& f, int pb, int np, int nrhs, const double* s,
                           const double* t, const double* jmp, const double* u) {
  ResidualDesc r;
  r.p = f.p; r.nx = f.nx; r.ny = f.ny; r.nprob = np; r.nrhs = nrhs;
  r.prm = f.dprm.d() + 4 * pb;
  r.D = f.dD.d(); r.c = f.dc.d() + (long)pb * f.nl1 * f.ni;
  r.u = u; r.s = s; r.t = t; r.jmp = jmp;
  return r;
}

int refine_iters(const hps_group& f) {
  if (f.opts.refine_max_iter >= 0) return f.opts.refine_max_iter;
  return f.opts.precision == HPS_PREC_MIXED ? 10 : 0;
}

// Solve problems [pb, pb + np), then (when enabled) residual correction in FP64:
// r = b - A u on the global collocation system, delta = Solve(r) with r's shared-edge
// rows as interface jumps, u += delta, until the relative correction |delta| / |u| of
// every right-hand side of every problem (each problem's share of a right-hand side
// measured on its own, so that problems of very different scale do not hide each other),
// or its contraction estimate of the next one, is <= tol, or the iteration limit.
void solve_impl(hps_group& f, int pb, int np, int nrhs, const double* s, const double* t,
                const double* jmp, double* u, hipStream_t st, hps_solve_info* info,
                size_t* ws_bytes = nullptr, char* fixed = nullptr, size_t fixed_cap = 0) {
  const int iters = refine_iters(f);
  const long nl = (long)np * f.nl1, n = f.n, nb = f.nb, ni = f.ni;
  const long nt = 2L * (f.nx + f.ny) * f.m;
  const int nblk = norms_blocks();
  Arena ws;
  ws.st = st;
  ws.fixed = fixed;
  ws.fixed_cap = fixed_cap;
  double *rs = nullptr, *rt = nullptr, *rj = nullptr, *dl = nullptr, *part = nullptr;
  size_t mark = 0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      if (ws_bytes) {  // sizing only
        *ws_bytes = std::max(ws.used, ws.peak) + ws.split_need + 256;
        return;
      }
      ws.allocate();
    }
    if (iters > 0) {
      rs = ws.get((size_t)nrhs * nl * ni * 16);
      rt = ws.get((size_t)np * nrhs * nt * 16);
      rj = ws.get((size_t)nrhs * nl * nb * 16);
      dl = ws.get((size_t)nrhs * nl * n * 16);
      part = ws.get((size_t)nrhs * np * nblk * 2 * sizeof(double));
    }
    mark = ws.used;
    solve_pass(f, pb, np, nrhs, s, t, jmp, u, ws);  // pass 0 only sizes the workspace
    if (pass == 0 && iters > 0) {
      // the correction sweeps always run the upward pass: size the workspace for them too
      ws.used = mark;
      solve_pass(f, pb, np, nrhs, rs, rt, rj, dl, ws);
    }
  }
  *info = hps_solve_info{};
  if (iters <= 0) return;
  // norms per right-hand side and problem: u is [nrhs][np][nl1 * n], so column
  // c = r * np + q of length nl1 * n is problem q's share of right-hand side r
  const long ncol = (long)nrhs * np, clen = (long)f.nl1 * n;
  std::vector<double> hpart((size_t)ncol * nblk * 2);
  std::vector<double> prev((size_t)ncol, 0.0);  // previous relative correction per column
  double corr = 0.0;
  int it = 0;
  bool conv = false;
  for (it = 1; it <= iters; ++it) {
    ResidualDesc r = residual_desc(f, pb, np, nrhs, s, t, jmp, u);
    r.rs = rs; r.rs_rhs = nl * ni; r.rs_leaf = ni;
    r.rb = rj; r.rb_rhs = nl * nb; r.rb_leaf = nb;
    r.rt = rt;
    residual(r, nrhs, st);
    ws.used = mark;
    solve_pass(f, pb, np, nrhs, rs, rt, rj, dl, ws);
    norms_partial(clen, (int)ncol, dl, u, part, st);
    axpy((long)nrhs * nl * n, dl, u, st);
    HPS_HIP(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(double),
                           hipMemcpyDeviceToHost, st));
    HPS_HIP(hipStreamSynchronize(st));
    // Per right-hand side of each problem: c = ||delta|| / ||u||.  Done when every c <=
    // tol, or when the corrections contract (c below half the previous one) fast enough
    // that the next one, estimated as c * (c / c_prev), is <= tol: then u already
    // carries the accuracy another sweep would only confirm.  corr reports the larger of
    // c and that estimate over the columns.
    corr = 0.0;
    bool all_done = true;
    for (long q = 0; q < ncol; ++q) {
      double dd = 0, uu = 0;
      for (int b = 0; b < nblk; ++b) {
        dd += hpart[2 * ((size_t)q * nblk + b)];
        uu += hpart[2 * ((size_t)q * nblk + b) + 1];
      }
      const double c = uu > 0 ? std::sqrt(dd / uu) : std::sqrt(dd);
      double left = c;
      if (c > f.opts.refine_tol) {
        const double pq = prev[q];
        if (pq > 0.0 && c < 0.5 * pq) left = c * (c / pq);
        if (left > f.opts.refine_tol) all_done = false;
      }
      corr = std::max(corr, std::min(c, left));
      prev[q] = c;
    }
    if (all_done) {
      conv = true;
      break;
    }
  }
  info->iterations = std::min(it, iters);
  info->converged = conv ? 1 : 0;
  info->correction = corr;
  if (!conv)
    throw Error(HPS_E_NOT_CONVERGED, "residual correction did not reach refine_tol (last "
                                     "relative correction " + std::to_string(corr) + ")");
}

size_t align_up(size_t b) { return (b + 255) & ~size_t(255); }

// Problems of two factors can share a solve's launches when their trees, operator shapes
// and level precisions agree and no residual correction runs (the correction reads each
// problem's collocation data, which the tabled launches do not carry).
bool shareable(const hps_group& a, const hps_group& b) {
  if (a.nx != b.nx || a.ny != b.ny || a.p != b.p || a.L != b.L || a.mixed != b.mixed)
    return false;
  if (refine_iters(a) > 0 || refine_iters(b) > 0) return false;
  for (int l = 0; l < a.L; ++l)
    if (a.lv[l].c64 != b.lv[l].c64) return false;
  return true;
}

bool same_problem(const hps_factor* a, const hps_factor* b) {
  return a->g.get() == b->g.get() && a->b0 == b->b0;
}

// One solve over the parts' problems (pairwise shareable, at most Across::kMax distinct):
// parts on one problem take consecutive right-hand-side columns of it.  Right-hand sides
// are staged side by side as for a group of the problems, the sweeps run once through
// the tabled launches, and each part's solution is copied out.  With ws_bytes set, only
// returns the device bytes the call allocates (workspace and staging).
void solve_across(const std::vector<SolvePart>& parts, hipStream_t st, size_t* ws_bytes) {
  if (parts.empty()) return;
  std::vector<const hps_factor*> fs;
  std::vector<int> qof(parts.size()), col0(parts.size()), nrq;
  bool any_s = false;
  for (size_t i = 0; i < parts.size(); ++i) {
    const SolvePart& pt = parts[i];
    if (!pt.f || !pt.t || !pt.u || pt.nrhs < 1) throw Error(HPS_E_INVALID, "bad solve part");
    size_t q = 0;
    while (q < fs.size() && !same_problem(fs[q], pt.f)) ++q;
    if (q == fs.size()) {
      if (q > 0 && !shareable(*fs[0]->g, *pt.f->g))
        throw Error(HPS_E_INVALID, "problems of different shapes cannot share a solve");
      fs.push_back(pt.f);
      nrq.push_back(0);
    }
    qof[i] = (int)q;
    col0[i] = nrq[q];
    nrq[q] += pt.nrhs;
    any_s = any_s || pt.s != nullptr;
  }
  const int np = (int)fs.size();
  if (np > Across::kMax)
    throw Error(HPS_E_INVALID, "more than " + std::to_string(Across::kMax) +
                                   " problems in one shared solve");
  hps_group& g0 = *fs[0]->g;
  const int R = *std::max_element(nrq.begin(), nrq.end());
  const long nl1 = g0.nl1, nl = (long)np * nl1, n = g0.n, ni = g0.ni;
  const long nt = 2L * (g0.nx + g0.ny) * g0.m;
  Across ax;
  ax.np = np;
  {
    hps_group t;  // leaf maps of an np-problem group of this shape
    t.p = g0.p; t.m = g0.m; t.n = g0.n; t.nb = g0.nb; t.ni = g0.ni;
    t.nx = g0.nx; t.ny = g0.ny; t.nprob = np; t.nl1 = g0.nl1; t.nleaf = np * g0.nl1;
    ax.sh = plan_for(t);
  }
  ax.lv.resize(g0.L);
  for (int q = 0; q < np; ++q) {
    const hps_group& G = *fs[q]->g;
    const long b = fs[q]->b0;
    ax.nrq[q] = nrq[q];
    ax.leaf[q] = (G.mixed ? G.BI32.d() : G.BI.d()) + (G.mixed ? 1 : 2) * b * nl1 * n * n;
    ax.prm.p[q] = G.dprm.d() + 4 * b;
    for (int l = 0; l < G.L; ++l) {
      const LevelPlan& P = G.lv[l];
      const long box0 = b << l, e = P.c64 ? 1 : 2;
      const long n1 = P.n1, n2 = P.n2, n3 = P.n3, nbp = P.nbp;
      Across::Level& T = ax.lv[l];
      T.R33b[q] = P.R33b.d() + box0 * n3 * n3 * e;
      T.Winv[q] = P.Winv.d() + box0 * n3 * n3 * e;
      T.R33a[q] = P.R33a.d() + box0 * n3 * n3 * e;
      T.R13a[q] = P.R13a.d() + box0 * n1 * n3 * e;
      T.R23b[q] = P.R23b.d() + box0 * n2 * n3 * e;
      T.PhiA[q] = P.PhiA.d() + box0 * n3 * nbp * e;
      T.PhiB[q] = P.PhiB.d() + box0 * n3 * nbp * e;
    }
  }
  const size_t bs = any_s ? align_up((size_t)R * nl * ni * 16) : 0;
  const size_t bt = align_up((size_t)np * R * nt * 16), bu = align_up((size_t)R * nl * n * 16);
  Arena ws;
  ws.st = st;
  // sizing pass: placeholders stand in for the vectors and are never dereferenced
  const double* ph = reinterpret_cast<const double*>(4096);
  solve_pass(g0, 0, np, R, any_s ? ph : nullptr, ph, nullptr, const_cast<double*>(ph), ws, &ax);
  if (ws_bytes) {
    *ws_bytes = std::max(ws.used, ws.peak) + ws.split_need + 256 + bs + bt + bu + 256;
    return;
  }
  void* stage = ws_alloc(bs + bt + bu + 256, st);
  struct Free {
    void* p; hipStream_t st;
    ~Free() { ws_free(p, st); }
  } fr{stage, st};
  char* base = static_cast<char*>(stage);
  double* S = any_s ? reinterpret_cast<double*>(base) : nullptr;
  double* T = reinterpret_cast<double*>(base + bs);
  double* U = reinterpret_cast<double*>(base + bs + bt);
  // columns of a problem beyond its own right-hand sides are never read: the tabled
  // launches skip them, so only the parts' columns are staged
  for (size_t i = 0; i < parts.size(); ++i) {
    const SolvePart& pt = parts[i];
    const long q = qof[i], c = col0[i];
    if (S) {
      double* dst = S + 2 * (c * nl + q * nl1) * ni;
      if (pt.s)
        HPS_HIP(hipMemcpy2DAsync(dst, (size_t)nl * ni * 16, pt.s, (size_t)nl1 * ni * 16,
                                 (size_t)nl1 * ni * 16, pt.nrhs, hipMemcpyDeviceToDevice, st));
      else
        for (int r = 0; r < pt.nrhs; ++r) fill_zero(dst + 2 * r * nl * ni, 2 * nl1 * ni, st);
    }
    HPS_HIP(hipMemcpyAsync(T + 2 * (q * R + c) * nt, pt.t, (size_t)pt.nrhs * nt * 16,
                           hipMemcpyDeviceToDevice, st));
  }
  ws.allocate();
  solve_pass(g0, 0, np, R, S, T, nullptr, U, ws, &ax);
  for (size_t i = 0; i < parts.size(); ++i) {
    const SolvePart& pt = parts[i];
    const long q = qof[i], c = col0[i];
    HPS_HIP(hipMemcpy2DAsync(pt.u, (size_t)nl1 * n * 16, U + 2 * (c * nl + q * nl1) * n,
                             (size_t)nl * n * 16, (size_t)nl1 * n * 16, pt.nrhs,
                             hipMemcpyDeviceToDevice, st));
  }
  for (int q = 0; q < np; ++q) fs[q]->g->last_info = hps_solve_info{};
}

}  // namespace
}  // namespace hps

extern "C" {

int hps_solve(hps_factor* f, int32_t nrhs, const double* s, const double* t, double* u) {
  return guard([&] {
    if (!f) throw Error(HPS_E_INVALID, "factor is NULL");
    if (!t || !u) throw Error(HPS_E_INVALID, "t and u must be non-NULL");
    if (nrhs < 1) throw Error(HPS_E_INVALID, "nrhs must be >= 1");
    hps_group& G = *f->g;
    solve_impl(G, f->b0, 1, nrhs, s, t, nullptr, u, G.stream, &G.last_info);
  });
}

int hps_solve_noalloc(hps_factor* f, int32_t nrhs, const double* s, const double* t,
                      double* u) {
  return guard([&] {
    if (!f) throw Error(HPS_E_INVALID, "factor is NULL");
    if (!t || !u) throw Error(HPS_E_INVALID, "t and u must be non-NULL");
    if (nrhs < 1) throw Error(HPS_E_INVALID, "nrhs must be >= 1");
    hps_group& G = *f->g;
    char* base = noalloc_scratch();
    solve_impl(G, f->b0, 1, nrhs, s, t, nullptr, u, G.stream, &G.last_info, nullptr, base,
               kNoAllocScratch);
  });
}

int hps_solve_jumps(hps_factor* f, int32_t nrhs, const double* s, const double* t,
                    const double* jumps, double* u) {
  return guard([&] {
    if (!f) throw Error(HPS_E_INVALID, "factor is NULL");
    if (!t || !u) throw Error(HPS_E_INVALID, "t and u must be non-NULL");
    if (nrhs < 1) throw Error(HPS_E_INVALID, "nrhs must be >= 1");
    hps_group& G = *f->g;
    solve_impl(G, f->b0, 1, nrhs, s, t, jumps, u, G.stream, &G.last_info);
  });
}

int hps_solve_batch(int32_t nprob, hps_factor* const* f, const int32_t* nrhs,
                    const double* const* s, const double* const* t, double* const* u) {
  return guard([&] {
    if (nprob < 1) throw Error(HPS_E_INVALID, "nprob must be >= 1");
    if (!f || !nrhs || !t || !u) throw Error(HPS_E_INVALID, "NULL argument");
    for (int i = 0; i < nprob; ++i) {
      if (!f[i] || !t[i] || !u[i]) throw Error(HPS_E_INVALID, "NULL factor, t or u");
      if (nrhs[i] < 1) throw Error(HPS_E_INVALID, "nrhs must be >= 1");
    }
    for (int i = 0; i < nprob; ++i)
      for (int j = 0; j < i; ++j)
        if (same_problem(f[i], f[j]))
          throw Error(HPS_E_INVALID, "a problem appears twice in one batch");
    // Requests of one group go through one batched solve over the problem range they
    // span (problems of the range without a request get zero data).  Requests on
    // shareable problems of several groups on one stream share tabled launches, up to
    // Across::kMax problems per solve.
    std::vector<char> done(nprob, 0);
    for (int i = 0; i < nprob; ++i) {
      if (done[i]) continue;
      hps_group& G = *f[i]->g;
      std::vector<int> mem, other;
      for (int j = i; j < nprob; ++j) {
        if (done[j]) continue;
        if (f[j]->g.get() == &G) mem.push_back(j);
        else if (f[j]->g->stream == G.stream && shareable(G, *f[j]->g)) other.push_back(j);
      }
      if (!other.empty()) {
        std::vector<int> all(mem);
        all.insert(all.end(), other.begin(), other.end());
        std::sort(all.begin(), all.end());
        for (size_t a = 0; a < all.size(); a += Across::kMax) {
          std::vector<SolvePart> parts;
          for (size_t b = a; b < std::min(all.size(), a + Across::kMax); ++b) {
            const int j = all[b];
            done[j] = 1;
            parts.push_back({f[j], nrhs[j], s ? s[j] : nullptr, t[j], u[j]});
          }
          solve_across(parts, G.stream, nullptr);
        }
        continue;
      }
      for (int j : mem) done[j] = 1;
      int pb = G.nprob, pe = 0, R = 1;
      bool any_s = false;
      for (int j : mem) {
        const int b = f[j]->b0;
        pb = std::min(pb, b);
        pe = std::max(pe, b + 1);
        R = std::max(R, (int)nrhs[j]);
        any_s = any_s || (s && s[j]);
      }
      const int np = pe - pb;
      const long nl = (long)np * G.nl1, n = G.n, ni = G.ni;
      const long nt = 2L * (G.nx + G.ny) * G.m;
      hipStream_t st = G.stream;
      const size_t bs = any_s ? (size_t)R * nl * ni * 16 : 0, bt = (size_t)np * R * nt * 16,
                   bu = (size_t)R * nl * n * 16;
      void* stage = ws_alloc(bs + bt + bu + 512, st);
      struct Free {
        void* p; hipStream_t st;
        ~Free() { ws_free(p, st); }
      } fr{stage, st};
      char* base = static_cast<char*>(stage);
      double* S = any_s ? reinterpret_cast<double*>(base) : nullptr;
      double* T = reinterpret_cast<double*>(base + ((bs + 255) & ~size_t(255)));
      double* U = reinterpret_cast<double*>(base + ((bs + 255) & ~size_t(255)) +
                                            ((bt + 255) & ~size_t(255)));
      if (S) fill_zero(S, (long)(bs / 8), st);
      fill_zero(T, (long)(bt / 8), st);
      for (int j : mem) {
        const long o = f[j]->b0 - pb;
        if (S && s[j])
          HPS_HIP(hipMemcpy2DAsync(S + 2 * o * G.nl1 * ni, (size_t)nl * ni * 16, s[j],
                                   (size_t)G.nl1 * ni * 16, (size_t)G.nl1 * ni * 16, nrhs[j],
                                   hipMemcpyDeviceToDevice, st));
        HPS_HIP(hipMemcpyAsync(T + 2 * o * R * nt, t[j], (size_t)nrhs[j] * nt * 16,
                               hipMemcpyDeviceToDevice, st));
      }
      solve_impl(G, pb, np, R, S, T, nullptr, U, st, &G.last_info);
      for (int j : mem) {
        const long o = f[j]->b0 - pb;
        HPS_HIP(hipMemcpy2DAsync(u[j], (size_t)G.nl1 * n * 16, U + 2 * o * G.nl1 * n,
                                 (size_t)nl * n * 16, (size_t)G.nl1 * n * 16, nrhs[j],
                                 hipMemcpyDeviceToDevice, st));
      }
    }
  });
}

int hps_residual(hps_factor* f, int32_t nrhs, const double* s, const double* t,
                 const double* jumps, const double* u, double* r) {
  return guard([&] {
    if (!f) throw Error(HPS_E_INVALID, "factor is NULL");
    if (!u || !r) throw Error(HPS_E_INVALID, "u and r must be non-NULL");
    if (nrhs < 1) throw Error(HPS_E_INVALID, "nrhs must be >= 1");
    hps_group& G = *f->g;
    const long nl = G.nl1, n = G.n, nb = G.nb;
    ResidualDesc d = residual_desc(G, f->b0, 1, nrhs, s, t, jumps, u);
    d.rs = r + 2 * nb; d.rs_rhs = nl * n; d.rs_leaf = n;
    d.rb = r; d.rb_rhs = nl * n; d.rb_leaf = n;
    residual(d, nrhs, G.stream);
  });
}

int hps_last_solve_info(const hps_factor* f, hps_solve_info* info) {
  return guard([&] {
    if (!f || !info) throw Error(HPS_E_INVALID, "factor and info must be non-NULL");
    *info = f->g->last_info;
  });
}

int hps_factor_query(const hps_factor* h, hps_factor_info* info) {
  return guard([&] {
    if (!h || !info) throw Error(HPS_E_INVALID, "NULL argument");
    const hps_group* f = h->g.get();
    info->p = f->p; info->nx = f->nx; info->ny = f->ny; info->levels = f->L;
    info->nleaf = f->nl1;
    info->n_leaf_nodes = (int64_t)f->nl1 * f->n;
    info->n_interior = (int64_t)f->nl1 * f->ni;
    info->n_root = 2L * (f->nx + f->ny) * f->m;
    info->device_bytes = (int64_t)f->bytes();
  });
}

int hps_factor_box(const hps_factor* h, int32_t level, int32_t box, int32_t* ix0, int32_t* ix1,
                   int32_t* iy0, int32_t* iy1) {
  return guard([&] {
    if (!h) throw Error(HPS_E_INVALID, "factor is NULL");
    const hps_group* f = h->g.get();
    if (level < 0 || level > f->L || box < 0 || box >= (1 << level))
      throw Error(HPS_E_INVALID, "level/box out of range");
    const Geo& g = f->geo[level][box];
    if (ix0) *ix0 = g.ix0;
    if (ix1) *ix1 = g.ix0 + g.wx;
    if (iy0) *iy0 = g.iy0;
    if (iy1) *iy1 = g.iy0 + g.wy;
  });
}

int hps_factor_get(const hps_factor* h, int32_t what, int32_t level, int32_t box, double* dst,
                   int64_t dst_len, int32_t* rows, int32_t* cols) {
  return guard([&] {
    if (!h || !dst) throw Error(HPS_E_INVALID, "NULL argument");
    const hps_group* f = h->g.get();
    if (level < 0 || level > f->L || box < 0 || box >= (1 << level))
      throw Error(HPS_E_INVALID, "level/box out of range");
    const double* src = nullptr;
    long r = 0, c = 0, ld = 0;
    long off = 0;
    bool c64 = false;  // stored as complex64
    if (what == HPS_OP_PSI || what == HPS_OP_Y) {
      if (level != f->L) throw Error(HPS_E_INVALID, "Psi/Y exist on the leaf level only");
      c64 = f->mixed;
      src = c64 ? f->BI32.d() : f->BI.d();
      r = f->n; ld = f->n;
      c = (what == HPS_OP_PSI) ? f->nb : f->ni;
      off = ((long)h->b0 * f->nl1 + box) * f->n * f->n +
            (what == HPS_OP_PSI ? 0 : (long)f->n * f->nb);
    } else if (what == HPS_OP_R) {
      if (!f->R_valid[level]) throw Error(HPS_E_INVALID, "R of this level is not kept");
      c64 = cbytes(*f, level) == 8;
      src = f->R[level].d();
      r = c = ld = f->nbl[level];
      off = (((long)h->b0 << level) + box) * r * r;
    } else {
      if (level >= f->L) throw Error(HPS_E_INVALID, "merge operators live on levels < leaves");
      const LevelPlan& P = f->lv[level];
      const View* b = nullptr;
      switch (what) {
        case HPS_OP_WINV: b = &P.Winv; r = c = P.n3; break;
        case HPS_OP_PHI_A: b = &P.PhiA; r = P.n3; c = P.nbp; break;
        case HPS_OP_PHI_B: b = &P.PhiB; r = P.n3; c = P.nbp; break;
        case HPS_OP_R33A: b = &P.R33a; r = c = P.n3; break;
        case HPS_OP_R33B: b = &P.R33b; r = c = P.n3; break;
        case HPS_OP_R13A: b = &P.R13a; r = P.n1; c = P.n3; break;
        case HPS_OP_R23B: b = &P.R23b; r = P.n2; c = P.n3; break;
        default: throw Error(HPS_E_INVALID, "unknown operator id");
      }
      src = b->d();
      c64 = P.c64;
      ld = r;
      off = (((long)h->b0 << level) + box) * r * c;
    }
    if (rows) *rows = (int32_t)r;
    if (cols) *cols = (int32_t)c;
    if (dst_len < r * c) throw Error(HPS_E_INVALID, "destination too small");
    HPS_HIP(hipStreamSynchronize(f->stream));
    if (!c64) {
      HPS_HIP(hipMemcpy2D(dst, r * 16, src + 2 * off, ld * 16, r * 16, c, hipMemcpyDeviceToHost));
    } else {
      // complex64 storage: copy, then widen to the complex128 layout of dst
      std::vector<float> tmp((size_t)2 * r * c);
      const float* s32 = reinterpret_cast<const float*>(src) + 2 * off;
      HPS_HIP(hipMemcpy2D(tmp.data(), r * 8, s32, ld * 8, r * 8, c, hipMemcpyDeviceToHost));
      for (size_t e = 0; e < tmp.size(); ++e) dst[e] = tmp[e];
    }
  });
}

int hps_stage_times(const hps_factor* h, int32_t which, hps_stage_time* out, int32_t cap,
                    int32_t* n) {
  return guard([&] {
    if (!h || !out || !n || cap < 0) throw Error(HPS_E_INVALID, "NULL argument");
    const hps_group* f = h->g.get();
    if (which != 0 && which != 1) throw Error(HPS_E_INVALID, "which must be 0 (build) or 1 (solve)");
    const Profiler& pr = which == 0 ? f->build_prof : f->solve_prof;
    std::vector<hps_stage_time> agg;
    for (const StageRec& r : pr.recs) {
      HPS_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      HPS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      hps_stage_time* s = nullptr;
      for (auto& a : agg)
        if (r.name == a.name) s = &a;
      if (!s) {
        hps_stage_time z;
        std::memset(&z, 0, sizeof(z));
        std::strncpy(z.name, r.name.c_str(), sizeof(z.name) - 1);
        agg.push_back(z);
        s = &agg.back();
      }
      s->launches += 1;
      s->ms += ms;
      s->flops += r.flops;
      s->bytes += r.bytes;
    }
    *n = (int32_t)std::min<size_t>(agg.size(), (size_t)cap);
    for (int i = 0; i < *n; ++i) out[i] = agg[i];
  });
}

void hps_free(hps_factor* f) { delete f; }

int hps_autotune_entries(int32_t* n) {
  return guard([&] {
    if (!n) throw Error(HPS_E_INVALID, "n is NULL");
    *n = zgemm_tune_entries();
  });
}

int hps_autotune_clear(void) {
  return guard([&] { zgemm_tune_clear(); });
}

int hps_autotune_save(const char* path) {
  return guard([&] {
    if (!path) throw Error(HPS_E_INVALID, "path is NULL");
    const std::string text = zgemm_tune_dump();
    FILE* fp = std::fopen(path, "w");
    if (!fp) throw Error(HPS_E_INVALID, std::string("cannot write ") + path);
    const size_t w = std::fwrite(text.data(), 1, text.size(), fp);
    const int c = std::fclose(fp);
    if (w != text.size() || c != 0) throw Error(HPS_E_INVALID, std::string("write failed: ") + path);
  });
}

int hps_autotune_load(const char* path) {
  return guard([&] {
    if (!path) throw Error(HPS_E_INVALID, "path is NULL");
    FILE* fp = std::fopen(path, "r");
    if (!fp) throw Error(HPS_E_INVALID, std::string("cannot read ") + path);
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, k);
    std::fclose(fp);
    zgemm_tune_load(text);
  });
}

int hps_release_cached(void) {
  return guard([&] {
    HPS_HIP(hipDeviceSynchronize());
    ws_trim();
    drop_plans();
  });
}

int hps_set_allocator(hps_alloc_fn alloc, hps_free_fn free, void* ctx) {
  return guard([&] {
    if ((alloc == nullptr) != (free == nullptr))
      throw Error(HPS_E_INVALID, "allocator hook: alloc and free must both be set or both NULL");
    set_hook(alloc, free, ctx);
    if (alloc) {
      HPS_HIP(hipDeviceSynchronize());
      ws_trim();
    }
  });
}

int hps_estimate_bytes(const hps_domain* dom, int32_t p, const hps_opts* opts,
                       int64_t* build_peak, int64_t* resident) {
  return guard([&] {
    validate_domain(dom, p);
    if (!build_peak && !resident) throw Error(HPS_E_INVALID, "no output requested");
    hps_group f;
    if (opts) f.opts = *opts; else hps_default_opts(&f.opts);
    f.mixed = f.opts.precision == HPS_PREC_MIXED;
    f.p = p; f.m = p - 2; f.n = p * p - 4; f.nb = 4 * (p - 2); f.ni = (p - 2) * (p - 2);
    f.nx = dom->nx; f.ny = dom->ny;
    f.nprob = 1; f.nl1 = dom->nx * dom->ny; f.nleaf = f.nl1;
    make_plan(f);
    for (int l = 0; l < f.L; ++l) {
      f.lv[l].c64 = f.mixed;
      f.lv[l].inv64 = f.mixed && l < f.opts.fp64_top_levels;
    }
    size_t pk = 0, rs = 0;
    estimate_bytes(f, &pk, &rs);
    if (build_peak) *build_peak = (int64_t)pk;
    if (resident) *resident = (int64_t)rs;
  });
}

}  // extern "C"

// ------------------------------------------------------------------ serving hooks
namespace hps {

// Solve workspaces and staging come from a cache of device buffers (plain hipMalloc
// allocations, whose cost is a fraction of a millisecond; a stream-ordered pool that
// maps fresh multi-GB blocks took tens of milliseconds per call).  A buffer in use
// belongs to one call; when the call ends an event is recorded on its stream, and the
// next call that takes the buffer makes its own stream wait for that event, so reuse is
// ordered on the device across streams.  A call takes the smallest idle buffer that
// fits; when none fits, a buffer of the requested size is added, and the largest idle
// buffer of the device is released first only while the idle buffers hold more than
// kWsIdleCap (a release synchronizes the device, which would stall every stream).
// Workspace sizes are rounded up to eight steps per power of two, so that requests of
// similar size share buffers.  A failed allocation releases every idle buffer and
// retries.
namespace {
struct WsBuf {
  int dev = 0;
  void* p = nullptr;
  size_t cap = 0;
  bool busy = false;
  hipEvent_t ev = nullptr;
  bool recorded = false;
};
std::mutex g_ws_mu;
std::vector<WsBuf> g_ws;
constexpr size_t kWsGrain = size_t(2) << 20;
constexpr size_t kWsIdleCap = size_t(16) << 30;

void ws_release(WsBuf& b) {
  (void)hipFree(b.p);  // waits for the device, so pending uses of the buffer have ended
  if (b.ev) (void)hipEventDestroy(b.ev);
}
}  // namespace

namespace {
void* ws_take(size_t bytes, hipStream_t st, bool host_wait);
}  // namespace

void* ws_alloc(size_t bytes, hipStream_t st) { return ws_take(bytes, st, false); }

namespace {
// host_wait: the caller's work is not ordered on one stream, so a reused buffer's last
// use is waited for on the host
void* ws_take(size_t bytes, hipStream_t st, bool host_wait) {
  if (void* q = hook_alloc(bytes, host_wait ? nullptr : st)) return q;
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  bytes = (std::max<size_t>(bytes, 1) + kWsGrain - 1) / kWsGrain * kWsGrain;
  if (!host_wait) {
    // eight size steps per power of two (at most 1/8 over the request)
    int lg = 0;
    while ((size_t(1) << (lg + 1)) <= bytes) ++lg;
    const size_t q = lg > 3 ? size_t(1) << (lg - 3) : 1;
    bytes = (bytes + q - 1) / q * q;
  }
  std::unique_lock<std::mutex> lk(g_ws_mu);
  // best fit among the idle buffers.  A host-waited request is a long-lived buffer (a
  // factor's arena, a build's scratch): it takes none much larger than itself, so that a
  // small factor never holds a large buffer (the largest idle one is released instead)
  long best = -1, largest = -1;
  size_t idle = 0;
  for (size_t i = 0; i < g_ws.size(); ++i) {
    const WsBuf& b = g_ws[i];
    if (b.busy || b.dev != dev) continue;
    idle += b.cap;
    const bool fits = b.cap >= bytes && (!host_wait || b.cap <= bytes + bytes / 4 + kWsGrain);
    if (fits && (best < 0 || b.cap < g_ws[best].cap)) best = (long)i;
    if (largest < 0 || b.cap > g_ws[largest].cap) largest = (long)i;
  }
  if (best >= 0) {
    WsBuf& b = g_ws[best];
    b.busy = true;
    void* const ptr = b.p;
    if (b.recorded) {
      if (host_wait) {
        const hipEvent_t ev = b.ev;  // not destroyed while the buffer is busy
        lk.unlock();
        HPS_HIP(hipEventSynchronize(ev));
        return ptr;
      }
      HPS_HIP(hipStreamWaitEvent(st, b.ev, 0));
    }
    return ptr;
  }
  std::vector<WsBuf> drop;
  if (largest >= 0 && idle > kWsIdleCap) {
    drop.push_back(g_ws[largest]);
    g_ws.erase(g_ws.begin() + largest);
  }
  lk.unlock();
  for (auto& b : drop) ws_release(b);
  WsBuf nb;
  nb.dev = dev;
  nb.cap = bytes;
  hipError_t e = hipMalloc(&nb.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ws_trim();  // idle buffers of other sizes may be what stands in the way
    e = hipMalloc(&nb.p, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(HPS_E_NOMEM, "workspace allocation of " + std::to_string(bytes) +
                                 " bytes failed");
  }
  e = hipEventCreateWithFlags(&nb.ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipFree(nb.p);
    throw Error(HPS_E_DEVICE, "event creation failed");
  }
  nb.busy = true;
  lk.lock();
  g_ws.push_back(nb);
  return nb.p;
}
}  // namespace

void* ws_alloc_idle(size_t bytes) { return ws_take(bytes, nullptr, true); }

void ws_free_idle(void* p) {
  if (!p || hook_free(p, nullptr, true)) return;
  (void)hipDeviceSynchronize();  // every use of the buffer, on any stream, has ended
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto& b : g_ws)
    if (b.p == p) {
      b.recorded = false;
      b.busy = false;
      return;
    }
}

void ws_free(void* p, hipStream_t st) {
  if (!p || hook_free(p, st)) return;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto& b : g_ws)
    if (b.p == p) {
      b.recorded = hipEventRecord(b.ev, st) == hipSuccess;
      if (!b.recorded) (void)hipGetLastError();
      b.busy = false;
      return;
    }
}

void ws_trim() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::vector<WsBuf> drop;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (size_t i = 0; i < g_ws.size();) {
      if (!g_ws[i].busy && g_ws[i].dev == dev) {
        drop.push_back(g_ws[i]);
        g_ws.erase(g_ws.begin() + (long)i);
      } else {
        ++i;
      }
    }
  }
  for (auto& b : drop) ws_release(b);
}

// ------------------------------------------------------------------ allocator hook
namespace {
struct Hook {
  hps_alloc_fn alloc = nullptr;
  hps_free_fn free = nullptr;
  void* ctx = nullptr;
};
std::mutex g_hook_mu;
Hook g_hook;                               // installed hook (alloc == nullptr: none)
std::unordered_map<void*, Hook> g_hooked;  // live memory from a hook, and which one
}  // namespace

void set_hook(hps_alloc_fn alloc, hps_free_fn free, void* ctx) {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  g_hook = Hook{alloc, free, alloc ? ctx : nullptr};
}

void* hook_alloc(size_t bytes, hipStream_t st) {
  Hook h;
  {
    std::lock_guard<std::mutex> lk(g_hook_mu);
    h = g_hook;
  }
  if (!h.alloc) return nullptr;
  void* p = h.alloc(std::max<size_t>(bytes, 1), st, h.ctx);
  if (!p)
    throw Error(HPS_E_NOMEM, "allocator hook returned no memory for " + std::to_string(bytes) +
                                 " bytes");
  std::lock_guard<std::mutex> lk(g_hook_mu);
  g_hooked[p] = h;
  return p;
}

bool hook_free(void* p, hipStream_t st, bool sync_device) {
  Hook h;
  {
    std::lock_guard<std::mutex> lk(g_hook_mu);
    auto it = g_hooked.find(p);
    if (it == g_hooked.end()) return false;
    h = it->second;
    g_hooked.erase(it);
  }
  if (sync_device) (void)hipDeviceSynchronize();
  h.free(p, st, h.ctx);
  return true;
}

void* dev_alloc(size_t bytes) {
  if (void* q = hook_alloc(bytes, nullptr)) return q;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 1));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ws_trim();  // idle cached buffers may be what stands in the way
    e = hipMalloc(&p, std::max<size_t>(bytes, 1));
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(e == hipErrorOutOfMemory ? HPS_E_NOMEM : HPS_E_DEVICE,
                "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void dev_free(void* p) {
  if (p && !hook_free(p, nullptr, true)) (void)hipFree(p);
}

void set_last_error(const std::string& msg) { g_err = msg; }

size_t solve_workspace_bytes(hps_factor* f, int nrhs, bool with_s) {
  hps_group& G = *f->g;
  // the sizing pass never dereferences the vectors: placeholders stand in for them
  const double* ph = reinterpret_cast<const double*>(4096);
  size_t bytes = 0;
  hps_solve_info info{};
  solve_impl(G, f->b0, 1, nrhs, with_s ? ph : nullptr, ph, nullptr, const_cast<double*>(ph),
             nullptr, &info, &bytes);
  return bytes;
}

void solve_on(hps_factor* f, int nrhs, const double* s, const double* t, double* u,
              hipStream_t st, hps_solve_info* info) {
  solve_impl(*f->g, f->b0, 1, nrhs, s, t, nullptr, u, st, info);
}

bool solve_shareable(const hps_factor* a, const hps_factor* b) {
  return shareable(*a->g, *b->g);
}

int solve_share_max() { return Across::kMax; }

void solve_parts(const std::vector<SolvePart>& parts, hipStream_t st, size_t* bytes) {
  solve_across(parts, st, bytes);
}

}  // namespace hps
