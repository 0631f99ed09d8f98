// Leaf stage (Sec. 2.1, 2.1.1, 2.1.2): for every leaf, the operators Psi (n x n_b) and
// Y (n x n_i) with B [Psi | Y] = I, and the ItI operator R = G Psi.
//
// With u = [u_b; u_i], B = [[F_bb, F_bi], [A_ib, A_ii]] (F = N + i eta E_b restricted to
// the boundary / interior columns, A = Ahat(I_i, :)).  The boundary unknowns are
// eliminated through the impedance rows, which keeps every step as well conditioned as
// B itself (Re eta != 0): the interior Dirichlet block A_ii alone is singular whenever
// kappa^2 c meets an eigenvalue of the leaf's Dirichlet Laplacian, which happens for
// leaves of a few wavelengths.  Derived from eqs. (homogeneous) and (particular):
//   u_b = F_bb^{-1} (f - F_bi u_i),   S_i u_i = s - A_ib F_bb^{-1} f,
//   S_i = A_ii - A_ib F_bb^{-1} F_bi,
//   Y_i = S_i^{-1},  Psi_i = -Y_i W  (W = A_ib F_bb^{-1}),
//   [Psi_b | Y_b] = [F_bb^{-1} | 0] - F_bb^{-1} F_bi [Psi_i | Y_i],
//   R = G Psi = I - 2 i eta Psi_b      (G = F - 2 i eta E_b and F Psi = I).
// F_bb couples only the two end nodes of each grid line (S_i with N_i, W_j with E_j),
// so F_bb^{-1} is a set of 2 x 2 inverses, F_bb^{-1} F_bi mixes the interior nodes of
// one grid line, and S_i = -(G_x (x) I) - (I (x) G_y) - kappa^2 diag(c) has the
// sparsity of the Laplacian with complex line operators G_x, G_y.  These line tables
// depend only on p, the leaf size and eta; the host builds them (LeafDesc::tab).
//
// Kernels: leaf_sinv (S_i^{-1} by blocked Gauss-Jordan with partial pivoting, the
// matrix held in registers (partly in a scratch copy for p >= 15), one workgroup per
// leaf), leaf_psi_bnd (Psi_i, the boundary rows of [Psi | Y] and R, in one pass over
// Y_i; for reduced-precision storage it writes the complex64 copy of the whole
// [Psi | Y]).
#include "kernels.hpp"

namespace hps {
namespace {

__host__ __device__ constexpr int leaf_table_len_dev(int p) {
  return 2 * (p - 2) * (p - 2) + 8 * (p - 2) + 8;
}

// offsets (complex entries) into the line table of LeafDesc::tab, m = p - 2
struct TabIdx {
  int m;
  __host__ __device__ int gx() const { return 0; }
  __host__ __device__ int gy() const { return m * m; }
  __host__ __device__ int sS() const { return 2 * m * m; }
  __host__ __device__ int sN() const { return 2 * m * m + m; }
  __host__ __device__ int oW() const { return 2 * m * m + 2 * m; }
  __host__ __device__ int oE() const { return 2 * m * m + 3 * m; }
  __host__ __device__ int wS() const { return 2 * m * m + 4 * m; }
  __host__ __device__ int wN() const { return 2 * m * m + 5 * m; }
  __host__ __device__ int wW() const { return 2 * m * m + 6 * m; }
  __host__ __device__ int wE() const { return 2 * m * m + 7 * m; }
  __host__ __device__ int by() const { return 2 * m * m + 8 * m; }
  __host__ __device__ int bx() const { return 2 * m * m + 8 * m + 4; }
};

// Thread grid GR x GC per leaf, each thread owning ER x EC complex entries of S_i
// (padded): rows tr + GR a, columns tc + GC b.  Rows a < AR of a thread's entries stay
// in registers for the whole inversion; the rows a >= AR (p >= 15, where the complex
// matrix outgrows the register file of a compute unit) live in a per-leaf scratch copy
// between block steps, in a thread-private interleaved layout.  Pivots are taken in
// blocks of NBK.
template <int P> struct LeafCfg {
  static constexpr int m = P - 2;
  static constexpr int NI = m * m;
  static constexpr int ER = P <= 7 ? 1 : P <= 10 ? 2 : P == 11 ? 3 : P <= 13 ? 4
                          : P == 14 ? 8 : P == 15 ? 9 : 10;
  static constexpr int EC = P <= 7 ? 1 : P <= 9 ? 2 : P == 10 ? 4 : P == 11 ? 3
                          : P <= 13 ? 4 : P == 14 ? 6 : P == 15 ? 7 : 8;
  static constexpr int AR = P <= 14 ? ER : 6;  // register-resident rows
  static constexpr int GR = (NI + ER - 1) / ER;
  static constexpr int GC = (NI + EC - 1) / EC;
  static constexpr int GE = (GC * EC > GR * ER ? GC * EC : GR * ER);  // LDS row stride
  static constexpr int NLIVE = GR * GC;                     // threads that own entries
  static constexpr int NT = ((NLIVE + 63) / 64) * 64;       // whole waves (shuffles)
  static constexpr int NBK = P >= 14 ? 16 : 8;              // pivots per block
  static constexpr int POOL = 2 * NBK * GE;                 // panel / Q, pivot rows X
  static constexpr int CW = (POOL / NI) < NI ? (POOL / NI) : NI;  // output chunk columns
  static constexpr long SCR = (long)(ER - AR) * EC * NT;    // scratch entries per leaf
  static_assert(NT <= 1024 && NT >= NI, "one thread per panel row, at most 1024");
  static_assert(GR * ER >= NI && GC * EC >= NI && CW >= 1, "bad leaf grid");
};

// S_i^{-1} by blocked Gauss-Jordan with partial pivoting.  Per block K of NBK pivot
// columns:
//   1. owners publish the panel columns M[:, K] to LDS;
//   2. the workgroup runs the NBK elimination steps on the panel in place (pivot =
//      largest unused |re| + |im|), giving the block transformation Q and the pivot
//      rows P_K;
//   3. owners of the pivot rows publish X = M[P_K, :];
//   4. every entry outside K becomes (pivot rows zeroed) + Q X, entries in K become Q.
// This is the same in-place elimination as column-at-a-time Gauss-Jordan (the block
// step applies the product of the NBK elementary transformations at once); the
// in-place result M satisfies S^{-1}[k][piv[j]] = M[piv[k]][j].  The inverse goes to
// the Y_i block of [Psi | Y].  Every thread only ever reads and writes its own entries
// in the scratch copy, so no cross-thread ordering is involved there.
template <int P>
__global__ __launch_bounds__(LeafCfg<P>::NT) void leaf_sinv_kernel(LeafDesc d) {
  using Cfg = LeafCfg<P>;
  constexpr int m = Cfg::m, NI = Cfg::NI, ER = Cfg::ER, EC = Cfg::EC, GR = Cfg::GR,
                GC = Cfg::GC, GE = Cfg::GE, AR = Cfg::AR;
  constexpr int NBK = Cfg::NBK;
  constexpr int NB = 4 * m, N = P * P - 4;
  __shared__ double2 pool[Cfg::POOL];
  __shared__ int piv[NI], ipiv[NI];
  __shared__ int slot[NI];          // position of a row in the current block's pivots, or -1
  __shared__ int used_s[NI];
  __shared__ double2 sG[2][m * m];  // G_x, G_y
  __shared__ int s_bad;
  __shared__ unsigned long long cand[2][LeafCfg<P>::NT / 64];  // per-wave pivot candidates
  double2* pan = pool;               // [NBK][GE]  panel, then the block transformation Q
  double2* Xs = pool + NBK * GE;     // [NBK][GE]  pivot rows

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const bool live = tid < Cfg::NLIVE;  // padding threads own nothing and publish nothing
  const int tr = tid % GR, tc = tid / GR;
  const long h = blockIdx.x;
  const int g = d.leaf_grid[h];
  const long prob = (d.h0 + h) / d.nl1;
  if (d.route && d.route[prob]) return;  // this problem takes the Dirichlet-block route
  const double2* tab = reinterpret_cast<const double2*>(d.tab) + prob * leaf_table_len_dev(P);
  for (int e = tid; e < m * m; e += Cfg::NT) {
    sG[0][e] = tab[TabIdx{m}.gx() + e];
    sG[1][e] = tab[TabIdx{m}.gy() + e];
  }
  for (int i = tid; i < NI; i += Cfg::NT) {
    slot[i] = -1;
    used_s[i] = 0;
  }
  for (int e = tid; e < Cfg::POOL; e += Cfg::NT) pool[e] = cmk(0, 0);
  if (tid == 0) s_bad = 0;
  __syncthreads();
  const double kap = d.prm[4 * prob];
  const double k2 = kap * kap;
  const double* cl = d.c + (long)g * NI;
  double2* Mg = reinterpret_cast<double2*>(d.Mg) + (AR < ER ? h * Cfg::SCR : 0);
  // scratch slot of this thread's entry (a >= AR, b): consecutive threads, consecutive
  // slots
  auto gaddr = [&](int a, int b) { return Mg + ((long)((a - AR) * EC + b) * Cfg::NT + tid); };

  // assemble S_i = -(G_x (x) I) - (I (x) G_y) - kappa^2 diag(c) on the interior nodes
  // (node r = (j-1) m + (i-1); G_x acts along x within a grid row, G_y along y)
  double2 M[AR][EC];
#pragma unroll
  for (int a = 0; a < ER; ++a) {
    const int r = tr + GR * a;
    const int ir = r % m, jr = r / m;
    const double cr = (live && r < NI) ? cl[r] : 0.0;
#pragma unroll
    for (int b = 0; b < EC; ++b) {
      const int c = tc + GC * b;
      double2 v = cmk(0, 0);
      if (live && r < NI && c < NI) {
        const int ic = c % m, jc = c / m;
        if (jr == jc) v = csub(v, sG[0][ir + m * ic]);
        if (ir == ic) v = csub(v, sG[1][jr + m * jc]);
        if (r == c) v.x -= k2 * cr;
      }
      if (a < AR) M[a < AR ? a : 0][b] = v;
      else if (live) *gaddr(a, b) = v;
    }
  }
  // visit the owned entries (a, b) that want(a, b) selects, with their values: register
  // rows unrolled, scratch rows one at a time (only the selected entries are loaded)
  auto for_entries = [&](auto&& want, auto&& fn) {
#pragma unroll
    for (int a = 0; a < AR; ++a)
#pragma unroll
      for (int b = 0; b < EC; ++b)
        if (want(a, b)) fn(a, b, M[a][b]);
#pragma unroll 1
    for (int a = AR; a < ER; ++a)
#pragma unroll
      for (int b = 0; b < EC; ++b)
        if (want(a, b)) fn(a, b, *gaddr(a, b));
  };

#pragma unroll 1
  for (int k0 = 0; k0 < NI; k0 += NBK) {
    const int nk = (NI - k0) < NBK ? (NI - k0) : NBK;
    // 1. panel columns
    if (live)
      for_entries(
          [&](int a, int b) {
            const int j = tc + GC * b - k0;
            return tr + GR * a < NI && j >= 0 && j < nk;
          },
          [&](int a, int b, double2 v) { pan[(tc + GC * b - k0) * GE + tr + GR * a] = v; });
    __syncthreads();
    // 2. elimination on the panel, in place, by the whole workgroup: thread i owns
    //    panel row i.  A pivot row is left unscaled during the block (its thread keeps
    //    the pending factor 1/pivot and applies it after the block's steps), so the
    //    other rows are updated from it while nothing writes it: one barrier per step,
    //    after every wave has offered its pivot candidate (double-buffered, so a wave
    //    that runs ahead does not overwrite candidates still being read).
    if (tid == 0 && k0 > 0)
      for (int s = 0; s < NBK; ++s) slot[piv[k0 - NBK + s]] = -1;
    bool mine_free = tid < NI && !used_s[tid < NI ? tid : 0];
    double2 pend = cmk(1.0, 0.0);   // pending scale of this thread's row
    bool pivoted = false;            // this row is a pivot row of this block
    int fix_s = -1;                  // column whose entry of this row is still to be set to 1
    double2 nextv = tid < NI ? pan[tid] : cmk(0, 0);  // this row's entry in column s
#pragma unroll 1
    for (int s = 0; s < nk; ++s) {
      const double mag = mine_free ? cabs1(nextv) : -1.0;
      // wave candidate: magnitude compared in single precision, ties to the lowest row
      const unsigned key = mag > 0.0 ? max(__float_as_uint((float)mag), 1u) : 0u;
      const unsigned wbest = wave_max_u32(key);
      const unsigned long long hit = __ballot(key == wbest && wbest != 0u);
      if (lane == 0) {
        const int wr = hit ? wave * 64 + __builtin_ctzll(hit) : 0;
        cand[s & 1][wave] = ((unsigned long long)wbest << 32) | (0xffffffffu - (unsigned)wr);
      }
      __syncthreads();
      unsigned long long bestc = 0;
#pragma unroll
      for (int w = 0; w < Cfg::NT / 64; ++w) bestc = cand[s & 1][w] > bestc ? cand[s & 1][w] : bestc;
      if ((bestc >> 32) == 0) {  // no nonzero candidate in this column: singular
        if (tid == 0) s_bad = k0 + s + 1;
        break;
      }
      const int r = (int)(0xffffffffu - (unsigned)(bestc & 0xffffffffu));
      const double2 ip = crcp_pivot(pan[s * GE + r]);
      // the entry of an earlier pivot row in its pivot column becomes 1 (1/pivot once
      // the pending factor is applied); written only now, after every thread has read
      // the pivot value in that row's own step
      if (fix_s >= 0) {
        pan[fix_s * GE + tid] = cmk(1.0, 0.0);
        fix_s = -1;
      }
      if (tid == r) {
        pend = ip;
        pivoted = true;
        fix_s = s;
        mine_free = false;
        piv[k0 + s] = r;
        slot[r] = s;
        used_s[r] = 1;
        if (s + 1 < nk) nextv = pan[(s + 1) * GE + tid];  // not updated in this step
      } else if (tid < NI) {
        const double2 f = cmul(nextv, ip);
        // the next column's values are loaded before this one is stored (the pivot row
        // is not written in this phase, and this row only by this thread).  All NBK
        // columns are swept; in a last, narrower block the columns from nk on hold
        // leftovers that nothing reads.
        double2 a_cur = pan[tid], p_cur = pan[r];
#pragma unroll
        for (int j = 0; j < NBK; ++j) {
          double2 a_nxt = a_cur, p_nxt = p_cur;
          if (j + 1 < NBK) {
            a_nxt = pan[(j + 1) * GE + tid];
            p_nxt = pan[(j + 1) * GE + r];
          }
          const double2 v = (j == s) ? cmk(-f.x, -f.y) : csub(a_cur, cmul(f, p_cur));
          pan[j * GE + tid] = v;
          if (j == s + 1) nextv = v;
          a_cur = a_nxt;
          p_cur = p_nxt;
        }
      }
    }
    __syncthreads();
    if (s_bad) break;
    // pending scales of this block's pivot rows (read by the update after the next
    // barrier)
    if (pivoted) {
      if (fix_s >= 0) pan[fix_s * GE + tid] = cmk(1.0, 0.0);
#pragma unroll
      for (int j = 0; j < NBK; ++j)
        if (j < nk) pan[j * GE + tid] = cmul(pan[j * GE + tid], pend);
    }
    // 3. pivot rows (values before this block's update); on the panel columns X is the
    //    identity, so that the update below writes Q there
    if (live)
      for_entries(
          [&](int a, int b) {
            const int ra = tr + GR * a;
            return ra < NI && tc + GC * b < NI && slot[ra] >= 0;
          },
          [&](int a, int b, double2 v) {
            const int sl = slot[tr + GR * a];
            const int j = tc + GC * b - k0;
            Xs[sl * GE + tc + GC * b] = (j >= 0 && j < nk) ? cmk(j == sl ? 1.0 : 0.0, 0.0) : v;
          });
    __syncthreads();
    // 4. block update: M <- (M with pivot rows and panel columns zeroed) + Q X
    if (live) {
      // a scratch row's entries, pivot rows and panel columns zeroed
      auto load_row = [&](int a, double2* row) {
        const int ra = tr + GR * a;
        const bool isP = ra < NI && slot[ra] >= 0;
#pragma unroll
        for (int b = 0; b < EC; ++b) {
          const int c = tc + GC * b;
          const int j = c - k0;
          const bool inK = j >= 0 && j < nk;
          row[b] = (ra >= NI || c >= NI || isP || inK) ? cmk(0, 0) : *gaddr(a, b);
        }
      };
      double2 row[EC];
      // register rows: each pivot's X values are loaded once for all of them
#pragma unroll
      for (int a = 0; a < AR; ++a) {
        const int ra = tr + GR * a;
        const bool isP = ra < NI && slot[ra] >= 0;
#pragma unroll
        for (int b = 0; b < EC; ++b) {
          const int j = tc + GC * b - k0;
          const bool inK = j >= 0 && j < nk;
          M[a][b] = (isP || inK) ? cmk(0, 0) : M[a][b];
        }
      }
      const double2* qb = pan + tr;
      const double2* xbp = Xs + tc;
#pragma unroll 1
      for (int j = 0; j < nk; ++j) {
        double2 xb[EC];
#pragma unroll
        for (int b = 0; b < EC; ++b) xb[b] = xbp[j * GE + GC * b];
#pragma unroll
        for (int a = 0; a < AR; ++a) {
          const double2 qa = qb[j * GE + GR * a];
#pragma unroll
          for (int b = 0; b < EC; ++b) M[a][b] = cfma(qa, xb[b], M[a][b]);
        }
      }
      // scratch rows, one at a time: update with all nk pivots, store
#pragma unroll 1
      for (int a = AR; a < ER; ++a) {
        const int ra = tr + GR * a;
        load_row(a, row);
        if (ra < NI) {
#pragma unroll 1
          for (int j = 0; j < nk; ++j) {
            const double2 qa = pan[j * GE + ra];
#pragma unroll
            for (int b = 0; b < EC; ++b) row[b] = cfma(qa, Xs[j * GE + tc + GC * b], row[b]);
          }
#pragma unroll
          for (int b = 0; b < EC; ++b) *gaddr(a, b) = row[b];
        }
      }
    }
    __syncthreads();  // Q and X are read above; the next block overwrites them
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) d.info[h] = s_bad;
    return;
  }
  for (int k = tid; k < NI; k += Cfg::NT) ipiv[piv[k]] = k;
  __syncthreads();
  // write S^{-1}[k][piv[c]] = M[piv[k]][c]:  entry (row ri, col c) goes to
  // (ipiv[ri], piv[c]); stage column chunks in LDS for coalesced stores into the Y_i
  // block of [Psi | Y].
  double2* BI = reinterpret_cast<double2*>(d.BI) + h * (long)N * N;
  for (int c0 = 0; c0 < NI; c0 += Cfg::CW) {
    const int cw = (NI - c0) < Cfg::CW ? (NI - c0) : Cfg::CW;
    if (live)
      for_entries(
          [&](int a, int b) {
            const int c = tc + GC * b;
            return tr + GR * a < NI && c < NI && piv[c] - c0 >= 0 && piv[c] - c0 < cw;
          },
          [&](int a, int b, double2 v) {
            pool[ipiv[tr + GR * a] + NI * (piv[tc + GC * b] - c0)] = v;
          });
    __syncthreads();
    for (int e = tid; e < NI * cw; e += Cfg::NT) {
      const int row = e % NI, col = e / NI;
      BI[(NB + row) + (long)N * (NB + c0 + col)] = pool[e];
    }
    __syncthreads();
  }
}

// One entry of the boundary rows [Psi_b | Y_b] = [F_bb^{-1} | 0] - F_bb^{-1} F_bi
// [Psi_i | Y_i] in column gcol, from that column's interior rows (col, LDS): the row of
// S_t combines the interior rows of grid column t with sS, N_t with sN, the rows of
// E_t / W_t combine grid row t with oE / oW; the 2 x 2 inverses of F_bb sit on the
// boundary columns.
template <int P>
__device__ inline double2 bnd_entry(int b, int gcol, const double2* col, const double2 (*sc)[P - 2],
                                    const double2* sb) {
  constexpr int m = P - 2;
  const int side = b / m, t = b % m;  // 0 S, 1 E, 2 N, 3 W
  double2 acc = cmk(0, 0);
  double2 base = cmk(0, 0);
  if (side == 0 || side == 2) {       // grid column t: interior rows (t, l)
    const double2* co = sc[side == 0 ? 0 : 1];
#pragma unroll
    for (int l = 0; l < m; ++l) acc = cfma(co[l], col[l * m + t], acc);
    const int rs = (side == 0) ? 0 : 2;          // b11 b12 | b21 b22
    if (gcol == t) base = sb[rs];                // column S_t
    else if (gcol == 2 * m + t) base = sb[rs + 1];  // column N_t
  } else {                            // grid row t: interior rows (k, t)
    const double2* co = sc[side == 3 ? 2 : 3];
#pragma unroll
    for (int k = 0; k < m; ++k) acc = cfma(co[k], col[t * m + k], acc);
    const int rs = (side == 3) ? 4 : 6;          // c11 c12 | c21 c22
    if (gcol == 3 * m + t) base = sb[rs];        // column W_t
    else if (gcol == m + t) base = sb[rs + 1];   // column E_t
  }
  return csub(base, acc);
}

// Psi_i = -Y_i W (W = A_ib F_bb^{-1}), the boundary rows of [Psi | Y] and R = I - 2 i eta
// Psi_b, in one pass over Y_i.  Row (i, j) of W has four entries, in the columns of S_i
// (wS[j]), N_i (wN[j]), W_j (wW[i]) and E_j (wE[i]).  Y_i is read by grid rows: chunk k
// stages the m columns of the interior nodes (i, k) in LDS, which completes the columns
// W_k and E_k of Psi_i (one thread per interior row) and adds the chunk's terms to the
// row's m S and m N entries (registers); the chunk's columns of Y, W_k and E_k then get
// their boundary rows.  The S and N columns get theirs after the last chunk.  Each
// interior row has two threads: one in the first half of the workgroup (the S columns
// and W_k), one in the second (the N columns and E_k), which halves the accumulators a
// thread holds so that two workgroups share a compute unit.  For reduced-precision
// storage every entry goes to the complex64 copy only.
template <int P>
__global__ __launch_bounds__(512) void leaf_psi_bnd_kernel(LeafDesc d) {
  constexpr int NT = 512;
  constexpr int m = P - 2, NI = m * m, NB = 4 * m, N = P * P - 4;
  constexpr int CC = m + 2;  // staged columns: a chunk of Y_i plus W_k and E_k of Psi_i
  static_assert(NI <= NT / 2, "two threads per interior row");
  __shared__ double2 sI[CC][NI];
  __shared__ double2 sw[4][m];  // wS wN wW wE
  __shared__ double2 sc[4][m];  // sS sN oW oE
  __shared__ double2 sb[8];
  const int tid = threadIdx.x;
  const long h = blockIdx.x;
  const long prob = (d.h0 + h) / d.nl1;
  if (d.route && d.route[prob]) return;  // this problem takes the Dirichlet-block route
  const double2* tab = reinterpret_cast<const double2*>(d.tab) + prob * leaf_table_len_dev(P);
  const TabIdx T{m};
  for (int e = tid; e < m; e += NT) {
    sw[0][e] = tab[T.wS() + e];
    sw[1][e] = tab[T.wN() + e];
    sw[2][e] = tab[T.wW() + e];
    sw[3][e] = tab[T.wE() + e];
    sc[0][e] = tab[T.sS() + e];
    sc[1][e] = tab[T.sN() + e];
    sc[2][e] = tab[T.oW() + e];
    sc[3][e] = tab[T.oE() + e];
  }
  if (tid < 4) {
    sb[tid] = tab[T.by() + tid];      // (S, N) pair: b11 b12 b21 b22
    sb[4 + tid] = tab[T.bx() + tid];  // (W, E) pair: c11 c12 c21 c22
  }
  double2* BI = reinterpret_cast<double2*>(d.BI) + h * (long)N * N;
  float2* B32 = d.BI32 ? reinterpret_cast<float2*>(d.BI32) + h * (long)N * N : nullptr;
  double2* R = reinterpret_cast<double2*>(d.R) + h * (long)NB * NB;
  // -2 i eta = (2 eta_im, -2 eta_re)
  const double2 m2ie = cmk(2.0 * d.prm[4 * prob + 2], -2.0 * d.prm[4 * prob + 1]);
  auto put = [&](int row, int gcol, double2 v) {
    if (B32) B32[row + (long)N * gcol] = make_float2((float)v.x, (float)v.y);
    else BI[row + (long)N * gcol] = v;
  };
  // boundary rows (and R) of the ncol staged columns sI[0..ncol), global columns gc(col)
  auto boundary = [&](int ncol, auto&& gc) {
    for (int e = tid; e < NB * ncol; e += NT) {
      const int b = e % NB, col = e / NB;
      const int gcol = gc(col);
      const double2 v = bnd_entry<P>(b, gcol, sI[col], sc, sb);
      put(b, gcol, v);
      if (gcol < NB) {
        double2 rv = cmul(m2ie, v);
        if (gcol == b) rv.x += 1.0;
        R[b + (long)NB * gcol] = rv;
      }
    }
  };
  const int r = tid % (NT / 2), hh = tid / (NT / 2);  // row; 0: S and W, 1: N and E
  double2 acc[m];
#pragma unroll
  for (int i = 0; i < m; ++i) acc[i] = cmk(0, 0);
  // chunk k's columns of Y_i: IT entries per thread, loaded together; the next chunk's
  // loads are issued as soon as this chunk is in LDS
  constexpr int IT = (NI * m + NT - 1) / NT;
  double2 yv[IT];
  auto load_chunk = [&](int k) {
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = tid + NT * q;
      yv[q] = e < NI * m ? BI[(NB + e % NI) + (long)N * (NB + k * m + e / NI)] : cmk(0, 0);
    }
  };
  load_chunk(0);
#pragma unroll 1
  for (int k = 0; k < m; ++k) {
    __syncthreads();  // the tables; the previous chunk's boundary rows are done
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = tid + NT * q;
      if (e < NI * m) {
        const int row = e % NI, i = e / NI;
        sI[i][row] = yv[q];
        if (B32)
          B32[(NB + row) + (long)N * (NB + k * m + i)] = make_float2((float)yv[q].x, (float)yv[q].y);
      }
    }
    if (k + 1 < m) load_chunk(k + 1);
    __syncthreads();
    if (r < NI) {
      // hh 0: S entries (weight wS[k]) and W_k (weights wW); hh 1: N and E_k
      const double2 wk = sw[hh][k];
      double2 a = cmk(0, 0);
#pragma unroll
      for (int i = 0; i < m; ++i) {
        const double2 y = sI[i][r];
        acc[i] = cfma(y, wk, acc[i]);
        a = cfma(y, sw[2 + hh][i], a);
      }
      const double2 pv = cmk(-a.x, -a.y);
      sI[m + hh][r] = pv;
      put(NB + r, hh ? m + k : 3 * m + k, pv);  // E_k or W_k
    }
    __syncthreads();
    boundary(CC, [&](int col) { return col < m ? NB + k * m + col : col == m ? 3 * m + k : m + k; });
  }
  // the S columns (q = 0, global column i) and N columns (q = 1, column 2m + i)
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    __syncthreads();
    if (r < NI && hh == q) {
#pragma unroll
      for (int i = 0; i < m; ++i) {
        const double2 v = cmk(-acc[i].x, -acc[i].y);
        sI[i][r] = v;
        put(NB + r, q * 2 * m + i, v);
      }
    }
    __syncthreads();
    boundary(m, [&](int col) { return q * 2 * m + col; });
  }
}

template <int P> void launch_sinv(const LeafDesc& d, hipStream_t st) {
  if (LeafCfg<P>::SCR > 0 && !d.Mg) throw Error(1, "leaf: scratch copy of S_i missing");
  hipLaunchKernelGGL(leaf_sinv_kernel<P>, dim3(d.nleaf), dim3(LeafCfg<P>::NT), 0, st, d);
}
template <int P> void scratch_of(long nleaf, size_t* out) {
  *out = (size_t)nleaf * LeafCfg<P>::SCR * 16;
}
template <int P> void launch_psi_bnd(const LeafDesc& d, hipStream_t st) {
  hipLaunchKernelGGL(leaf_psi_bnd_kernel<P>, dim3(d.nleaf), dim3(512), 0, st, d);
}

#define HPS_P_SWITCH(FN, p, ...)                   \
  switch (p) {                                     \
    case 4: FN<4>(__VA_ARGS__); break;             \
    case 5: FN<5>(__VA_ARGS__); break;             \
    case 6: FN<6>(__VA_ARGS__); break;             \
    case 7: FN<7>(__VA_ARGS__); break;             \
    case 8: FN<8>(__VA_ARGS__); break;             \
    case 9: FN<9>(__VA_ARGS__); break;             \
    case 10: FN<10>(__VA_ARGS__); break;           \
    case 11: FN<11>(__VA_ARGS__); break;           \
    case 12: FN<12>(__VA_ARGS__); break;           \
    case 13: FN<13>(__VA_ARGS__); break;           \
    case 14: FN<14>(__VA_ARGS__); break;           \
    case 15: FN<15>(__VA_ARGS__); break;           \
    case 16: FN<16>(__VA_ARGS__); break;           \
    default: throw Error(1, "unsupported p (4..16)"); \
  }

}  // namespace

size_t leaf_scratch_bytes(int p, long nleaf) {
  size_t b = 0;
  HPS_P_SWITCH(scratch_of, p, nleaf, &b);
  return b;
}

int leaf_table_len(int p) { return leaf_table_len_dev(p); }

void leaf_interior_inverse(const LeafDesc& d, hipStream_t st) {
  if (d.nleaf <= 0) return;
  HPS_P_SWITCH(launch_sinv, d.p, d, st);
  HPS_LAUNCH_CHECK();
}

void leaf_psi_and_boundary(const LeafDesc& d, hipStream_t st) {
  if (d.nleaf <= 0) return;
  HPS_P_SWITCH(launch_psi_bnd, d.p, d, st);
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
