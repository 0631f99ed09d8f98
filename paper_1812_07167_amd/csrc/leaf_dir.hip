// Leaf stage through the interior Dirichlet block (Sec. 2.1, 2.1.1, 2.1.2), for leaves
// whose interior collocation block is safely invertible.
//
// With u = [u_b; u_i] the leaf matrix is B = [[F_bb, N_i], [A_ib, A]] (impedance rows
// F = N + i eta E_b, then the interior collocation rows Ahat(I_i, :) = [A_ib, A]).  For
// real c the interior block A = -(I (x) L_x) - (L_y (x) I) - kappa^2 diag(c) is real
// (L_x, L_y the interior parts of the second-derivative matrices).  Eliminating the
// interior unknowns first (block elimination of eqs. (homogeneous), (particular)):
//   X = A^{-1} A_ib,  Z = N_i A^{-1},  S = F_bb - N_i X   (n_b x n_b, complex),
//   Psi_b = S^{-1},  Psi_i = -X S^{-1},  Y_b = -S^{-1} Z,  Y_i = A^{-1} - X Y_b,
//   R = G Psi = I - 2 i eta Psi_b   (G = F - 2 i eta E_b and F Psi = I).
// A^{-1} is real, so the O(n_i^3) inversion runs in real arithmetic (a quarter of the
// complex one).  A is safe to invert when kappa^2 c stays below half the smallest
// eigenvalue pi^2 (1/h_x^2 + 1/h_y^2) of the leaf's Dirichlet Laplacian (then
// -Lap - kappa^2 c is coercive on the leaf); the host takes this route per problem
// only then (leaf_route), and the impedance route of leaf.hip otherwise.
//
// Kernels: leaf_cmax (largest c of each problem, for that test), leaf_ainv (A^{-1} by
// blocked Gauss-Jordan with partial pivoting in registers, into a compact real scratch
// copy), leaf_xz (X, Z and S from A^{-1}, S into the Psi_b block), leaf_dir_R
// (R from Psi_b once S is inverted).  S^{-1} and the three products run on the shared
// inversion and GEMM kernels (api.hip).
#include <cstring>

#include "kernels.hpp"

namespace hps {
namespace {

// offsets (doubles) into the real line table of a problem, m = p - 2, indices 1..p-2
// of the interior points:
//   Lx, Ly  [m*m]  interior parts of D_xx, D_yy (column-major)
//   aS, aN  [m]    -D_yy(j, 0), -D_yy(j, p-1): A_ib couples (i, j) to S_i, N_i
//   aW, aE  [m]    -D_xx(i, 0), -D_xx(i, p-1): A_ib couples (i, j) to W_j, E_j
//   nS, nN  [m]    -D_y(0, j), D_y(p-1, j): N_i rows of S_i, N_i on nodes (i, j)
//   nW, nE  [m]    -D_x(0, i), D_x(p-1, i): N_i rows of W_j, E_j on nodes (i, j)
//   fy      [4]    N_bb on (S_i, N_i): rows S, N x columns S, N
//   fx      [4]    N_bb on (W_j, E_j): rows W, E x columns W, E
struct RIdx {
  int m;
  __host__ __device__ int lx() const { return 0; }
  __host__ __device__ int ly() const { return m * m; }
  __host__ __device__ int aS() const { return 2 * m * m; }
  __host__ __device__ int aN() const { return 2 * m * m + m; }
  __host__ __device__ int aW() const { return 2 * m * m + 2 * m; }
  __host__ __device__ int aE() const { return 2 * m * m + 3 * m; }
  __host__ __device__ int nS() const { return 2 * m * m + 4 * m; }
  __host__ __device__ int nN() const { return 2 * m * m + 5 * m; }
  __host__ __device__ int nW() const { return 2 * m * m + 6 * m; }
  __host__ __device__ int nE() const { return 2 * m * m + 7 * m; }
  __host__ __device__ int fy() const { return 2 * m * m + 8 * m; }
  __host__ __device__ int fx() const { return 2 * m * m + 8 * m + 4; }
  __host__ __device__ int len() const { return 2 * m * m + 8 * m + 8; }
};

// ------------------------------------------------------------------ largest c per problem
// Order-preserving map of doubles to unsigned integers (NaN is taken as +infinity), so
// that an integer atomic max finds the largest c.
__device__ inline unsigned long long cmax_key(double x) {
  if (x != x) x = INFINITY;
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ void leaf_cmax_init_kernel(int nprob, unsigned long long* key) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nprob) key[b] = cmax_key(-INFINITY);
}

// key[b] = max over problem b's samples (of a slice of them per workgroup: x covers the
// samples, y the problems), as cmax_key.
__global__ __launch_bounds__(256) void leaf_cmax_kernel(const double* c, long per_prob,
                                                        int nprob, unsigned long long* key) {
  __shared__ unsigned long long red[256];
  for (long b = blockIdx.y; b < nprob; b += gridDim.y) {
  const double* cb = c + b * per_prob;
  unsigned long long v = cmax_key(-INFINITY);
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < per_prob; e += (long)gridDim.x * 256) {
    const unsigned long long k = cmax_key(cb[e]);
    v = k > v ? k : v;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(key + b, red[0]);
  __syncthreads();  // red is reused for the next problem
  }  // problems
}

// ------------------------------------------------------------------ A^{-1} (real)
// Thread grid GR x GC per leaf (as the impedance route's inverse), each thread owning
// ER x EC entries of A: rows tr + GR a, columns tc + GC b, all in registers.
//
// Blocked Gauss-Jordan with the diagonal blocks as pivots.  Under the route's test A is
// -Lap_h - kappa^2 c with kappa^2 c at most half the smallest Dirichlet eigenvalue: the
// discrete operator stays coercive, its diagonal dominates the elimination (no entry
// grows beyond the largest of A in the measured cases), and row exchanges are not
// needed.  Per block K of NBK columns (pivot block P = M[K, K]):
//   1. owners publish the panel columns M[:, K] to LDS;
//   2. one wave inverts P (Gauss-Jordan on its diagonal, P in registers, rows and
//      columns exchanged by cross-lane reads); a zero or non-finite pivot, or entries
//      grown beyond 1e8 times the largest of A, mark the leaf (the build then falls back
//      to the impedance route);
//   3. the block transformation Q (an LDS array of its own): rows K take P^{-1}, every
//      other row i takes -M[i, K] P^{-1}; owners publish the block's rows X = M[K, :]
//      (the identity on the columns K);
//   4. every entry becomes (rows K and columns K zeroed) + Q X.
// After the last block M holds A^{-1} in place, which is written to the real scratch copy
// (n_i x n_i per leaf; the Y_i product adds it as a real addend).
template <int P> struct DirCfg {
  static constexpr int m = P - 2;
  static constexpr int NI = m * m;
  static constexpr int ER = P <= 7 ? 1 : P <= 10 ? 2 : P == 11 ? 3 : P <= 13 ? 4
                          : P == 14 ? 8 : P == 15 ? 9 : 10;
  static constexpr int EC = P <= 7 ? 1 : P <= 9 ? 2 : P == 10 ? 4 : P == 11 ? 3
                          : P <= 13 ? 4 : P == 14 ? 6 : P == 15 ? 7 : 8;
  static constexpr int GR = (NI + ER - 1) / ER;
  static constexpr int GC = (NI + EC - 1) / EC;
  static constexpr int GE = (GC * EC > GR * ER ? GC * EC : GR * ER);  // LDS row stride
  static constexpr int NLIVE = GR * GC;
  static constexpr int NT = ((NLIVE + 63) / 64) * 64;
  static constexpr int NBK = 16;  // pivot block: one wave holds it, 4 entries per lane
  static_assert(NT <= 1024 && NT >= NI, "one thread per row, at most 1024");
  static_assert(GR * ER >= NI && GC * EC >= NI, "bad leaf grid");
};

// lane l of the inverting wave holds entries (l % 16, l / 16 + 4 q) of the 16 x 16 block
__device__ inline double pick4(const double (&v)[4], int q) {
  return q == 0 ? v[0] : q == 1 ? v[1] : q == 2 ? v[2] : v[3];
}

template <int P>
__global__ __launch_bounds__(DirCfg<P>::NT) void leaf_ainv_kernel(LeafDesc d) {
  using Cfg = DirCfg<P>;
  constexpr int m = Cfg::m, NI = Cfg::NI, ER = Cfg::ER, EC = Cfg::EC, GR = Cfg::GR,
                GC = Cfg::GC, GE = Cfg::GE, NBK = Cfg::NBK;
  constexpr int NB = 4 * m, N = P * P - 4;
  __shared__ double pan[NBK * GE];    // panel columns M[:, K]
  __shared__ double Qs[NBK * GE];     // block transformation Q
  __shared__ double Xs[NBK * GE];     // block rows M[K, :] (identity on K)
  __shared__ double sP[NBK][NBK];     // P^{-1}
  __shared__ double sL[2][m * m];
  __shared__ int s_bad;
  __shared__ unsigned long long s_amax;  // largest |entry| of A (bit pattern of a double >= 0)

  const long h = blockIdx.x;
  const long prob = (d.h0 + h) / d.nl1;
  if (!d.route[prob]) return;  // this problem takes the impedance route
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const bool live = tid < Cfg::NLIVE;
  const int tr = tid % GR, tc = tid / GR;
  const int g = d.leaf_grid[h];
  const double* rt = d.rtab + prob * RIdx{m}.len();
  for (int e = tid; e < m * m; e += Cfg::NT) {
    sL[0][e] = rt[RIdx{m}.lx() + e];
    sL[1][e] = rt[RIdx{m}.ly() + e];
  }
  // padding rows (beyond n_i) of the thread grid read Q and X there: keep them zero
  for (int e = tid; e < NBK * GE; e += Cfg::NT) {
    pan[e] = 0.0;
    Qs[e] = 0.0;
    Xs[e] = 0.0;
  }
  if (tid == 0) {
    s_bad = 0;
    s_amax = 0ull;
  }
  __syncthreads();
  const double kap = d.prm[4 * prob];
  const double k2 = kap * kap;
  const double* cl = d.c + (long)g * NI;

  // A = -(I (x) L_x) - (L_y (x) I) - kappa^2 diag(c) on the interior nodes
  // (node r = j m + i; L_x acts along x within a grid row, L_y along y)
  double M[ER][EC];
  double amax = 0.0;
#pragma unroll
  for (int a = 0; a < ER; ++a) {
    const int r = tr + GR * a;
    const int ir = r % m, jr = r / m;
    const double cr = (live && r < NI) ? cl[r] : 0.0;
#pragma unroll
    for (int b = 0; b < EC; ++b) {
      const int c = tc + GC * b;
      double v = 0.0;
      if (live && r < NI && c < NI) {
        const int ic = c % m, jc = c / m;
        if (jr == jc) v -= sL[0][ir + m * ic];
        if (ir == ic) v -= sL[1][jr + m * jc];
        if (r == c) v -= k2 * cr;
      }
      M[a][b] = v;
      amax = fmax(amax, fabs(v));
    }
  }
  atomicMax(&s_amax, (unsigned long long)__double_as_longlong(amax));

#pragma unroll 1
  for (int k0 = 0; k0 < NI; k0 += NBK) {
    const int nk = (NI - k0) < NBK ? (NI - k0) : NBK;
    // 1. panel columns
    if (live) {
#pragma unroll
      for (int a = 0; a < ER; ++a)
#pragma unroll
        for (int b = 0; b < EC; ++b) {
          const int j = tc + GC * b - k0;
          if (tr + GR * a < NI && j >= 0 && j < nk) pan[j * GE + tr + GR * a] = M[a][b];
        }
    }
    __syncthreads();
    // 2. P^{-1} by the first wave: lane holds P[i][jq], i = lane % 16, jq = lane / 16 + 4 q
    if (tid < 64) {
      const int i = lane & 15, c0 = lane >> 4;
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = c0 + 4 * q;
        v[q] = (i < nk && j < nk) ? pan[j * GE + k0 + i] : (i == j ? 1.0 : 0.0);
      }
      bool bad = false;
#pragma unroll 1
      for (int k = 0; k < NBK; ++k) {
        // row k's entries in this lane's columns (lanes k + 16 c0 hold them), and this
        // lane's row's entry in column k (lane i + 16 (k % 4), slot k / 4)
        double rk[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rk[q] = __shfl(v[q], k + 16 * c0);
        const double vk = pick4(v, k >> 2);
        const double cik = __shfl(vk, i + 16 * (k & 3));
        const double pk = __shfl(vk, k + 16 * (k & 3));
        bad = bad || !(fabs(pk) > 0.0) || !isfinite(pk);
        const double ip = 1.0 / pk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = c0 + 4 * q;
          if (i == k) v[q] = (j == k) ? ip : rk[q] * ip;
          else v[q] = (j == k) ? -cik * ip : fma(-cik * ip, rk[q], v[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) sP[i][c0 + 4 * q] = v[q];
      if (bad && lane == 0) s_bad = k0 + 1;
    }
    __syncthreads();
    if (s_bad) break;
    // 3. Q = -M[:, K] P^{-1} on rows outside K, P^{-1} on rows K (thread i, row i, four
    //    columns at a time, into its own LDS array); then the block's rows X = M[K, :]
    //    (identity on K) from their owners
    if (tid < NI) {
      const int ir = tid - k0;
      const bool inK = ir >= 0 && ir < nk;
#pragma unroll 1
      for (int j0 = 0; j0 < nk; j0 += 4) {
        double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int t = 0; t < nk; ++t) {
          const double rv = pan[t * GE + tid];
#pragma unroll
          for (int j = 0; j < 4; ++j) q[j] = fma(rv, sP[t][j0 + j], q[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j0 + j < nk) Qs[(j0 + j) * GE + tid] = inK ? sP[ir][j0 + j] : -q[j];
      }
    }
    if (live) {
#pragma unroll
      for (int a = 0; a < ER; ++a) {
        const int ir = tr + GR * a - k0;
        if (ir >= 0 && ir < nk) {
#pragma unroll
          for (int b = 0; b < EC; ++b) {
            const int c = tc + GC * b;
            const int j = c - k0;
            if (c < NI) Xs[ir * GE + c] = (j >= 0 && j < nk) ? (j == ir ? 1.0 : 0.0) : M[a][b];
          }
        }
      }
    }
    __syncthreads();
    // 4. block update: M <- (rows K and columns K zeroed) + Q X
    if (live) {
#pragma unroll
      for (int a = 0; a < ER; ++a) {
        const int ir = tr + GR * a - k0;
        const bool isP = ir >= 0 && ir < nk;
#pragma unroll
        for (int b = 0; b < EC; ++b) {
          const int j = tc + GC * b - k0;
          const bool inK = j >= 0 && j < nk;
          M[a][b] = (isP || inK) ? 0.0 : M[a][b];
        }
      }
      const double* qb = Qs + tr;
      const double* xbp = Xs + tc;
#pragma unroll 2
      for (int j = 0; j < nk; ++j) {
        double xb[EC];
#pragma unroll
        for (int b = 0; b < EC; ++b) xb[b] = xbp[j * GE + GC * b];
#pragma unroll
        for (int a = 0; a < ER; ++a) {
          const double qa = qb[j * GE + GR * a];
#pragma unroll
          for (int b = 0; b < EC; ++b) M[a][b] = fma(qa, xb[b], M[a][b]);
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
  // A^{-1} in place: consecutive threads hold consecutive rows of a column, so the
  // stores into the column-major scratch copy are coalesced.  An entry beyond 1e8 times the
  // largest of A, or a non-finite one, marks the leaf (growth check).
  const double lim = 1e8 * __longlong_as_double((long long)s_amax);
  bool grown = false;
  if (live) {
    // the output addresses are formed here (the empty asm hides the base from loop-invariant
    // code motion, which would otherwise keep 80 addresses live through the elimination)
    double* base = d.Ai;
    asm volatile("" : "+s"(base));
    double* Ai = base + h * (long)NI * NI;
#pragma unroll
    for (int a = 0; a < ER; ++a)
#pragma unroll
      for (int b = 0; b < EC; ++b) {
        const int ra = tr + GR * a, c = tc + GC * b;
        if (ra < NI && c < NI) {
          grown |= !(fabs(M[a][b]) <= lim);
          Ai[ra + (long)NI * c] = M[a][b];
        }
      }
  }
  if (grown) d.info[h] = NI + 1;  // every writer stores the same value
}

// ------------------------------------------------------------------ X, Z and S
// One workgroup per leaf.  A^{-1} (the real scratch copy) is read by grid rows:
// chunk k stages the m columns of the interior nodes (i, k) in LDS.  Then
//   X[r, W_k] = sum_i A^{-1}[r, (i,k)] aW[i] and X[r, E_k] likewise are complete, and
//   X[r, S_i] += A^{-1}[r, (i,k)] aS[k], X[r, N_i] += ... aN[k] accumulate (registers);
//   Z[b, (i,k)] for every boundary row b combines the rows of one grid line of the
//   staged column: S_t / N_t the rows (t, j) with nS[j] / nN[j], W_t / E_t the rows
//   (i', t) with nW[i'] / nE[i'].
// Each interior row has two threads: one for the S and W columns of X, one for N and E.
// X (n_i x n_b, column-major) and Z (n_b x n_i, column-major) go to scratch for the
// products; X also to LDS, from which S = F_bb - N_i X is formed into the Psi_b block
// (F_bb = N_bb + i eta I: each boundary row couples to the other end of its line).
template <int P>
__global__ __launch_bounds__(512) void leaf_xz_kernel(LeafDesc d) {
  constexpr int NT = 512;
  constexpr int m = P - 2, NI = m * m, NB = 4 * m, N = P * P - 4;
  static_assert(NI <= NT / 2, "two threads per interior row");
  __shared__ double sA[m][NI];
  __shared__ double sX[NB][NI];
  __shared__ double st[8 * m + 8];  // aS aN aW aE nS nN nW nE | fy fx
  const int tid = threadIdx.x;
  const long h = blockIdx.x;
  const long prob = (d.h0 + h) / d.nl1;
  double2* BI = reinterpret_cast<double2*>(d.BI) + h * (long)N * N;
  if (!d.route[prob]) {
    // impedance route: leave a harmless S = I for the shared inversion (the impedance
    // kernels overwrite this leaf's operators afterwards)
    for (int e = tid; e < NB * NB; e += NT) {
      const int b = e % NB, bp = e / NB;
      BI[b + (long)N * bp] = make_double2(b == bp ? 1.0 : 0.0, 0.0);
    }
    return;
  }
  const RIdx T{m};
  const double* rt = d.rtab + prob * T.len();
  for (int e = tid; e < 8 * m + 8; e += NT) st[e] = rt[T.aS() + e];
  const double* aS = st;
  const double* aN = st + m;
  const double* aW = st + 2 * m;
  const double* aE = st + 3 * m;
  const double* nS = st + 4 * m;
  const double* nN = st + 5 * m;
  const double* nW = st + 6 * m;
  const double* nE = st + 7 * m;
  const double* fy = st + 8 * m;
  const double* fx = st + 8 * m + 4;
  double* X = d.X + h * (long)NI * NB;
  double* Z = d.Z + h * (long)NB * NI;
  const double* Ai = d.Ai + h * (long)NI * NI;
  const int r = tid % (NT / 2), hh = tid / (NT / 2);  // hh 0: S and W columns; 1: N and E
  double acc[m];
#pragma unroll
  for (int i = 0; i < m; ++i) acc[i] = 0.0;
  constexpr int IT = (NI * m + NT - 1) / NT;
  double av[IT];
  auto load_chunk = [&](int k) {
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = tid + NT * q;
      av[q] = e < NI * m ? Ai[e % NI + (long)NI * (k * m + e / NI)] : 0.0;
    }
  };
  load_chunk(0);
#pragma unroll 1
  for (int k = 0; k < m; ++k) {
    __syncthreads();  // tables; the previous chunk's reads are done
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = tid + NT * q;
      if (e < NI * m) sA[e / NI][e % NI] = av[q];
    }
    if (k + 1 < m) load_chunk(k + 1);
    __syncthreads();
    if (r < NI) {
      const double wk = hh ? aN[k] : aS[k];
      const double* wl = hh ? aE : aW;
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < m; ++i) {
        const double y = sA[i][r];
        acc[i] = fma(y, wk, acc[i]);
        a = fma(y, wl[i], a);
      }
      const int bcol = hh ? m + k : 3 * m + k;  // E_k or W_k
      X[r + (long)NI * bcol] = a;
      sX[bcol][r] = a;
    }
    // Z on the chunk's columns (i, k), i < m
    for (int e = tid; e < NB * m; e += NT) {
      const int b = e % NB, i = e / NB;
      const int side = b / m, t = b % m;
      double z = 0.0;
      if (side == 0 || side == 2) {  // S_t, N_t: rows (t, j)
        const double* w = side == 0 ? nS : nN;
#pragma unroll
        for (int j = 0; j < m; ++j) z = fma(w[j], sA[i][j * m + t], z);
      } else {                       // E_t, W_t: rows (i', t)
        const double* w = side == 1 ? nE : nW;
#pragma unroll
        for (int q = 0; q < m; ++q) z = fma(w[q], sA[i][t * m + q], z);
      }
      Z[b + (long)NB * (k * m + i)] = z;
    }
  }
  if (r < NI) {
#pragma unroll
    for (int i = 0; i < m; ++i) {
      const int bcol = hh ? 2 * m + i : i;  // N_i or S_i
      X[r + (long)NI * bcol] = acc[i];
      sX[bcol][r] = acc[i];
    }
  }
  __syncthreads();
  // S = F_bb - N_i X  (F_bb = N_bb + i eta I)
  const double er = d.prm[4 * prob + 1], ei = d.prm[4 * prob + 2];
  for (int e = tid; e < NB * NB; e += NT) {
    const int b = e % NB, bp = e / NB;
    const int side = b / m, t = b % m;
    double v = 0.0;
    if (side == 0 || side == 2) {
      const double* w = side == 0 ? nS : nN;
#pragma unroll
      for (int j = 0; j < m; ++j) v = fma(w[j], sX[bp][j * m + t], v);
    } else {
      const double* w = side == 1 ? nE : nW;
#pragma unroll
      for (int q = 0; q < m; ++q) v = fma(w[q], sX[bp][t * m + q], v);
    }
    double2 s = make_double2(-v, 0.0);
    // N_bb: S_t <-> N_t through D_y's end rows, W_t <-> E_t through D_x's
    const int pside = bp / m, pt = bp % m;
    if (pt == t) {
      if (side == 0 && pside == 0) s.x += fy[0];
      if (side == 0 && pside == 2) s.x += fy[1];
      if (side == 2 && pside == 0) s.x += fy[2];
      if (side == 2 && pside == 2) s.x += fy[3];
      if (side == 3 && pside == 3) s.x += fx[0];
      if (side == 3 && pside == 1) s.x += fx[1];
      if (side == 1 && pside == 3) s.x += fx[2];
      if (side == 1 && pside == 1) s.x += fx[3];
    }
    if (b == bp) {  // + i eta
      s.x -= ei;
      s.y += er;
    }
    BI[b + (long)N * bp] = s;
  }
}

// R = I - 2 i eta Psi_b for the leaves of this route.
template <int P>
__global__ __launch_bounds__(256) void leaf_dir_R_kernel(LeafDesc d) {
  constexpr int m = P - 2, NB = 4 * m, N = P * P - 4;
  const long h = blockIdx.x;
  const long prob = (d.h0 + h) / d.nl1;
  if (!d.route[prob]) return;
  const double2* BI = reinterpret_cast<const double2*>(d.BI) + h * (long)N * N;
  double2* R = reinterpret_cast<double2*>(d.R) + h * (long)NB * NB;
  // -2 i eta = (2 eta_im, -2 eta_re)
  const double2 m2ie = make_double2(2.0 * d.prm[4 * prob + 2], -2.0 * d.prm[4 * prob + 1]);
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int b = e % NB, bp = e / NB;
    double2 v = cmul(m2ie, BI[b + (long)N * bp]);
    if (b == bp) v.x += 1.0;
    R[e] = v;
  }
}

template <int P> void launch_ainv(const LeafDesc& d, hipStream_t st) {
  hipLaunchKernelGGL(leaf_ainv_kernel<P>, dim3(d.nleaf), dim3(DirCfg<P>::NT), 0, st, d);
}
template <int P> void launch_xz(const LeafDesc& d, hipStream_t st) {
  hipLaunchKernelGGL(leaf_xz_kernel<P>, dim3(d.nleaf), dim3(512), 0, st, d);
}
template <int P> void launch_dir_R(const LeafDesc& d, hipStream_t st) {
  hipLaunchKernelGGL(leaf_dir_R_kernel<P>, dim3(d.nleaf), dim3(256), 0, st, d);
}

#define HPS_P_SWITCH_DIR(FN, p, ...)               \
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

int leaf_rtable_len(int p) { return RIdx{p - 2}.len(); }

void leaf_cmax(const double* c, int nprob, long per_prob, double* cmax, hipStream_t st) {
  if (nprob <= 0) return;
  unsigned long long* key = reinterpret_cast<unsigned long long*>(cmax);
  hipLaunchKernelGGL(leaf_cmax_init_kernel, dim3(cdiv(nprob, 256)), dim3(256), 0, st, nprob, key);
  HPS_LAUNCH_CHECK();
  const unsigned gx = (unsigned)std::min<long>(64, std::max<long>(1, cdiv(per_prob, 4096)));
  hipLaunchKernelGGL(leaf_cmax_kernel, dim3(gx, grid_y(nprob)), dim3(256), 0, st, c, per_prob,
                     nprob, key);
  HPS_LAUNCH_CHECK();
}

double leaf_cmax_value(unsigned long long k) {
  const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  double x;
  std::memcpy(&x, &u, sizeof x);
  return x;
}

void leaf_dirichlet_inverse(const LeafDesc& d, hipStream_t st) {
  if (d.nleaf <= 0) return;
  HPS_P_SWITCH_DIR(launch_ainv, d.p, d, st);
  HPS_LAUNCH_CHECK();
}

void leaf_dirichlet_xz(const LeafDesc& d, hipStream_t st) {
  if (d.nleaf <= 0) return;
  HPS_P_SWITCH_DIR(launch_xz, d.p, d, st);
  HPS_LAUNCH_CHECK();
}

void leaf_dirichlet_R(const LeafDesc& d, hipStream_t st) {
  if (d.nleaf <= 0) return;
  HPS_P_SWITCH_DIR(launch_dir_R, d.p, d, st);
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
