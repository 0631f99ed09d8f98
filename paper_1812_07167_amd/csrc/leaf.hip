// Leaf stage (Sec. 2.1, 2.1.1, 2.1.2): for every leaf, the operators Psi (n x n_b),
// Y (n x n_i) with B [Psi | Y] = I, and the ItI operator R = G Psi.
//
// With u = [u_b; u_i], B = [[N_b + i eta I, N_i], [A_ib, A_ii]] where A = Ahat(I_i, :)
// is real for real c.  Block elimination (derived from eqs. (homogeneous) and
// (particular)):
//   X = A_ii^{-1} A_ib,  Z = N_i A_ii^{-1},  S = N_b + i eta I - N_i X
//   Psi_b = S^{-1},  Psi_i = -X Psi_b,  Y_b = -Psi_b Z,  Y_i = A_ii^{-1} - X Y_b
//   R = G Psi = I - 2 i eta Psi_b      (G = F - 2 i eta E_b and F Psi = I)
// Only S and what follows are complex.  A_ib, N_i, N_b are sparse (one grid line per
// boundary node), so X, Z and S are formed by line sums.
//
// Kernels: leaf_inv (A_ii^{-1} by register-resident blocked Gauss-Jordan with partial
// pivoting, one workgroup per leaf), leaf_xzs (X, Z, S), then the batched complex
// inverse of S and three batched MFMA GEMMs (launched by the host driver).
#include "kernels.hpp"

namespace hps {
namespace {

// Thread grid GR x GC per leaf, each thread owning ER x EC entries of A_ii (padded):
// rows tr + GR a, columns tc + GC b.  Pivots are taken in blocks of NBK columns.
template <int P> struct LeafInvCfg {
  static constexpr int m = P - 2;
  static constexpr int NI = m * m;
  static constexpr int ER = P <= 9 ? (m > 0 ? m : 1)
                          : P == 10 ? 4 : P <= 13 ? 5 : P == 14 ? 6 : 7;
  static constexpr int EC = P == 16 ? 9 : ER;               // p=16: 616 threads, 63 entries
  static constexpr int GR = (NI + ER - 1) / ER;
  static constexpr int GC = (NI + EC - 1) / EC;
  static constexpr int GE = (GC * EC > GR * ER ? GC * EC : GR * ER);  // LDS row stride
  static constexpr int NLIVE = GR * GC;                     // threads that own entries
  static constexpr int NT = ((NLIVE + 63) / 64) * 64;       // whole waves (shuffles)
  static constexpr int NBK = 8;                             // pivots per block
  static constexpr int PQ = (NI + 63) / 64;                 // panel rows per lane
  static constexpr int LDS_DOUBLES = 19200;                 // GJ buffers / output staging
  static constexpr int CW = (LDS_DOUBLES / NI) < NI ? (LDS_DOUBLES / NI) : NI;
  static_assert(NT <= 1024, "too many threads");
  static_assert(GR * ER >= NI && 3 * NBK * GE <= LDS_DOUBLES, "bad leaf grid");
};

// A_ii^{-1} by blocked Gauss-Jordan with partial pivoting, matrix resident in
// registers.  Per block K of NBK pivot columns:
//   1. owners publish the panel columns M[:, K] to LDS;
//   2. wave 0 runs the NBK elimination steps on the panel (pivot = largest unused
//      |entry|), giving the block transformation Q and the pivot rows P_K;
//   3. owners of the pivot rows publish X = M[P_K, :];
//   4. every entry outside K becomes (pivot rows zeroed) + Q X, entries in K become Q.
// This is the same in-place elimination as column-at-a-time Gauss-Jordan (the block
// step applies the product of the NBK elementary transformations at once); the
// in-place result M satisfies A^{-1}[k][piv[j]] = M[piv[k]][j].
template <int P>
__global__ __launch_bounds__(LeafInvCfg<P>::NT) void leaf_inv_kernel(LeafDesc d) {
  using Cfg = LeafInvCfg<P>;
  constexpr int m = Cfg::m, NI = Cfg::NI, ER = Cfg::ER, EC = Cfg::EC, GR = Cfg::GR,
                GC = Cfg::GC, GE = Cfg::GE;
  constexpr int NBK = Cfg::NBK, PQ = Cfg::PQ;
  constexpr int NB = 4 * m, N = P * P - 4;
  __shared__ double pool[Cfg::LDS_DOUBLES];
  __shared__ int piv[NI], ipiv[NI];
  __shared__ int slot[NI];          // position of a row in the current block's pivots, or -1
  __shared__ int used_s[NI];
  __shared__ double sD[2][P * P];
  __shared__ int s_bad;
  double* bufA = pool;              // [NBK][GE]  panel / block transformation
  double* bufB = pool + NBK * GE;   // [NBK][GE]  (ping-pong partner)
  double* Xs = pool + 2 * NBK * GE; // [NBK][GE]  pivot rows
  double* pan = bufA;               // receives the next block's panel columns
  double* oth = bufB;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const bool live = tid < Cfg::NLIVE;  // padding threads own nothing and publish nothing
  const int tr = tid % GR, tc = tid / GR;
  const long h = blockIdx.x;
  const int g = d.leaf_grid[h];
  for (int e = tid; e < P * P; e += Cfg::NT) {
    sD[0][e] = d.D[2 * P * P + e];  // Dxx
    sD[1][e] = d.D[3 * P * P + e];  // Dyy
  }
  for (int i = tid; i < NI; i += Cfg::NT) {
    slot[i] = -1;
    used_s[i] = 0;
  }
  for (int e = tid; e < 3 * NBK * GE; e += Cfg::NT) pool[e] = 0.0;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  const double k2 = d.kappa * d.kappa;
  const double* cl = d.c + (long)g * NI;

  // assemble A_ii = -Dxx (x) I - I (x) Dyy - kappa^2 diag(c) on interior nodes
  double M[ER][EC];
#pragma unroll
  for (int a = 0; a < ER; ++a) {
    const int r = tr + GR * a;
    const int ir = r % m + 1, jr = r / m + 1;
    const double cr = (live && r < NI) ? cl[r] : 0.0;
#pragma unroll
    for (int b = 0; b < EC; ++b) {
      const int c = tc + GC * b;
      double v = 0.0;
      if (live && r < NI && c < NI) {
        const int ic = c % m + 1, jc = c / m + 1;
        if (jr == jc) v -= sD[0][ir + P * ic];
        if (ir == ic) v -= sD[1][jr + P * jc];
        if (r == c) v -= k2 * cr;
      }
      M[a][b] = v;
    }
  }

#pragma unroll 1
  for (int k0 = 0; k0 < NI; k0 += NBK) {
    const int nk = (NI - k0) < NBK ? (NI - k0) : NBK;
    // 1. panel columns (into the buffer that does not hold the previous block's Q)
    if (live) {
#pragma unroll
      for (int a = 0; a < ER; ++a) {
        const int ra = tr + GR * a;
#pragma unroll
        for (int b = 0; b < EC; ++b) {
          const int j = tc + GC * b - k0;
          if (ra < NI && j >= 0 && j < nk) pan[j * GE + ra] = M[a][b];
        }
      }
    }
    __syncthreads();
    // 2. elimination on the panel (wave 0); each step reads one LDS buffer and writes
    //    the other, so the pivot row is never read after it has been rescaled
    if (wave == 0) {
      if (lane == 0 && k0 > 0)
        for (int s = 0; s < NBK; ++s) slot[piv[k0 - NBK + s]] = -1;
      unsigned usedq = 0;
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int i = lane + 64 * q;
        if (i >= NI || used_s[i]) usedq |= 1u << q;
      }
#pragma unroll 1
      for (int s = 0; s < nk; ++s) {
        const double* src = (s & 1) ? oth : pan;
        double* dst = (s & 1) ? pan : oth;
        double best = -1.0;
        int bi = NI;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int i = lane + 64 * q;
          const double v = ((usedq >> q) & 1u) ? -1.0 : fabs(src[s * GE + (i < NI ? i : 0)]);
          if (v > best) { best = v; bi = i; }
        }
        const int r = wave_argmax(best, bi);
        if (r < 0) {
          if (lane == 0) s_bad = k0 + s + 1;
          break;
        }
        const double ip = 1.0 / src[s * GE + r];
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int i = lane + 64 * q;
          if (i < NI) {
            const bool isr = (i == r);
            const double f = src[s * GE + i] * ip;
#pragma unroll
            for (int j = 0; j < NBK; ++j) {
              if (j < nk) {
                const double pv = src[j * GE + i];
                double v = fma(-f, src[j * GE + r], pv);
                v = isr ? pv * ip : v;
                v = (j == s) ? (isr ? ip : -f) : v;
                dst[j * GE + i] = v;
              }
            }
            if (isr) usedq |= 1u << q;
          }
        }
        if (lane == 0) {
          piv[k0 + s] = r;
          slot[r] = s;
          used_s[r] = 1;
        }
      }
    }
    __syncthreads();
    if (s_bad) break;
    const double* Qs = (nk & 1) ? oth : pan;  // buffer written by the last step
    // 3. pivot rows (values before this block's update); on the panel columns X is the
    //    identity, so that the update below writes Q there
    if (live) {
#pragma unroll
      for (int a = 0; a < ER; ++a) {
        const int ra = tr + GR * a;
        const int sl = ra < NI ? slot[ra] : -1;
        if (sl >= 0)
#pragma unroll
          for (int b = 0; b < EC; ++b) {
            const int j = tc + GC * b - k0;
            Xs[sl * GE + tc + GC * b] = (j >= 0 && j < nk) ? (j == sl ? 1.0 : 0.0) : M[a][b];
          }
      }
    }
    __syncthreads();
    // 4. block update: M <- (M with pivot rows and panel columns zeroed) + Q X
    if (live) {
#pragma unroll
      for (int a = 0; a < ER; ++a) {
        const int ra = tr + GR * a;
        const bool isP = ra < NI && slot[ra] >= 0;
#pragma unroll
        for (int b = 0; b < EC; ++b) {
          const int j = tc + GC * b - k0;
          const bool inK = j >= 0 && j < nk;
          M[a][b] = (isP || inK) ? 0.0 : M[a][b];
        }
      }
      const double* qb = Qs + tr;
      const double* xbp = Xs + tc;
#pragma unroll 1
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
    if (!(nk & 1)) {  // Q is in pan: the next panel goes to the other buffer
      double* t = pan;
      pan = oth;
      oth = t;
    }
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) d.info[h] = s_bad;
    return;
  }
  for (int k = tid; k < NI; k += Cfg::NT) ipiv[piv[k]] = k;
  __syncthreads();
  // write A_ii^{-1}[k][piv[c]] = M[piv[k]][c]:  entry (row ri, col c) goes to
  // (ipiv[ri], piv[c]); stage column chunks in LDS for coalesced complex stores into
  // the Y_i block of [Psi | Y].
  double2* BI = reinterpret_cast<double2*>(d.BI) + h * (long)N * N;
  for (int c0 = 0; c0 < NI; c0 += Cfg::CW) {
    const int cw = (NI - c0) < Cfg::CW ? (NI - c0) : Cfg::CW;
#pragma unroll
    for (int a = 0; a < ER; ++a) {
      const int ra = tr + GR * a;
      if (!live || ra >= NI) continue;
      const int orow = ipiv[ra];
#pragma unroll
      for (int b = 0; b < EC; ++b) {
        const int c = tc + GC * b;
        if (c >= NI) continue;
        const int ocol = piv[c] - c0;
        if (ocol >= 0 && ocol < cw) pool[orow + NI * ocol] = M[a][b];
      }
    }
    __syncthreads();
    for (int e = tid; e < NI * cw; e += Cfg::NT) {
      const int row = e % NI, col = e / NI;
      BI[(NB + row) + (long)N * (NB + c0 + col)] = make_double2(pool[e], 0.0);
    }
    __syncthreads();
  }
}

// X (ni x nb), Z (nb x ni), S (nb x nb) of one leaf from A_ii^{-1} (real parts of
// the Y_i block).  One 256-thread workgroup per leaf.
template <int P>
__global__ __launch_bounds__(256) void leaf_xzs_kernel(LeafDesc d) {
  constexpr int m = P - 2, NI = m * m, NB = 4 * m, N = P * P - 4;
  __shared__ double sX[NI * NB];
  __shared__ double sD[4][P * P];
  const int tid = threadIdx.x;
  const long h = blockIdx.x;
  for (int e = tid; e < 4 * P * P; e += 256) sD[e / (P * P)][e % (P * P)] = d.D[e];
  __syncthreads();
  const double* Dx1 = sD[0];
  const double* Dy1 = sD[1];
  const double* Dxx = sD[2];
  const double* Dyy = sD[3];
  const double2* BI = reinterpret_cast<const double2*>(d.BI) + h * (long)N * N;
  auto ainv = [&](int r, int q) { return BI[(NB + r) + (long)N * (NB + q)].x; };

  if (tid < NI) {
    // X[r, b] = sum_{q on b's line} Ainv[r, q] A_ib[q, b]
    const int r = tid;
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
#pragma unroll
    for (int j = 0; j < m; ++j)
#pragma unroll
      for (int i = 0; i < m; ++i) {
        const double a = ainv(r, i + m * j);
        acc[i] = fma(a, -Dyy[(j + 1) + P * 0], acc[i]);                    // S_i
        acc[2 * m + i] = fma(a, -Dyy[(j + 1) + P * (P - 1)], acc[2 * m + i]);  // N_i
        acc[m + j] = fma(a, -Dxx[(i + 1) + P * (P - 1)], acc[m + j]);      // E_j
        acc[3 * m + j] = fma(a, -Dxx[(i + 1) + P * 0], acc[3 * m + j]);    // W_j
      }
    double* X = d.X + h * (long)NI * NB;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      X[r + (long)NI * b] = acc[b];
      sX[r + NI * b] = acc[b];
    }
  } else {
    // idle threads of the X phase
  }
  if (tid < NI) {
    // Z[b, c] = sum_{q on b's line} N_i[b, q] Ainv[q, c]
    const int c = tid;
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
#pragma unroll
    for (int j = 0; j < m; ++j)
#pragma unroll
      for (int i = 0; i < m; ++i) {
        const double a = ainv(i + m * j, c);
        acc[i] = fma(-Dy1[0 + P * (j + 1)], a, acc[i]);                        // S_i: -D_y
        acc[2 * m + i] = fma(Dy1[(P - 1) + P * (j + 1)], a, acc[2 * m + i]);   // N_i: +D_y
        acc[m + j] = fma(Dx1[(P - 1) + P * (i + 1)], a, acc[m + j]);           // E_j: +D_x
        acc[3 * m + j] = fma(-Dx1[0 + P * (i + 1)], a, acc[3 * m + j]);        // W_j: -D_x
      }
    double* Z = d.Z + h * (long)NB * NI;
#pragma unroll
    for (int b = 0; b < NB; ++b) Z[b + (long)NB * c] = acc[b];
  }
  __syncthreads();
  // S = N_b + i eta I - N_i X
  double2* S = reinterpret_cast<double2*>(d.S) + h * (long)NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int b = e % NB, bp = e / NB;
    const int side = b / m, t = b % m;  // 0 S, 1 E, 2 N, 3 W; t = position on the side
    double s = 0.0, nb = 0.0;
    if (side == 0) {          // S_t: -D_y row 0 along column i = t+1
      for (int j = 0; j < m; ++j) s = fma(-Dy1[0 + P * (j + 1)], sX[(t + m * j) + NI * bp], s);
      if (bp == b) nb = -Dy1[0];
      if (bp == 2 * m + t) nb = -Dy1[0 + P * (P - 1)];
    } else if (side == 1) {   // E_t: +D_x row p-1 along row j = t+1
      for (int i = 0; i < m; ++i) s = fma(Dx1[(P - 1) + P * (i + 1)], sX[(i + m * t) + NI * bp], s);
      if (bp == b) nb = Dx1[(P - 1) + P * (P - 1)];
      if (bp == 3 * m + t) nb = Dx1[(P - 1) + P * 0];
    } else if (side == 2) {   // N_t: +D_y row p-1 along column i = t+1
      for (int j = 0; j < m; ++j) s = fma(Dy1[(P - 1) + P * (j + 1)], sX[(t + m * j) + NI * bp], s);
      if (bp == b) nb = Dy1[(P - 1) + P * (P - 1)];
      if (bp == t) nb = Dy1[(P - 1) + P * 0];
    } else {                  // W_t: -D_x row 0 along row j = t+1
      for (int i = 0; i < m; ++i) s = fma(-Dx1[0 + P * (i + 1)], sX[(i + m * t) + NI * bp], s);
      if (bp == b) nb = -Dx1[0];
      if (bp == m + t) nb = -Dx1[0 + P * (P - 1)];
    }
    double re = nb - s, im = 0.0;
    if (bp == b) {  // + i eta
      re -= d.eta_im;
      im += d.eta_re;
    }
    S[b + (long)NB * bp] = make_double2(re, im);
  }
}

__global__ void leaf_r_kernel(int nleaf, int n, int nb, double er, double ei, const double* BIg,
                              double* Rg) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)nleaf * nb * nb;
  if (e >= tot) return;
  const long h = e / ((long)nb * nb);
  const int loc = e % ((long)nb * nb);
  const int i = loc % nb, j = loc / nb;
  const double2 psi = reinterpret_cast<const double2*>(BIg)[h * (long)n * n + i + (long)n * j];
  // -2 i eta = (2 eta_im, -2 eta_re)
  double2 v = cmul(cmk(2.0 * ei, -2.0 * er), psi);
  if (i == j) v.x += 1.0;
  reinterpret_cast<double2*>(Rg)[e] = v;
}

template <int P> void launch_inv(const LeafDesc& d, hipStream_t st) {
  hipLaunchKernelGGL(leaf_inv_kernel<P>, dim3(d.nleaf), dim3(LeafInvCfg<P>::NT), 0, st, d);
}
template <int P> void launch_xzs(const LeafDesc& d, hipStream_t st) {
  hipLaunchKernelGGL(leaf_xzs_kernel<P>, dim3(d.nleaf), dim3(256), 0, st, d);
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

void leaf_inverse_interior(const LeafDesc& d, hipStream_t st) {
  if (d.nleaf <= 0) return;
  HPS_P_SWITCH(launch_inv, d.p, d, st);
  HPS_LAUNCH_CHECK();
}

void leaf_xzs(const LeafDesc& d, hipStream_t st) {
  if (d.nleaf <= 0) return;
  HPS_P_SWITCH(launch_xzs, d.p, d, st);
  HPS_LAUNCH_CHECK();
}

void leaf_r_from_psib(const LeafDesc& d, hipStream_t st) {
  const int n = d.p * d.p - 4, nb = 4 * d.p - 8;
  const long tot = (long)d.nleaf * nb * nb;
  hipLaunchKernelGGL(leaf_r_kernel, dim3(cdiv(tot, 256)), dim3(256), 0, st, d.nleaf, n, nb,
                     d.eta_re, d.eta_im, d.BI, d.R);
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
