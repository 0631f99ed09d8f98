// Batched complex GEMM on the FP64 matrix cores of gfx950 (v_mfma_f64_16x16x4f64).
//
// A complex product is formed from four real products (Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br); a real operand drops two of them.  Tiles of BM x BN outputs
// per 256-thread workgroup (four waves in a 2 x 2 arrangement), K staged through LDS
// in chunks of 16 with the next chunk's global loads issued before the current
// chunk's MFMAs.  Used by the leaf stage (Sec. 2.1: Psi_i, Y_b, Y_i) and by every
// merge product of Sec. 2.2 (W, Phi^a, Phi^b, R^tau).
//
// MFMA f64 16x16x4 lane layout (measured on gfx950): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element v of lane l is D[l/16 + 4 v][l%16].
#include "kernels.hpp"

namespace hps {
namespace {

constexpr int BK = 16;

template <int BM, int BN, bool AR, bool BR>
__global__ __launch_bounds__(256) void zgemm_kernel(GemmDesc d) {
  constexpr int NPA = AR ? 1 : 2;  // planes (re, im) of A
  constexpr int NPB = BR ? 1 : 2;
  constexpr int WM = BM / 2, WN = BN / 2;  // per-wave tile
  constexpr int MB = WM / 16, NB = WN / 16;
  static_assert(MB >= 1 && NB >= 1, "tile too small");
  __shared__ double As[2][NPA][BK][BM];
  __shared__ double Bs[2][NPB][BK][BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int i0 = tm * BM, j0 = tn * BN;
  const long b = blockIdx.y;

  const double* A = d.A + b * d.sA * NPA;
  const double* B = d.B + b * d.sB * NPB;

  d4v accR[MB][NB], accI[MB][NB];
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      accR[x][y] = d4v{0, 0, 0, 0};
      accI[x][y] = d4v{0, 0, 0, 0};
    }

  constexpr int EA = BM * BK / 256;  // A elements per thread per chunk
  constexpr int EB = BN * BK / 256;
  double ra[EA][NPA], rb[EB][NPB];

  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + 256 * e;
      int i = idx % BM, k = idx / BM;
      int gi = i0 + i, gk = k0 + k;
      bool ok = gi < d.M && gk < d.K;
      long off = (long)gi + d.lda * (long)gk;
      if (AR) {
        ra[e][0] = ok ? A[off] : 0.0;
      } else {
        double2 v = ok ? reinterpret_cast<const double2*>(A)[off] : make_double2(0.0, 0.0);
        ra[e][0] = v.x;
        ra[e][NPA - 1] = v.y;
      }
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + 256 * e;
      int k = idx % BK, j = idx / BK;
      int gk = k0 + k, gj = j0 + j;
      bool ok = gk < d.K && gj < d.N;
      long off = (long)gk + d.ldb * (long)gj;
      if (BR) {
        rb[e][0] = ok ? B[off] : 0.0;
      } else {
        double2 v = ok ? reinterpret_cast<const double2*>(B)[off] : make_double2(0.0, 0.0);
        rb[e][0] = v.x;
        rb[e][NPB - 1] = v.y;
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + 256 * e;
      int i = idx % BM, k = idx / BM;
#pragma unroll
      for (int pl = 0; pl < NPA; ++pl) As[buf][pl][k][i] = ra[e][pl];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + 256 * e;
      int k = idx % BK, j = idx / BK;
#pragma unroll
      for (int pl = 0; pl < NPB; ++pl) Bs[buf][pl][k][j] = rb[e][pl];
    }
  };

  const int nk = (d.K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kl = kk + (lane >> 4);
      double ar[MB], ai[MB], br[NB], bi[NB];
#pragma unroll
      for (int x = 0; x < MB; ++x) {
        int r = wr * WM + 16 * x + (lane & 15);
        ar[x] = As[buf][0][kl][r];
        ai[x] = AR ? 0.0 : As[buf][NPA - 1][kl][r];
      }
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        int c = wc * WN + 16 * y + (lane & 15);
        br[y] = Bs[buf][0][kl][c];
        bi[y] = BR ? 0.0 : Bs[buf][NPB - 1][kl][c];
      }
#pragma unroll
      for (int x = 0; x < MB; ++x)
#pragma unroll
        for (int y = 0; y < NB; ++y) {
          accR[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[x], br[y], accR[x][y], 0, 0, 0);
          if (!AR && !BR)
            accR[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[x], bi[y], accR[x][y], 0, 0, 0);
          if (!BR)
            accI[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[x], bi[y], accI[x][y], 0, 0, 0);
          if (!AR)
            accI[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[x], br[y], accI[x][y], 0, 0, 0);
        }
    }
    if (kc + 1 < nk) {
      sstore(buf ^ 1);
    }
    __syncthreads();
  }

  // epilogue
  double2* C = reinterpret_cast<double2*>(d.C) + b * d.sC;
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + wr * WM + 16 * x + (lane >> 4) + 4 * v;
        int j = j0 + wc * WN + 16 * y + (lane & 15);
        if (i < d.M && j < d.N) {
          long ri = d.crow ? d.crow[i] : i;
          long cj = d.ccol ? d.ccol[j] : j;
          double2* p = C + ri + d.ldc * cj;
          double2 val = cmk(d.alpha * accR[x][y][v], d.alpha * accI[x][y][v]);
          if (d.beta != 0.0) {
            double2 old = *p;
            val.x += d.beta * old.x;
            val.y += d.beta * old.y;
          }
          *p = val;
        }
      }
}

template <int BM, int BN>
void launch_tile(const GemmDesc& d, hipStream_t st) {
  int tiles = cdiv(d.M, BM) * cdiv(d.N, BN);
  dim3 grid(tiles, d.batch);
  if (d.a_real && d.b_real)
    hipLaunchKernelGGL((zgemm_kernel<BM, BN, true, true>), grid, dim3(256), 0, st, d);
  else if (d.a_real)
    hipLaunchKernelGGL((zgemm_kernel<BM, BN, true, false>), grid, dim3(256), 0, st, d);
  else if (d.b_real)
    hipLaunchKernelGGL((zgemm_kernel<BM, BN, false, true>), grid, dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL((zgemm_kernel<BM, BN, false, false>), grid, dim3(256), 0, st, d);
}

}  // namespace

void zgemm(const GemmDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  if (d.batch > 65535) throw Error(1, "zgemm: batch exceeds grid limit");
  if (d.K <= 0) {
    // C = beta*C only; K == 0 does not occur on the solver's paths.
    throw Error(1, "zgemm: K must be positive");
  }
  if (d.M <= 32 && d.N <= 32)
    launch_tile<32, 32>(d, st);
  else
    launch_tile<64, 64>(d, st);
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
