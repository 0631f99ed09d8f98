// Batched complex matrix inversion by Gauss-Jordan elimination with partial pivoting
// (the explicit W^{-1} of the merge, Sec. 2.2 / Sec. 2.4, and the leaf's boundary
// Schur complement).
//
// Pivoting is implicit: the pivot of column k is the unused row r_k of largest
// |re|+|im|; rows are never moved.  After all n steps the in-place matrix M satisfies
// inv(A)[k][r_j] = M[r_k][j], which the final write-out applies.
//
// * n <= SMALL_MAX: one workgroup per matrix, matrix resident in LDS.
// * larger n: blocked right-looking form.  For each block K of 16 columns a panel
//   kernel (one 16-wave workgroup per matrix, one panel column per wave, rows in
//   registers) runs the 16 elimination steps on the panel, emits the block
//   transformation Q, gathers the pivot rows X = M[P_K, :] (zero on K) and clears
//   them; a batched MFMA GEMM then applies M += Q X to every column.
#include "kernels.hpp"

namespace hps {
namespace {

constexpr int SMALL_MAX = 96;
constexpr int PNB = 16;  // panel width of the blocked path

// ------------------------------------------------------------------ small (LDS)
__global__ __launch_bounds__(256) void zinv_small_kernel(int n, const double* Ain, long lda,
                                                         long sA, double* Out, long ldo,
                                                         long sO, int* info) {
  extern __shared__ double2 sm[];
  double2* M = sm;                                   // n*n
  int* piv = reinterpret_cast<int*>(M + n * n);      // n
  int* ipiv = piv + n;                               // n
  int* used = ipiv + n;                              // n
  __shared__ int s_r;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const long b = blockIdx.x;
  const double2* A = reinterpret_cast<const double2*>(Ain) + b * sA;
  for (int e = tid; e < n * n; e += 256) {
    int i = e % n, j = e / n;
    M[e] = A[i + lda * j];
  }
  for (int i = tid; i < n; i += 256) used[i] = 0;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = n;
      for (int i = tid; i < n; i += 64) {
        double v = used[i] ? -1.0 : cabs1(M[i + n * k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ob = __shfl_xor(best, off);
        int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        s_r = bi;
        if (!(best > 0.0)) s_bad = k + 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int r = s_r;
    const double2 ip = crcp(M[r + n * k]);
    for (int e = tid; e < n * n; e += 256) {
      int i = e % n, c = e / n;
      if (i != r && c != k) {
        double2 f = cmul(M[i + n * k], ip);
        M[e] = csub(M[e], cmul(f, M[r + n * c]));
      }
    }
    __syncthreads();
    for (int e = tid; e < n; e += 256) {
      if (e != k) M[r + n * e] = cmul(M[r + n * e], ip);
      if (e != r) M[e + n * k] = cmk(-(M[e + n * k].x * ip.x - M[e + n * k].y * ip.y),
                                     -(M[e + n * k].x * ip.y + M[e + n * k].y * ip.x));
    }
    if (tid == 0) {
      M[r + n * k] = ip;
      used[r] = 1;
      piv[k] = r;
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) info[b] = s_bad;
    return;
  }
  for (int k = tid; k < n; k += 256) ipiv[piv[k]] = k;
  __syncthreads();
  double2* O = reinterpret_cast<double2*>(Out) + b * sO;
  for (int e = tid; e < n * n; e += 256) {
    int k = e % n, j = e / n;
    O[k + ldo * j] = M[piv[k] + n * ipiv[j]];
  }
}

// ------------------------------------------------------------------ blocked
template <int Q>
__global__ __launch_bounds__(1024) void zinv_panel_kernel(int n, double* Mg, int k0,
                                                          double* Qbuf, double* Xbuf, int* piv,
                                                          int* used, int* info) {
  __shared__ double2 colbuf[2][64 * Q];
  __shared__ int s_r[2];
  __shared__ double s_v[2];
  __shared__ int s_piv[PNB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long b = blockIdx.x;
  double2* M = reinterpret_cast<double2*>(Mg) + b * (long)n * n;
  int* pv = piv + b * (long)n;
  int* us = used + b * (long)n;
  const int c = k0 + w;
  double2 v[Q];
  unsigned long long umask = 0;  // bit q: row lane+64q already used as a pivot
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int i = lane + 64 * q;
    v[q] = (i < n && c < n) ? M[i + (long)n * c] : cmk(0, 0);
    if (i >= n || us[i]) umask |= (1ull << q);
  }
  int bad = 0;
  for (int s = 0; s < PNB; ++s) {
    const int k = k0 + s;
    if (k >= n) break;
    const int buf = s & 1;
    if (w == s) {
      double best = -1.0;
      int bi = n;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        int i = lane + 64 * q;
        double val = (umask >> q) & 1 ? -1.0 : cabs1(v[q]);
        if (val > best) { best = val; bi = i; }
        if (i < n) colbuf[buf][i] = v[q];
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ob = __shfl_xor(best, off);
        int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) { s_r[buf] = bi; s_v[buf] = best; }
    }
    __syncthreads();
    const int r = s_r[buf];
    if (!(s_v[buf] > 0.0)) { bad = k + 1; break; }
    const double2 ip = crcp(colbuf[buf][r]);
    // value of this wave's column at the pivot row
    double2 mine = cmk(0, 0);
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (q == (r >> 6)) mine = v[q];
    double2 prw;
    prw.x = __shfl(mine.x, r & 63);
    prw.y = __shfl(mine.y, r & 63);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      int i = lane + 64 * q;
      if (i < n) {
        if (i == r) {
          v[q] = (w == s) ? ip : cmul(v[q], ip);
          umask |= (1ull << q);
        } else {
          double2 f = cmul(colbuf[buf][i], ip);
          v[q] = (w == s) ? cmk(-f.x, -f.y) : csub(v[q], cmul(f, prw));
        }
      }
    }
    if (threadIdx.x == 0) {
      pv[k] = r;
      s_piv[s] = r;
    }
  }
  if (bad) {
    if (threadIdx.x == 0) info[b] = bad;
    return;
  }
  __syncthreads();
  double2* Qb = reinterpret_cast<double2*>(Qbuf) + b * (long)n * PNB;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int i = lane + 64 * q;
    if (i < n) {
      if (c < n) M[i + (long)n * c] = v[q];
      Qb[i + (long)n * w] = (c < n) ? v[q] : cmk(0, 0);
    }
  }
  // rows that became pivots in this panel
  if (w == 0) {
    for (int s = lane; s < PNB; s += 64)
      if (k0 + s < n) us[s_piv[s]] = 1;
  }
  // pivot rows X = M[P_K, :] (zero on the panel columns) for the update M += Q X, and
  // clear those rows outside the panel
  __syncthreads();
  double2* X = reinterpret_cast<double2*>(Xbuf) + b * (long)n * PNB;
  for (long e = threadIdx.x; e < (long)PNB * n; e += blockDim.x) {
    const int k = e % PNB, j = e / PNB;
    double2 val = cmk(0, 0);
    if (k0 + k < n && (j < k0 || j >= k0 + PNB)) {
      const int r = s_piv[k];
      val = M[r + (long)n * j];
      M[r + (long)n * j] = cmk(0, 0);
    }
    X[k + (long)PNB * j] = val;
  }
}

__global__ void zinv_permute_kernel(int n, const double* Mg, const int* piv, double* Out,
                                    long ldo, long sO, const int* info) {
  extern __shared__ int ip_s[];
  const long b = blockIdx.y;
  if (info[b]) return;
  const int* pv = piv + b * (long)n;
  for (int k = threadIdx.x; k < n; k += blockDim.x) ip_s[pv[k]] = k;
  __syncthreads();
  const double2* M = reinterpret_cast<const double2*>(Mg) + b * (long)n * n;
  double2* O = reinterpret_cast<double2*>(Out) + b * sO;
  // this block handles a range of output columns
  const int cols_per_block = (n + gridDim.x - 1) / gridDim.x;
  const int j0 = blockIdx.x * cols_per_block;
  const int j1 = min(n, j0 + cols_per_block);
  for (int j = j0; j < j1; ++j) {
    const long src_col = (long)n * ip_s[j];
    for (int k = threadIdx.x; k < n; k += blockDim.x) O[k + ldo * j] = M[pv[k] + src_col];
  }
}

__global__ void copy_in_kernel(int n, const double* A, long lda, long sA, double* M) {
  const long b = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = e % n, j = e / n;
  reinterpret_cast<double2*>(M)[b * (long)n * n + e] =
      reinterpret_cast<const double2*>(A)[b * sA + i + lda * j];
}

__global__ void zero_int_kernel(int* p, long cnt) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) p[e] = 0;
}

template <int Q>
void launch_panel(int n, int batch, double* M, int k0, double* Qb, double* Xb, int* piv,
                  int* used, int* info, hipStream_t st) {
  hipLaunchKernelGGL(zinv_panel_kernel<Q>, dim3(batch), dim3(1024), 0, st, n, M, k0, Qb, Xb,
                     piv, used, info);
}

}  // namespace

size_t zinv_workspace_bytes(int n, int batch) {
  if (n <= SMALL_MAX) return 0;
  size_t nn = (size_t)n * n * 16;
  size_t q = (size_t)n * PNB * 16;
  size_t x = (size_t)n * PNB * 16;
  size_t ints = (size_t)n * 4 * 2;
  return (size_t)batch * (nn + q + x + ints) + 256;
}

void zinv(int n, int batch, const double* A, long lda, long sA, double* Out, long ldo,
          long sO, int* info, void* work, hipStream_t st) {
  if (n <= 0 || batch <= 0) return;
  if (batch > 65535) throw Error(1, "zinv: batch exceeds grid limit");
  if (n <= SMALL_MAX) {
    size_t shm = (size_t)n * n * 16 + (size_t)n * 12;
    hipLaunchKernelGGL(zinv_small_kernel, dim3(batch), dim3(256), shm, st, n, A, lda, sA, Out,
                       ldo, sO, info);
    HPS_LAUNCH_CHECK();
    return;
  }
  if (n > 64 * 32) throw Error(1, "zinv: n too large (max 2048)");
  char* w = static_cast<char*>(work);
  double* M = reinterpret_cast<double*>(w);
  w += (size_t)batch * n * n * 16;
  double* Qb = reinterpret_cast<double*>(w);
  w += (size_t)batch * n * PNB * 16;
  double* Xb = reinterpret_cast<double*>(w);
  w += (size_t)batch * n * PNB * 16;
  int* piv = reinterpret_cast<int*>(w);
  int* used = piv + (size_t)batch * n;
  {
    long tot = (long)n * n;
    hipLaunchKernelGGL(copy_in_kernel, dim3(cdiv(tot, 256), batch), dim3(256), 0, st, n, A, lda,
                       sA, M);
    long ni = 2L * batch * n;
    hipLaunchKernelGGL(zero_int_kernel, dim3(cdiv(ni, 256)), dim3(256), 0, st, piv, ni);
    HPS_LAUNCH_CHECK();
  }
  const int Qr = (n + 63) / 64;
  for (int k0 = 0; k0 < n; k0 += PNB) {
    if (Qr <= 2) launch_panel<2>(n, batch, M, k0, Qb, Xb, piv, used, info, st);
    else if (Qr <= 4) launch_panel<4>(n, batch, M, k0, Qb, Xb, piv, used, info, st);
    else if (Qr <= 8) launch_panel<8>(n, batch, M, k0, Qb, Xb, piv, used, info, st);
    else if (Qr <= 16) launch_panel<16>(n, batch, M, k0, Qb, Xb, piv, used, info, st);
    else if (Qr <= 28) launch_panel<28>(n, batch, M, k0, Qb, Xb, piv, used, info, st);
    else launch_panel<32>(n, batch, M, k0, Qb, Xb, piv, used, info, st);
    HPS_LAUNCH_CHECK();
    GemmDesc g;
    g.M = n; g.N = n; g.K = PNB; g.batch = batch;
    g.A = Qb; g.lda = n; g.sA = (long)n * PNB;
    g.B = Xb; g.ldb = PNB; g.sB = (long)n * PNB;
    g.C = M; g.ldc = n; g.sC = (long)n * n;
    g.alpha = 1.0; g.beta = 1.0;
    zgemm(g, st);
  }
  int blocks_x = std::min(n, 64);
  hipLaunchKernelGGL(zinv_permute_kernel, dim3(blocks_x, batch), dim3(256), n * sizeof(int), st,
                     n, M, piv, Out, ldo, sO, info);
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
