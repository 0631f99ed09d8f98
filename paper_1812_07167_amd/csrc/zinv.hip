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
//   kernel (one workgroup per matrix, panel rows spread over its waves, each row's
//   16 panel entries in registers) runs the 16 elimination steps on the panel and emits the block
//   transformation Q; an extract kernel gathers the pivot rows X = M[P_K, :] (zero on
//   K) and clears them; a batched MFMA GEMM then applies M += Q X to every column.
#include "kernels.hpp"

namespace hps {
namespace {

constexpr int SMALL_MAX = 96;
constexpr int PNB = 8;   // panel width of the blocked path

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
      const int r = wave_argmax(best, bi);
      if (tid == 0) {
        s_r = r < 0 ? 0 : r;
        if (r < 0) s_bad = k + 1;
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
// Panel of the blocked path: the n x 16 panel (columns k0..k0+15) of one matrix, rows
// distributed over the (at most 8) waves of the workgroup (row i: wave i / (64 RPL), slot
// (i / 64) % RPL, lane i % 64), all 16 panel columns of a row in the owning lane's
// registers.  Per elimination step: every wave offers its best unused row of the pivot
// column (DPP reduction), the winner is found from the per-wave candidates in LDS, the
// owner publishes the pivot row (16 entries), and every lane updates its own rows:
//     M[i][c] -= f_i M[r][c],  f_i = M[i][k]/p  (f_r = 1 - 1/p, so the pivot row
//     becomes M[r][c]/p),   and column k becomes -f_i (1/p on the pivot row).
// Two barriers per step; nothing but the pivot row goes through LDS.
template <int RPL>
__global__ __launch_bounds__(512) void zinv_panel_kernel(int n, double* Mg, int k0,
                                                         double* Qbuf, int* piv, int* used,
                                                         int* info) {
  __shared__ unsigned s_key[8];
  __shared__ int s_row[8];
  __shared__ double2 prow[PNB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const long b = blockIdx.x;
  double2* M = reinterpret_cast<double2*>(Mg) + b * (long)n * n;
  int* pv = piv + b * (long)n;
  int* us = used + b * (long)n;
  const int nk = (n - k0) < PNB ? (n - k0) : PNB;
  double2 v[RPL][PNB];
  unsigned umask = 0;  // bit q: row of slot q is used (or beyond n)
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int i = (w * RPL + q) * 64 + lane;
    const bool ok = i < n;
    if (!ok || us[i]) umask |= 1u << q;
#pragma unroll
    for (int c = 0; c < PNB; ++c)
      v[q][c] = (ok && c < nk) ? M[i + (long)n * (k0 + c)] : cmk(0, 0);
  }
  int bad = 0;
#pragma unroll
  for (int s = 0; s < PNB; ++s) {
    if (s >= nk || bad) continue;  // uniform over the workgroup; keeps the loop unrolled
    const int k = k0 + s;
    // candidate of this wave
    double best = -1.0;
    int bi = 0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const double val = ((umask >> q) & 1u) ? -1.0 : cabs1(v[q][s]);
      if (val > best) { best = val; bi = (w * RPL + q) * 64 + lane; }
    }
    {
      const unsigned key = best > 0.0 ? max(__float_as_uint((float)best), 1u) : 0u;
      const unsigned wkey = wave_max_u32(key);
      const unsigned long long hit = __ballot(key == wkey);
      const int src = __builtin_ctzll(hit);
      const int wrow = __builtin_amdgcn_readlane(bi, src);
      if (lane == 0) { s_key[w] = wkey; s_row[w] = wrow; }
    }
    __syncthreads();
    // winner over the waves
    int r;
    {
      const unsigned key = lane < nw ? s_key[lane] : 0u;
      const int row = lane < nw ? s_row[lane] : 0;
      const unsigned gkey = wave_max_u32(key);
      if (gkey == 0u) {
        r = -1;
      } else {
        const unsigned long long hit = __ballot(key == gkey);
        r = __builtin_amdgcn_readlane(row, __builtin_ctzll(hit));
      }
    }
    if (r < 0) {
      bad = k + 1;
      continue;
    }
    // the owner publishes the pivot row
    const int rw = r / (64 * RPL), rq = (r / 64) % RPL, rl = r & 63;
    if (w == rw && lane == rl) {
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if (q == rq)
#pragma unroll
          for (int c = 0; c < PNB; ++c) prow[c] = v[q][c];
    }
    __syncthreads();
    const double2 ip = crcp(prow[s]);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = (w * RPL + q) * 64 + lane;
      const bool isr = (i == r);
      const double2 f0 = cmul(v[q][s], ip);
      const double2 f = isr ? cmk(1.0 - ip.x, -ip.y) : f0;
#pragma unroll
      for (int c = 0; c < PNB; ++c) {
        if (c == s) continue;
        const double2 pc = prow[c];  // LDS broadcast read
        v[q][c].x = fma(-f.x, pc.x, fma(f.y, pc.y, v[q][c].x));
        v[q][c].y = fma(-f.x, pc.y, fma(-f.y, pc.x, v[q][c].y));
        // bound the scheduler's look-ahead: hoisting every pivot-row read of the
        // unrolled steps would need more registers than a 16-wave workgroup has
        if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
      v[q][s] = isr ? ip : cmk(-f0.x, -f0.y);
      if (isr) umask |= 1u << q;
    }
    if (threadIdx.x == 0) pv[k] = r;
  }
  if (bad) {
    if (threadIdx.x == 0) info[b] = bad;
    return;
  }
  // write the panel back (it now holds Q) and keep a copy for the update GEMM.  The
  // column stride is re-read through an empty asm so that these addresses are formed
  // here instead of being kept live from the loads at the top (which costs registers).
  long ld = n;
  asm volatile("" : "+s"(ld));
  double2* Mw = reinterpret_cast<double2*>(Mg) + b * ld * ld;
  double2* Qb = reinterpret_cast<double2*>(Qbuf) + b * ld * PNB;
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int i = (w * RPL + q) * 64 + lane;
    if (i < n) {
#pragma unroll
      for (int c = 0; c < PNB; ++c) {
        if (c < nk) Mw[i + ld * (k0 + c)] = v[q][c];
        Qb[i + ld * c] = c < nk ? v[q][c] : cmk(0, 0);
      }
      if ((umask & 1u << q) && !us[i]) us[i] = 1;
    }
  }
}

// X = M[P_K, :] (zero on the panel columns), and those rows cleared outside the panel.
__global__ void zinv_extract_kernel(int n, double* Mg, int k0, double* Xg, const int* piv,
                                    const int* info) {
  const long b = blockIdx.y;
  if (info[b]) return;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)PNB * n) return;
  const int k = e % PNB, j = e / PNB;
  double2* M = reinterpret_cast<double2*>(Mg) + b * (long)n * n;
  double2* X = reinterpret_cast<double2*>(Xg) + b * (long)PNB * n;
  double2 val = cmk(0, 0);
  if (k0 + k < n && (j < k0 || j >= k0 + PNB)) {
    const int r = piv[b * (long)n + k0 + k];
    val = M[r + (long)n * j];
    M[r + (long)n * j] = cmk(0, 0);
  }
  X[k + (long)PNB * j] = val;
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

template <int RPL>
void launch_panel(int n, int batch, double* M, int k0, double* Qb, int* piv, int* used,
                  int* info, hipStream_t st) {
  const int waves = std::max(1, std::min(8, (n + 64 * RPL - 1) / (64 * RPL)));
  hipLaunchKernelGGL(zinv_panel_kernel<RPL>, dim3(batch), dim3(64 * waves), 0, st, n, M, k0, Qb,
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
  for (int k0 = 0; k0 < n; k0 += PNB) {
    if (n <= 512) launch_panel<1>(n, batch, M, k0, Qb, piv, used, info, st);
    else if (n <= 1024) launch_panel<2>(n, batch, M, k0, Qb, piv, used, info, st);
    else launch_panel<4>(n, batch, M, k0, Qb, piv, used, info, st);
    HPS_LAUNCH_CHECK();
    {
      const long tot = (long)PNB * n;
      hipLaunchKernelGGL(zinv_extract_kernel, dim3(cdiv(tot, 256), batch), dim3(256), 0, st, n,
                         M, k0, Xb, piv, info);
      HPS_LAUNCH_CHECK();
    }
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
