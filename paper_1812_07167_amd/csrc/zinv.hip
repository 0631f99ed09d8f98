// Batched complex matrix inversion by Gauss-Jordan elimination with partial pivoting
// (the explicit W^{-1} of the merge, Sec. 2.2 / Sec. 2.4, and the leaf's boundary
// Schur complement).
//
// Pivoting is implicit: the pivot of column k is the unused row r_k of largest
// |re|+|im|; rows are never moved.  After all n steps the in-place matrix M satisfies
// inv(A)[k][r_j] = M[r_k][j], which the final write-out applies.
//
// * n <= SMALL_MAX: one workgroup per matrix, matrix resident in registers.
// * larger n, by default: blocked Gauss-Jordan with the diagonal blocks of BNB columns as
//   pivots (each block inverted in LDS with its own 16 x 16 diagonal blocks as pivots),
//   the block transformations applied by the matrix-core GEMM.  The interface matrices
//   W = I - R33^b R33^a of the merge are identity minus a product of two compressions of
//   ItI operators (contractions in the boundary quadrature norm for real c and eta), so
//   the elimination needs no row exchanges (the measured growth of their entries is at
//   most 3); a zero pivot, or growth past a bound, is reported, and the build then
//   repeats with the fully pivoted form.
// * larger n, fully pivoted (the fallback): blocked right-looking form.  For each block K
//   of PNB (16 or 8) columns a panel kernel (one workgroup per matrix, panel rows spread
//   over its waves, each row's PNB panel entries in registers) runs the PNB elimination
//   steps on the panel and emits the block transformation Q; an update kernel then forms
//   M = (pivot rows of K cleared) + Q M[P_K, :] on every column outside K.
#include "kernels.hpp"

namespace hps {
namespace {

constexpr int SMALL_MAX = 64;  // the small kernel: a row per lane, 4 x 16 columns

// ------------------------------------------------------------------ small (registers)
// n <= SMALL_MAX: one workgroup of 4 waves per matrix, the matrix in registers.  Wave w
// holds the columns c = w + 4 j (j < NJ) of every row; row i sits in lane i.  For step
// k the wave that holds column k picks the pivot (the unused row of
// largest |re| + |im|, a wave reduction) and publishes r and column k through LDS; after
// one barrier every wave reads the pivot row's values of its own columns from lane r
// (readlane) and updates its rows:  M[i][c] -= (M[i][k] / p) M[r][c],  the pivot row
// becomes M[r][c] / p,  and column k becomes -M[i][k] / p (1 / p on the pivot row).
// Column k and r are double-buffered by the parity of k, so one barrier per step
// suffices.
__device__ inline double2 readlane_c(double2 v, int lane) {
  return make_double2(readlane_f64(v.x, lane), readlane_f64(v.y, lane));
}
__device__ inline float2 readlane_c(float2 v, int lane) {
  return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), lane)),
                     __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), lane)));
}

template <class T, int NJ>
__global__ __launch_bounds__(256) void zinv_small_kernel(int n, const double* Ain, long lda,
                                                         long sA, double* Out, long ldo,
                                                         long sO, int* info) {
  typedef typename Cx<T>::t C2;
  __shared__ C2 colv[2][64];
  __shared__ int s_r[2];
  __shared__ int piv[64], ipiv[64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const long b = blockIdx.x;
  const C2* A = reinterpret_cast<const C2*>(Ain) + b * sA;
  const int i = lane;  // this lane's row
  C2 M[NJ];
  bool used = i >= n;  // a pivot row already, or beyond n
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int c = wv + 4 * j;
    M[j] = (i < n && c < n) ? A[i + lda * c] : Cx<T>::mk(0, 0);
  }
  // step k = 4 jk + wk: column k is slot jk of wave wk (the slot loop is unrolled so
  // that every register index is a constant)
  int bad = 0;
#pragma unroll
  for (int jk = 0; jk < NJ; ++jk) {
#pragma unroll 1
    for (int wk = 0; wk < 4; ++wk) {
      const int k = 4 * jk + wk;
      if (k >= n || bad) break;  // uniform over the workgroup
      const int sb = k & 1;
      if (wv == wk) {
        if (i < n) colv[sb][i] = M[jk];
        const int r = wave_argmax(used ? -1.0 : (double)cabs1(M[jk]), i);
        if (lane == 0) s_r[sb] = r;
      }
      __syncthreads();
      const int r = s_r[sb];
      if (r < 0) {  // no nonzero entry left in column k: singular
        bad = k + 1;
        break;
      }
      // (one division: the pivot is its column's largest entry, so |p|^2 stays in range
      // unless the matrix's own scale is extreme, and then the guarded form falls back)
      const C2 ip = crcp_pivot(colv[sb][r]);
      // the pivot row's values in this wave's columns, read before this step's updates
      C2 pr[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) pr[j] = readlane_c(M[j], r);
      if (i == r) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) M[j] = cmul(M[j], ip);
        used = true;
        if (wv == wk) M[jk] = ip;
      } else if (i < n) {
        const C2 f = cmul(colv[sb][i], ip);
#pragma unroll
        for (int j = 0; j < NJ; ++j) M[j] = csub(M[j], cmul(f, pr[j]));
        if (wv == wk) M[jk] = Cx<T>::mk(-f.x, -f.y);
      }
      if (tid == 0) piv[k] = r;
    }
  }
  if (bad) {
    if (tid == 0) info[b] = bad;
    return;
  }
  __syncthreads();
  for (int k = tid; k < n; k += 256) ipiv[piv[k]] = k;
  __syncthreads();
  // inv[ipiv[i]][piv[c]] = M[i][c]
  C2* O = reinterpret_cast<C2*>(Out) + b * sO;
  if (i < n) {
    const long oi = ipiv[i];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int c = wv + 4 * j;
      if (c < n) O[oi + ldo * (long)piv[c]] = M[j];
    }
  }
}

// ------------------------------------------------------------------ blocked
// The blocked path keeps two copies of every matrix and alternates between them: block
// K reads the current copy and writes the next one (the panel kernel writes the block
// transformation Q into the next copy's panel columns, the update kernel every other
// column).  The update can then read the pivot rows of the current copy directly, with
// no gather pass and no race between workgroups.
//
// Panel kernel: the n x PNB panel (columns k0..k0+PNB-1) of one matrix, rows
// distributed over the (at most NW, 8 or 16) waves of the workgroup (row i: wave i / (64 RPL),
// slot (i / 64) % RPL, lane i % 64), all PNB panel columns of a row in the owning lane's
// registers.  For elimination step s every wave publishes its best unused row of column
// s (DPP reduction): key, row index and the row's PNB values, in an LDS slot; after one
// barrier every lane picks the winner among the slots and reads the pivot row from it.
// Each lane then updates its own rows,
//     M[i][c] -= f_i M[r][c],  f_i = M[i][k]/p  (f_r = 1 - 1/p, so the pivot row
//     becomes M[r][c]/p),   and column k becomes -f_i (1/p on the pivot row),
// updating column s+1 first so that the next step's pivot search overlaps the update of
// the remaining columns (the candidate row's values are published once final).  The slots alternate between two buffers, so one
// barrier per step suffices: a wave can only overwrite a buffer after every wave has
// passed the following step's barrier.
template <class T, int RPL, int PNB, int NW>
__global__ __launch_bounds__(64 * NW) void zinv_panel_kernel(int n, const double* Mcur,
                                                             double* Mnext, int k0, int* piv,
                                                             int* used, int* info) {
  typedef typename Cx<T>::t C2;
  __shared__ unsigned s_key[2][NW];
  __shared__ int s_row[2][NW];
  __shared__ C2 s_val[2][NW][PNB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const long b = blockIdx.x;
  if (info[b]) return;
  const C2* M = reinterpret_cast<const C2*>(Mcur) + b * (long)n * n;
  int* pv = piv + b * (long)n;
  int* us = used + b * (long)n;
  const int nk = (n - k0) < PNB ? (n - k0) : PNB;
  C2 v[RPL][PNB];
  unsigned umask = 0;  // bit q: row of slot q is used (or beyond n)
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int i = (w * RPL + q) * 64 + lane;
    const bool ok = i < n;
    if (!ok || us[i]) umask |= 1u << q;
#pragma unroll
    for (int c = 0; c < PNB; ++c)
      v[q][c] = (ok && c < nk) ? M[i + (long)n * (k0 + c)] : Cx<T>::mk(0, 0);
  }
  // this wave's candidate for column s: key and row into slot buffer sb (the row's
  // values follow with publish_row once they are final)
  int psrc = 0, pbrow = 0;
  auto publish_key = [&](int s, int sb) {
    double best = -1.0;
    int brow = 0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const double val = ((umask >> q) & 1u) ? -1.0 : cabs1(v[q][s]);
      if (val > best) { best = val; brow = (w * RPL + q) * 64 + lane; }
    }
    const unsigned key = best > 0.0 ? max(__float_as_uint((float)best), 1u) : 0u;
    const unsigned wkey = wave_max_u32(key);
    psrc = __builtin_ctzll(__ballot(key == wkey));
    pbrow = brow;
    if (lane == psrc) {
      s_key[sb][w] = wkey;
      s_row[sb][w] = brow;
    }
  };
  auto publish_row = [&](int sb) {
    if (lane == psrc) {
      // select the slot by its row index (a compare the compiler cannot turn into a
      // dynamically indexed register array)
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if ((w * RPL + q) * 64 + lane == pbrow)
#pragma unroll
          for (int c = 0; c < PNB; ++c) s_val[sb][w][c] = v[q][c];
    }
  };
  publish_key(0, 0);
  publish_row(0);
  // Every step runs (no branch around the updates, which would keep a second copy of
  // the panel live at each join): a step past the panel's end, or one with no nonzero
  // candidate (singular; reported at the end), takes the multiplier 0 and changes no
  // column that is written out.
  int bad = 0;
#pragma unroll
  for (int s = 0; s < PNB; ++s) {
    const int k = k0 + s;
    const int sb = s & 1;
    const bool live = s < nk;  // uniform over the workgroup
    __syncthreads();
    // winner over the waves (ties to the lowest wave): lane x reads wave x's key
    const unsigned kx = lane < nw ? s_key[sb][lane] : 0u;
    const unsigned gkey = wave_max_u32(kx);
    const int ww = __builtin_ctzll(__ballot(kx == gkey));
    const bool go = live && gkey != 0u;
    if (live && gkey == 0u && !bad) bad = k + 1;
    const int r = go ? s_row[sb][ww] : -1;
    const C2 ip = go ? crcp_fast(s_val[sb][ww][s]) : Cx<T>::mk(0, 0);
    C2 f[RPL], f0[RPL];
    bool isr[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = (w * RPL + q) * 64 + lane;
      isr[q] = (i == r);
      f0[q] = cmul(v[q][s], ip);
      f[q] = isr[q] ? Cx<T>::mk(T(1) - ip.x, -ip.y) : f0[q];
      if (isr[q]) umask |= 1u << q;
    }
    auto upd = [&](int c) {
      const C2 pc = s_val[sb][ww][c];  // LDS broadcast read
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        v[q][c].x = fma(-f[q].x, pc.x, fma(f[q].y, pc.y, v[q][c].x));
        v[q][c].y = fma(-f[q].x, pc.y, fma(-f[q].y, pc.x, v[q][c].y));
      }
    };
    if (s + 1 < PNB) {
      upd(s + 1);
      publish_key(s + 1, sb ^ 1);
    }
#pragma unroll
    for (int c = 0; c < PNB; ++c) {
      if (c == s || c == s + 1) continue;
      upd(c);
      // bound the scheduler's look-ahead: hoisting every pivot-row read of the
      // unrolled steps would need more registers than the workgroup has
      if ((c & 1) == 1) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) v[q][s] = isr[q] ? ip : Cx<T>::mk(-f0[q].x, -f0[q].y);
    if (s + 1 < PNB) publish_row(sb ^ 1);
    if (live && threadIdx.x == 0) pv[k] = r;
  }
  if (bad) {
    if (threadIdx.x == 0) info[b] = bad;
    return;
  }
  // the panel (now Q) goes into the next copy.  The column stride is re-read through an
  // empty asm so that these addresses are formed here instead of being kept live from
  // the loads at the top (which costs registers).
  long ld = n;
  asm volatile("" : "+s"(ld));
  C2* Mw = reinterpret_cast<C2*>(Mnext) + b * ld * ld;
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int i = (w * RPL + q) * 64 + lane;
    if (i < n) {
#pragma unroll
      for (int c = 0; c < PNB; ++c)
        if (c < nk) Mw[i + ld * (k0 + c)] = v[q][c];
      if ((umask & 1u << q) && !us[i]) us[i] = 1;
    }
  }
}

// Block update, for every column j outside the panel K:
//     next[i][j] = (i a pivot row of K ? 0 : cur[i][j]) + sum_s Q[i][s] cur[r_s][j],
// with Q = next[:, K] (written by the panel kernel) and r_s the pivot rows of K.
// Memory-bound (PNB complex multiply-adds per element read and written).  A workgroup
// covers 64 rows (one per lane) and UJ consecutive columns (UJ / 4 per wave) of one
// matrix.  Its 64 rows of Q and the pivot rows' entries on its columns are staged in LDS
// with every global load issued at once; the terms are then added in order from LDS.
constexpr int UJ = 16;
template <class T, int PNB>
__global__ __launch_bounds__(256) void zinv_update_kernel(int n,
                                                          const double* __restrict__ Mcur,
                                                          double* __restrict__ Mnext, int k0,
                                                          const int* piv, const int* info) {
  typedef typename Cx<T>::t C2;
  constexpr int CW = UJ / 4;  // columns per wave
  __shared__ C2 s_p[PNB][UJ];
  __shared__ C2 s_q[PNB][64];
  const long b = blockIdx.z;
  if (info[b]) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 64, i = i0 + lane;
  const int nk = (n - k0) < PNB ? (n - k0) : PNB;
  // columns outside the panel, compacted: column index jj skips [k0, k0 + nk)
  const int ncol = n - nk;
  const int jb = blockIdx.y * UJ, jj0 = jb + w * CW;
  const C2* Mc = reinterpret_cast<const C2*>(Mcur) + b * (long)n * n;
  C2* Mn = reinterpret_cast<C2*>(Mnext) + b * (long)n * n;
  const int* pv = piv + b * (long)n + k0;
  const bool mine = i < n && jj0 < ncol;
  bool isp = false;
#pragma unroll
  for (int s = 0; s < PNB; ++s) isp |= (s < nk && pv[s] == i);
  C2 acc[CW];
  int col[CW];
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int jj = min(jj0 + c, ncol - 1);
    col[c] = jj < k0 ? jj : jj + nk;
    acc[c] = (mine && !isp) ? Mc[min(i, n - 1) + (long)n * col[c]] : Cx<T>::mk(0, 0);
  }
  // Q rows i0..i0+63 (coalesced), then the pivot rows on this workgroup's columns
  constexpr int QPT = PNB * 64 / 256;
  C2 qv[QPT];
#pragma unroll
  for (int e = 0; e < QPT; ++e) {
    const int t = threadIdx.x + 256 * e, s = t >> 6, r = i0 + (t & 63);
    qv[e] = (s < nk && r < n) ? Mn[r + (long)n * (k0 + s)] : Cx<T>::mk(0, 0);
  }
  constexpr int PPT = (PNB * UJ + 255) / 256;
  C2 pvv[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int t = threadIdx.x + 256 * e, s = t / UJ;
    const int jj = min(jb + t % UJ, ncol - 1);
    const int cc = jj < k0 ? jj : jj + nk;
    pvv[e] = (t < PNB * UJ && s < nk) ? Mc[pv[s] + (long)n * cc] : Cx<T>::mk(0, 0);
  }
#pragma unroll
  for (int e = 0; e < QPT; ++e) {
    const int t = threadIdx.x + 256 * e;
    s_q[t >> 6][t & 63] = qv[e];
  }
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int t = threadIdx.x + 256 * e;
    if (t < PNB * UJ) s_p[t / UJ][t % UJ] = pvv[e];
  }
  __syncthreads();
  if (!mine) return;
#pragma unroll 4
  for (int s = 0; s < nk; ++s) {
    const C2 q = s_q[s][lane];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = cfma(q, s_p[s][w * CW + c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < CW; ++c)
    if (jj0 + c < ncol) Mn[i + (long)n * col[c]] = acc[c];
}

template <class T>
__global__ void zinv_permute_kernel(int n, const double* Mg, const int* piv, double* Out,
                                    long ldo, long sO, const int* info) {
  typedef typename Cx<T>::t C2;
  extern __shared__ int ip_s[];
  const long b = blockIdx.y;
  if (info[b]) return;
  const int* pv = piv + b * (long)n;
  for (int k = threadIdx.x; k < n; k += blockDim.x) ip_s[pv[k]] = k;
  __syncthreads();
  const C2* M = reinterpret_cast<const C2*>(Mg) + b * (long)n * n;
  C2* O = reinterpret_cast<C2*>(Out) + b * sO;
  // this block handles a range of output columns
  const int cols_per_block = (n + gridDim.x - 1) / gridDim.x;
  const int j0 = blockIdx.x * cols_per_block;
  const int j1 = min(n, j0 + cols_per_block);
  for (int j = j0; j < j1; ++j) {
    const long src_col = (long)n * ip_s[j];
    for (int k = threadIdx.x; k < n; k += blockDim.x) O[k + ldo * j] = M[pv[k] + src_col];
  }
}

template <class T>
__global__ void copy_in_kernel(int n, const double* A, long lda, long sA, double* M) {
  typedef typename Cx<T>::t C2;
  const long b = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = e % n, j = e / n;
  reinterpret_cast<C2*>(M)[b * (long)n * n + e] =
      reinterpret_cast<const C2*>(A)[b * sA + i + lda * j];
}

__global__ void zero_int_kernel(int* p, long cnt) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
       e += (long)gridDim.x * blockDim.x)
    p[e] = 0;
}

template <class T, int RPL, int PNB, int NW>
void launch_panel(int n, int batch, const double* Mc, double* Mn, int k0, int* piv, int* used,
                  int* info, hipStream_t st) {
  const int waves = std::max(1, std::min(NW, (n + 64 * RPL - 1) / (64 * RPL)));
  hipLaunchKernelGGL((zinv_panel_kernel<T, RPL, PNB, NW>), dim3(batch), dim3(64 * waves), 0, st,
                     n, Mc, Mn, k0, piv, used, info);
}

// One block step of the blocked path: panel columns [k0, k0 + PNB), then the update of
// every other column.
template <class T, int RPL, int PNB, int NW>
void block_step(int n, int batch, const double* Mc, double* Mn, int k0, int* piv, int* used,
                int* info, hipStream_t st) {
  launch_panel<T, RPL, PNB, NW>(n, batch, Mc, Mn, k0, piv, used, info, st);
  HPS_LAUNCH_CHECK();
  const int ncol = n - std::min(PNB, n - k0);
  if (ncol > 0) {
    hipLaunchKernelGGL((zinv_update_kernel<T, PNB>), dim3(cdiv(n, 64), cdiv(ncol, UJ), batch),
                       dim3(256), 0, st, n, Mc, Mn, k0, piv, info);
    HPS_LAUNCH_CHECK();
  }
}

template <class T>
void zinv_t(int n, int batch, const double* A, long lda, long sA, double* Out, long ldo,
            long sO, int* info, void* work, hipStream_t st) {
  typedef typename Cx<T>::t C2;
  if (n <= SMALL_MAX) {
    // columns per wave: n / 4 rounded up to the instantiated widths
    if (n <= 16)
      hipLaunchKernelGGL((zinv_small_kernel<T, 4>), dim3(batch), dim3(256), 0, st, n, A, lda, sA,
                         Out, ldo, sO, info);
    else if (n <= 32)
      hipLaunchKernelGGL((zinv_small_kernel<T, 8>), dim3(batch), dim3(256), 0, st, n, A, lda, sA,
                         Out, ldo, sO, info);
    else
      hipLaunchKernelGGL((zinv_small_kernel<T, 16>), dim3(batch), dim3(256), 0, st, n, A, lda, sA,
                         Out, ldo, sO, info);
    HPS_LAUNCH_CHECK();
    return;
  }
  if (n > 64 * 32) throw Error(1, "zinv: n too large (max 2048)");
  char* w = static_cast<char*>(work);
  double* Mcur = reinterpret_cast<double*>(w);
  w += (size_t)batch * n * n * sizeof(C2);
  double* Mnext = reinterpret_cast<double*>(w);
  w += (size_t)batch * n * n * sizeof(C2);
  int* piv = reinterpret_cast<int*>(w);
  int* used = piv + (size_t)batch * n;
  {
    long tot = (long)n * n;
    hipLaunchKernelGGL(copy_in_kernel<T>, dim3(cdiv(tot, 256), batch), dim3(256), 0, st, n, A,
                       lda, sA, Mcur);
    long ni = 2L * batch * n;
    hipLaunchKernelGGL(zero_int_kernel, dim3(grid1d(ni)), dim3(256), 0, st, piv, ni);
    HPS_LAUNCH_CHECK();
  }
  // panel shape: a lane holds one panel row of 16 columns (n <= 512), two rows of 8
  // (n <= 2048), with 8 waves up to n = 1024 and 16 above.  A panel step's work grows
  // with the panel width on the one compute unit that runs it, the update's passes over
  // the matrix shrink with it; these widths measured fastest.
  const int pnb = n <= 512 ? 16 : 8;
  for (int k0 = 0; k0 < n; k0 += pnb) {
    if (n <= 512) block_step<T, 1, 16, 8>(n, batch, Mcur, Mnext, k0, piv, used, info, st);
    else if (n <= 1024) block_step<T, 2, 8, 8>(n, batch, Mcur, Mnext, k0, piv, used, info, st);
    else block_step<T, 2, 8, 16>(n, batch, Mcur, Mnext, k0, piv, used, info, st);
    std::swap(Mcur, Mnext);
  }
  int blocks_x = std::min(n, 64);
  hipLaunchKernelGGL(zinv_permute_kernel<T>, dim3(blocks_x, batch), dim3(256), n * sizeof(int),
                     st, n, Mcur, piv, Out, ldo, sO, info);
  HPS_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ block pivots
// One block step of the block-pivot form, after P^{-1} (Pinv, nb x nb per matrix) and
// Q = -M[:, K] P^{-1} (n x nb per matrix) are formed: Q's rows K take P^{-1}; the block's
// rows go to X = M[K, :] (nb x n, the identity on the columns K) and are zeroed in M, and
// M's columns K are zeroed, so that the update M += Q X completes the step.  A thread's
// element belongs to exactly one of the three index sets.
template <class T>
__global__ __launch_bounds__(256) void zinv_bstep_kernel(int n, int nb, int k0, double* Mg,
                                                         long ld, long sM, const double* Pinv,
                                                         double* Qg, double* Xg,
                                                         const int* info) {
  typedef typename Cx<T>::t C2;
  const long b = blockIdx.y;
  if (info[b]) return;
  C2* M = reinterpret_cast<C2*>(Mg) + b * sM;
  const C2* Pi = reinterpret_cast<const C2*>(Pinv) + b * (long)nb * nb;
  C2* Q = reinterpret_cast<C2*>(Qg) + b * (long)n * nb;
  C2* X = reinterpret_cast<C2*>(Xg) + b * (long)nb * n;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nq = (long)nb * nb, nx = (long)nb * n, nz = (long)n * nb;
  if (e < nq) {  // Q's rows K
    const int r = (int)(e % nb), j = (int)(e / nb);
    Q[(k0 + r) + (long)n * j] = Pi[r + (long)nb * j];
  } else if (e < nq + nx) {  // X and the rows K of M
    const long f = e - nq;
    const int r = (int)(f % nb), c = (int)(f / nb);
    const int jc = c - k0;
    const long at = (k0 + r) + ld * c;
    X[r + (long)nb * c] = (jc >= 0 && jc < nb) ? Cx<T>::mk(jc == r ? 1 : 0, 0) : M[at];
    M[at] = Cx<T>::mk(0, 0);
  } else if (e < nq + nx + nz) {  // the columns K of M
    const long f = e - nq - nx;
    const int r = (int)(f % n), j = (int)(f / n);
    M[r + ld * (k0 + j)] = Cx<T>::mk(0, 0);
  }
}

// Inverse of the n x n diagonal block P of a matrix (n <= 64) with its own 16 x 16
// diagonal blocks as pivots: one workgroup of 1024 threads (16 waves) per matrix, P in
// LDS; the block transformations and updates spread over all of them.  Per
// block K of 16 columns, the first wave inverts P[K, K] by Gauss-Jordan in LDS, then
// Q = -P[:, K] P[K, K]^{-1} (rows K: P[K, K]^{-1}) and X = P[K, :] (identity on K), and
// P <- (rows K and columns K zeroed) + Q X.  A zero or non-finite pivot, or an entry of
// the inverse beyond 1e12 times the largest of P, sets info (the build then repeats with
// full pivoting).
template <class T>
__global__ __launch_bounds__(1024) void zinv_np_kernel(int n, const double* Ain, long lda,
                                                      long sA, double* Out, long ldo, long sO,
                                                      int* info) {
  typedef typename Cx<T>::t C2;
  constexpr int LD = 65;         // column stride of the LDS copy (odd: no bank pattern)
  __shared__ C2 Ms[64 * LD];     // Ms[c * LD + r] = P[r][c], padded with the identity
  __shared__ C2 Qs[16 * 64];     // Qs[t * 64 + r] = Q[r][t]
  __shared__ C2 Xs[16 * 64];     // Xs[t * 64 + c] = X[t][c]
  __shared__ C2 Pk[16 * 16];     // Pk[j * 16 + i] = P[K, K]^{-1}[i][j]
  __shared__ int s_bad;
  __shared__ float s_max;
  const int tid = threadIdx.x, lane = tid & 63;
  const long b = blockIdx.x;
  const C2* A = reinterpret_cast<const C2*>(Ain) + b * sA;
  float amax = 0.f;
  for (int e = tid; e < 64 * 64; e += 1024) {
    const int r = e & 63, c = e >> 6;
    const C2 v = (r < n && c < n) ? A[r + lda * c] : Cx<T>::mk(r == c ? 1 : 0, 0);
    Ms[c * LD + r] = v;
    amax = fmaxf(amax, (float)cabs1(v));
  }
  if (tid == 0) {
    s_bad = 0;
    s_max = 0.f;
  }
  __syncthreads();
  atomicMax(reinterpret_cast<unsigned*>(&s_max), __float_as_uint(amax));
#pragma unroll 1
  for (int k0 = 0; k0 < 64; k0 += 16) {
    if (tid < 64) {
      // Gauss-Jordan on P[K, K] in Pk (LDS): lane l owns row i = l % 16, columns
      // c0 + 4 q (c0 = l / 16).  A step reads the pivot row, the lane's column-k entry and
      // the pivot with broadcast LDS reads, all issued together, and writes the lane's
      // four entries back; one wave, so its LDS accesses stay in program order.
      const int i = lane & 15, c0 = lane >> 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) Pk[(c0 + 4 * q) * 16 + i] = Ms[(k0 + c0 + 4 * q) * LD + k0 + i];
      bool bad = false;
#pragma unroll 1
      for (int k = 0; k < 16; ++k) {
        C2 v[4], rk[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[q] = Pk[(c0 + 4 * q) * 16 + i];
          rk[q] = Pk[(c0 + 4 * q) * 16 + k];
        }
        const C2 cik = Pk[k * 16 + i];
        const C2 pk = Pk[k * 16 + k];
        bad = bad || !(cabs1(pk) > 0) || !isfinite((double)pk.x) || !isfinite((double)pk.y);
        const C2 ip = crcp_pivot(pk);
        const C2 f = cmul(cik, ip);
        __builtin_amdgcn_wave_barrier();  // every lane's reads of the step precede the writes
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = c0 + 4 * q;
          C2 w;
          if (i == k) w = (j == k) ? ip : cmul(rk[q], ip);
          else w = (j == k) ? Cx<T>::mk(-f.x, -f.y) : csub(v[q], cmul(f, rk[q]));
          Pk[j * 16 + i] = w;
        }
        __builtin_amdgcn_wave_barrier();  // and the next step's reads follow them
      }
      if (bad) s_bad = 1;
    }
    __syncthreads();
    // Q (64 x 16) and X (16 x 64): one entry of each per thread
    for (int e = tid; e < 64 * 16; e += 1024) {
      const int r = e & 63, j = e >> 6;
      const int ir = r - k0;
      C2 q = Cx<T>::mk(0, 0);
      if (ir >= 0 && ir < 16) {
        q = Pk[j * 16 + ir];
      } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) q = cfma(Ms[(k0 + t) * LD + r], Pk[j * 16 + t], q);
        q = Cx<T>::mk(-q.x, -q.y);
      }
      Qs[j * 64 + r] = q;
      const int c = r, t = j;  // X[t][c]
      const int jc = c - k0;
      Xs[t * 64 + c] = (jc >= 0 && jc < 16) ? Cx<T>::mk(jc == t ? 1 : 0, 0) : Ms[c * LD + k0 + t];
    }
    __syncthreads();
    // P <- (rows K and columns K zeroed) + Q X: thread row r = lane, columns w + 16 q
    {
      const int r = lane, w = tid >> 6;
      const bool rK = r >= k0 && r < k0 + 16;
      C2 qr[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) qr[t] = Qs[t * 64 + r];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = w + 16 * q;
        const bool cK = c >= k0 && c < k0 + 16;
        C2 acc = (rK || cK) ? Cx<T>::mk(0, 0) : Ms[c * LD + r];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc = cfma(qr[t], Xs[t * 64 + c], acc);
        Ms[c * LD + r] = acc;
      }
    }
    __syncthreads();
  }
  C2* O = reinterpret_cast<C2*>(Out) + b * sO;
  const float lim = 1e12f * fmaxf(s_max, 1e-30f);
  bool grown = false;
  for (int e = tid; e < n * n; e += 1024) {
    const int r = e % n, c = e / n;
    const C2 v = Ms[c * LD + r];
    grown |= !((float)cabs1(v) <= lim);
    O[r + ldo * c] = v;
  }
  if (grown) s_bad = 1;
  __syncthreads();
  if (s_bad && tid == 0) info[b] = 1;
}

// Block-pivot inversion in place: for each block K of BNB columns, P^{-1} = inv(M[K, K])
// (the kernel above), Q = -M[:, K] P^{-1} (GEMM), the step kernel, then M += Q X (GEMM).
constexpr int BNB = 64;
void zinv_blockpivot(int n, int batch, double* A, long lda, long sA, int* info, void* work,
                     hipStream_t st, bool c64) {
  const size_t e = c64 ? 8 : 16;
  char* w = static_cast<char*>(work);
  double* Pinv = reinterpret_cast<double*>(w);
  w += ((size_t)batch * BNB * BNB * e + 255) & ~size_t(255);
  double* Qg = reinterpret_cast<double*>(w);
  w += ((size_t)batch * n * BNB * e + 255) & ~size_t(255);
  double* Xg = reinterpret_cast<double*>(w);
  for (int k0 = 0; k0 < n; k0 += BNB) {
    const int nb = std::min(BNB, n - k0);
    // the diagonal block's inverse (16 x 16 blocks as its pivots)
    double* Ablk = A + (c64 ? 1 : 2) * (size_t)(k0 + lda * (long)k0);
    if (c64)
      hipLaunchKernelGGL(zinv_np_kernel<float>, dim3(batch), dim3(1024), 0, st, nb, Ablk, lda,
                         sA, Pinv, nb, (long)nb * nb, info);
    else
      hipLaunchKernelGGL(zinv_np_kernel<double>, dim3(batch), dim3(1024), 0, st, nb, Ablk, lda,
                         sA, Pinv, nb, (long)nb * nb, info);
    HPS_LAUNCH_CHECK();
    GemmDesc g;
    g.M = n; g.N = nb; g.K = nb; g.batch = batch;
    g.A = A + (c64 ? 1 : 2) * (size_t)lda * k0; g.lda = lda; g.sA = sA;
    g.B = Pinv; g.ldb = nb; g.sB = (long)nb * nb;
    g.C = Qg; g.ldc = n; g.sC = (long)n * nb;
    g.alpha = -1.0; g.beta = 0.0; g.c64 = c64;
    zgemm(g, st);
    const long tot = (long)nb * nb + 2L * nb * n;
    if (c64)
      hipLaunchKernelGGL(zinv_bstep_kernel<float>, dim3(cdiv(tot, 256), batch), dim3(256), 0,
                         st, n, nb, k0, A, lda, sA, Pinv, Qg, Xg, info);
    else
      hipLaunchKernelGGL(zinv_bstep_kernel<double>, dim3(cdiv(tot, 256), batch), dim3(256), 0,
                         st, n, nb, k0, A, lda, sA, Pinv, Qg, Xg, info);
    HPS_LAUNCH_CHECK();
    g = GemmDesc();
    g.M = n; g.N = n; g.K = nb; g.batch = batch;
    g.A = Qg; g.lda = n; g.sA = (long)n * nb;
    g.B = Xg; g.ldb = nb; g.sB = (long)nb * n;
    g.C = A; g.ldc = lda; g.sC = sA;
    g.alpha = 1.0; g.beta = 1.0; g.c64 = c64;
    zgemm(g, st);
  }
}

}  // namespace

size_t zinv_workspace_bytes(int n, int batch, bool c64) {
  if (n <= SMALL_MAX) return 0;
  const size_t e = c64 ? 8 : 16;
  // fully pivoted form: two copies of the matrix and the pivot records
  const size_t nn = (size_t)n * n * e;
  const size_t ints = (size_t)n * 4 * 2;
  const size_t piv = (size_t)batch * (2 * nn + ints) + 256;
  // block-pivot form: P^{-1}, Q and X
  auto r256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t blk = r256((size_t)batch * BNB * BNB * e) + r256((size_t)batch * n * BNB * e) +
                     r256((size_t)batch * BNB * n * e);
  return std::max(piv, blk);
}

void zinv(int n, int batch, const double* A, long lda, long sA, double* Out, long ldo,
          long sO, int* info, void* work, hipStream_t st, bool c64, bool full_pivoting) {
  if (n <= 0 || batch <= 0) return;
  if (batch > 65535) {
    // consecutive slices within the grid's limits; each reuses the workspace
    const long e = c64 ? 1 : 2;  // doubles per complex entry
    for (long b0 = 0; b0 < batch; b0 += 65535)
      zinv(n, (int)std::min<long>(65535, batch - b0), A + b0 * sA * e, lda, sA,
           Out + b0 * sO * e, ldo, sO, info + b0, work, st, c64, full_pivoting);
    return;
  }
  if (n > SMALL_MAX && !full_pivoting) {
    if (A != Out || lda != ldo || sA != sO)
      throw Error(1, "zinv: the block-pivot form works in place");
    zinv_blockpivot(n, batch, Out, ldo, sO, info, work, st, c64);
    return;
  }
  if (c64) zinv_t<float>(n, batch, A, lda, sA, Out, ldo, sO, info, work, st);
  else zinv_t<double>(n, batch, A, lda, sA, Out, ldo, sO, info, work, st);
}

}  // namespace hps
