// Solve-stage operator application (Algorithm 2): out = alpha * A X + addend for a
// batch of stored operators A (M x K, complex) and a block of nrhs right-hand sides.
//
// This is HBM-bound: every operator entry is read once per call and used for all
// nrhs columns.  One workgroup covers a tile of rows of one batch entry; the X block
// (K x NR) is staged through LDS in chunks and read by broadcast, each thread keeps NR
// complex accumulators for its row.  Operators with few rows and a long K (the top
// merges) are split along K across workgroups; the partial sums are reduced in a
// fixed order by a second kernel, so results do not depend on scheduling.
#include "kernels.hpp"

namespace hps {
namespace {

constexpr int KC = 64;  // K chunk staged in LDS

template <int NR, int BT>
__global__ __launch_bounds__(BT) void skinny_kernel(SkinnyDesc d, int r0, int nr, int kper,
                                                    double2* partial) {
  __shared__ double2 Xs[KC][NR];
  const int tid = threadIdx.x;
  const long b = blockIdx.y;
  const int ks = blockIdx.z;
  const int i = blockIdx.x * BT + tid;
  const int kbeg = ks * kper, kend = min(d.K, kbeg + kper);
  const double2* A = reinterpret_cast<const double2*>(d.A) + b * d.sA;
  const double2* X = reinterpret_cast<const double2*>(d.X) + (d.xoff ? d.xoff[b] : b * d.sX);
  double2 acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = cmk(0, 0);
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    const int kc = min(KC, kend - k0);
    __syncthreads();
    for (int e = tid; e < KC * NR; e += BT) {
      const int k = e % KC, r = e / KC;
      Xs[k][r] = (k < kc && r < nr) ? X[(k0 + k) + d.ldx * (long)(r0 + r)] : cmk(0, 0);
    }
    __syncthreads();
    if (i < d.M) {
      const double2* Ai = A + i + d.lda * (long)k0;
      for (int k = 0; k < kc; ++k) {
        const double2 a = Ai[d.lda * (long)k];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = cfma(a, Xs[k][r], acc[r]);
      }
    }
  }
  if (i >= d.M) return;
  if (partial) {
    // [ks][b][r][i]
    double2* P = partial + (((long)ks * d.batch + b) * NR) * d.M;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) P[(long)r * d.M + i] = acc[r];
    return;
  }
  double2* C = reinterpret_cast<double2*>(d.C) + (d.coff ? d.coff[b] : b * d.sC);
  const long ci = d.crow ? d.crow[i] : i;
  const double2* C0 = d.C0 ? reinterpret_cast<const double2*>(d.C0) +
                                 (d.c0off ? d.c0off[b] : b * d.s0)
                           : nullptr;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) break;
    double2 v = cscale(acc[r], d.alpha);
    double2* p = C + ci + d.ldc * (long)(r0 + r);
    if (C0) v = cadd(v, C0[i + d.ld0 * (long)(r0 + r)]);
    else if (d.accumulate) v = cadd(v, *p);
    *p = v;
  }
}

template <int NR>
__global__ void skinny_reduce_kernel(SkinnyDesc d, int r0, int nr, int nsplit,
                                     const double2* partial) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)d.batch * d.M * nr;
  if (e >= tot) return;
  const int i = e % d.M;
  const int r = (e / d.M) % nr;
  const long b = e / ((long)d.M * nr);
  double2 acc = cmk(0, 0);
  for (int s = 0; s < nsplit; ++s)
    acc = cadd(acc, partial[(((long)s * d.batch + b) * NR + r) * d.M + i]);
  double2* C = reinterpret_cast<double2*>(d.C) + (d.coff ? d.coff[b] : b * d.sC);
  const long ci = d.crow ? d.crow[i] : i;
  double2 v = cscale(acc, d.alpha);
  double2* p = C + ci + d.ldc * (long)(r0 + r);
  if (d.C0) {
    const double2* C0 = reinterpret_cast<const double2*>(d.C0) + (d.c0off ? d.c0off[b] : b * d.s0);
    v = cadd(v, C0[i + d.ld0 * (long)(r0 + r)]);
  } else if (d.accumulate) {
    v = cadd(v, *p);
  }
  *p = v;
}

int block_threads(int M) { return M <= 64 ? 64 : (M <= 128 ? 128 : 256); }

// K is split across workgroups when the row tiles x batch cannot fill the device.
// Returns the number of splits and the K range per split.
int split_plan(const SkinnyDesc& d, int* kper_out) {
  const int tiles = cdiv(d.M, block_threads(d.M));
  int nsplit = 1;
  const long blocks = (long)tiles * d.batch;
  if (blocks < 512 && d.K >= 2 * KC) {
    nsplit = (int)std::min<long>((512 + blocks - 1) / blocks, (d.K + KC - 1) / KC);
    nsplit = std::max(1, std::min(nsplit, 64));
  }
  int kper = d.K;
  if (nsplit > 1) {
    kper = (d.K + nsplit - 1) / nsplit;
    kper = ((kper + KC - 1) / KC) * KC;
    nsplit = (d.K + kper - 1) / kper;
  }
  *kper_out = kper;
  return nsplit;
}

template <int NR, int BT>
void run_chunk(const SkinnyDesc& d, int r0, int nr, hipStream_t st) {
  const int tiles = cdiv(d.M, BT);
  int kper = 0;
  const int nsplit = split_plan(d, &kper);
  if (nsplit == 1) {
    hipLaunchKernelGGL((skinny_kernel<NR, BT>), dim3(tiles, d.batch, 1), dim3(BT), 0, st, d, r0,
                       nr, d.K, (double2*)nullptr);
    HPS_LAUNCH_CHECK();
    return;
  }
  if (!d.work) throw Error(1, "zgemm_skinny: split-K needs a workspace");
  double2* part = static_cast<double2*>(d.work);
  hipLaunchKernelGGL((skinny_kernel<NR, BT>), dim3(tiles, d.batch, nsplit), dim3(BT), 0, st, d,
                     r0, nr, kper, part);
  HPS_LAUNCH_CHECK();
  long tot = (long)d.batch * d.M * nr;
  hipLaunchKernelGGL(skinny_reduce_kernel<NR>, dim3(cdiv(tot, 256)), dim3(256), 0, st, d, r0, nr,
                     nsplit, (const double2*)part);
  HPS_LAUNCH_CHECK();
}

template <int NR>
void run_nr(const SkinnyDesc& d, int r0, int nr, hipStream_t st) {
  if (d.M <= 64) run_chunk<NR, 64>(d, r0, nr, st);
  else if (d.M <= 128) run_chunk<NR, 128>(d, r0, nr, st);
  else run_chunk<NR, 256>(d, r0, nr, st);
}

}  // namespace

size_t skinny_work_bytes(const SkinnyDesc& d) {
  if (d.M <= 0 || d.batch <= 0 || d.K <= 0) return 0;
  int kper = 0;
  const int nsplit = split_plan(d, &kper);
  if (nsplit == 1) return 0;
  return (size_t)nsplit * d.batch * 16 * d.M * sizeof(double2);
}

void zgemm_skinny(const SkinnyDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.batch <= 0 || d.nrhs <= 0) return;
  if (d.batch > 65535) throw Error(1, "zgemm_skinny: batch exceeds grid limit");
  if (d.K <= 0) throw Error(1, "zgemm_skinny: K must be positive");
  for (int r0 = 0; r0 < d.nrhs; r0 += 16) {
    const int nr = std::min(16, d.nrhs - r0);
    if (nr <= 1) run_nr<1>(d, r0, nr, st);
    else if (nr <= 2) run_nr<2>(d, r0, nr, st);
    else if (nr <= 4) run_nr<4>(d, r0, nr, st);
    else if (nr <= 8) run_nr<8>(d, r0, nr, st);
    else run_nr<16>(d, r0, nr, st);
  }
}

}  // namespace hps
