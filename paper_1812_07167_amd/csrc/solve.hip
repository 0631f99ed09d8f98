// Solve-stage operator application (Algorithm 2): out = alpha * A X + addend for a
// batch of stored operators A (M x K, complex) and a block of nrhs right-hand sides.
//
// This is HBM-bound: every operator entry is read once per pass and used for all (up to
// 64) right-hand sides of the pass.  The product runs on the matrix cores: a wave owns
// 16 rows, and each group of 16 right-hand sides is the 16 columns of one MFMA's B
// operand; NB such groups (NB = 1, 2 or 4) share every operator load.  The right-hand
// side block is staged through LDS in chunks of 64 (32 for NB = 4) k rows; each lane
// reads one complex value per 4-deep k step, so there are no broadcast reads.  Operator
// entries go from memory straight into the A operand registers, through a buffer
// resource (one 32-bit offset per lane; columns past K read as zero): a wave requests all
// of its fragments of a chunk before the chunk's right-hand sides are staged, which keeps
// enough loads in flight to cover the memory latency (one dependent load per step does
// not).  A complex product takes three real MFMAs (the 3M method: ArXr, AiXi and
// (Ar + Ai)(Xr + Xi), folded into the real and imaginary parts after the K loop).  A
// workgroup covers at most 64 rows; for short operators its waves split K and add their
// partial tiles through LDS in a fixed order.
// Operators with few rows and a long K (the top merges) are also split along K across
// workgroups; those partial sums are reduced in a fixed order by a second kernel, so
// results never depend on scheduling.  Two operators of one shape share a launch: applied
// to the same right-hand sides (the two children's Phi in the downward pass) or each to
// its own block (the two halves of h^tau in the upward pass).
//
// MFMA 16x16x4 lane layouts: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element v of lane l is D[l/16 + 4 v][l%16] (f64) or D[4 (l/16) + v][l%16]
// (f32).  Complex64 operators (the reduced-precision levels) run on the f32 instruction
// with FP32 accumulation; vectors stay complex128 in memory and are rounded when staged.
#include "kernels.hpp"

namespace hps {
namespace {

template <class T> struct SkMfma;
template <> struct SkMfma<double> {
  typedef d4v acc;
  static __device__ inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct SkMfma<float> {
  typedef f4v acc;
  static __device__ inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int v) { return 4 * lk + v; }
};

constexpr int KC = 64;   // K granularity of the split-K plan
constexpr int NRB = 16;  // right-hand sides of one MFMA column block (the MFMA's N)
constexpr int MAXNB = 4; // column blocks per pass at most: 64 right-hand sides

// column blocks of a pass over nr right-hand sides
inline int nb_of(int nr) { return nr > 2 * NRB ? 4 : nr > NRB ? 2 : 1; }

// a second operator is applied in the same launch
__host__ __device__ inline bool has2(const SkinnyDesc& d) {
  return d.aper > 0 ? d.Atab2[0] != nullptr : d.A2 != nullptr;
}
// batch entries of a launch: the second operator's follow the first's
__host__ __device__ inline int nbatch(const SkinnyDesc& d) { return has2(d) ? 2 * d.batch : d.batch; }

// One operator entry through a buffer resource: an offset past the resource's extent
// reads as zero (the range check takes the per-lane offset; the scalar offset is 0).
template <class T> struct SkLoad;
template <> struct SkLoad<double> {
  static __device__ inline double2 ld(__amdgpu_buffer_rsrc_t r, int off) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    return make_double2(v.x, v.y);
  }
};
template <> struct SkLoad<float> {
  static __device__ inline float2 ld(__amdgpu_buffer_rsrc_t r, int off) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    return make_float2(v.x, v.y);
  }
};

// buffer resource word 3 of a raw (stride 0) buffer of 32-bit elements on this target
constexpr int kBufWord3 = 0x00020000;

template <class T, int WK, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB == 1 ? 3 : 2))) void skinny_kernel(SkinnyDesc d, int r0, int nr, int kper,
                                                     double2* partial, long y0, bool xcd) {
  typedef typename Cx<T>::t C2;
  typedef SkMfma<T> MF;
  typedef typename MF::acc acc_t;
  constexpr int WR = 4 / WK;              // row groups of waves
  constexpr int ROWS = 16 * WR;           // rows per workgroup
  constexpr int NC = NRB * NB;            // right-hand sides of the pass
  constexpr int KCX = NB == 4 ? 32 : 64;  // K chunk staged in LDS
  constexpr int XLD = NC + 1;             // LDS row pitch (padded: staging writes spread banks)
  constexpr int NS = KCX / 4 / WK;        // 4-deep k steps of one wave per chunk
  constexpr int NX = KCX * NC / 256;      // staged right-hand side entries per thread
  constexpr int XS_BYTES = KCX * XLD * (int)sizeof(C2);
  constexpr int RED_BYTES = WK > 1 ? (WK - 1) * WR * 2 * NB * 64 * (int)sizeof(acc_t) : 0;
  static_assert(NX * 256 == KCX * NC, "staging covers the chunk in whole rounds");
  // the staged right-hand sides, and after the K loop the cross-wave partial tiles
  __shared__ __align__(16) char smem[XS_BYTES > RED_BYTES ? XS_BYTES : RED_BYTES];
  C2 (*Xs)[XLD] = reinterpret_cast<C2 (*)[XLD]>(smem);
  acc_t* red = reinterpret_cast<acc_t*>(smem);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave % WR, kw = wave / WR;
  const int li = lane & 15, lk = lane >> 4;
  // Workgroups are dealt to the 8 XCDs in turn by their linear index.  With xcd set
  // (launches without a K split), the index is remapped so that all row blocks of one
  // batch entry run on the same XCD and its right-hand sides are fetched into one L2;
  // the grid then has the batch rounded up to a multiple of 8 and extra entries exit.
  int tile = blockIdx.x;
  long bb = y0 + blockIdx.y;  // batch entry of the launch
  if (xcd) {
    const long L = blockIdx.x + (long)gridDim.x * blockIdx.y;
    const long slot = L >> 3;
    tile = (int)(slot % gridDim.x);
    bb = y0 + (slot / gridDim.x) * 8 + (L & 7);
    if (bb >= nbatch(d)) return;
  }
  const bool two = has2(d) && bb >= d.batch;
  const long b = two ? bb - d.batch : bb;  // entry of its operator
  const int ks = blockIdx.z;
  const int kbeg = ks * kper, kend = min(d.K, kbeg + kper);
  const int row0 = tile * ROWS + wr * 16;
  const C2* A;
  if (d.aper > 0) {
    const int q = (int)(b / d.aper);
    if (d.nrq[q] > 0) {
      if (d.nrq[q] <= r0) return;  // whole workgroup: this factor has no such columns
      nr = min(nr, d.nrq[q] - r0);
    }
    A = reinterpret_cast<const C2*>(two ? d.Atab2[q] : d.Atab[q]) + (b % d.aper) * d.sA;
  } else {
    A = reinterpret_cast<const C2*>(two ? d.A2 : d.A) + b * d.sA;
  }
  const double2* X = reinterpret_cast<const double2*>(two && d.X2 ? d.X2 : d.X) +
                     (d.xoff ? d.xoff[b] - d.xbase : b * d.sX);
  // The entry's operator as a buffer of lda x K entries: a column past K reads as zero.
  // A lane's byte offset is its row (rows past M repeat the last, never written) at its
  // k of a step; consecutive 4-deep steps are kstep bytes apart.  The host keeps every
  // offset below 2^31.
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<C2*>(A), (short)0, (int)((long)d.lda * d.K * (long)sizeof(C2)), kBufWord3);
  const int aoff = (min(row0 + li, d.M - 1) + d.lda * lk) * (int)sizeof(C2);
  const int kstep = 4 * d.lda * (int)sizeof(C2);

  // The output and its addend (C0, or the current C when accumulating).  Without a K
  // split the addends are requested now, so that they arrive during the K loop instead
  // of costing the epilogue a memory round trip.
  double2* C = reinterpret_cast<double2*>(two ? d.C2 : d.C) +
               (d.coff ? d.coff[b] - d.cbase : b * d.sC);
  const double* c0p = two ? d.C02 : d.C0;
  const double2* C0 =
      c0p ? reinterpret_cast<const double2*>(c0p) + (d.c0off ? d.c0off[b] : b * d.s0) : nullptr;
  const int* crow = two ? d.crow2 : d.crow;
  double2 addend[NB][4];
  if (!partial && (C0 || d.accumulate)) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rhs = NRB * j + li;
        const int i = row0 + MF::row(lk, v);
        addend[j][v] = cmk(0, 0);
        if (rhs < nr && i < d.M)
          addend[j][v] = C0 ? C0[i + d.ld0 * (long)(r0 + rhs)]
                            : C[(crow ? crow[i] : i) + d.ldc * (long)(r0 + rhs)];
      }
  }

  // 3M: accR, accX, accI hold ArXr, AiXi, (Ar + Ai)(Xr + Xi) until after the K loop
  acc_t accR[NB], accI[NB], accX[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    accR[j] = acc_t{0, 0, 0, 0};
    accI[j] = acc_t{0, 0, 0, 0};
    accX[j] = acc_t{0, 0, 0, 0};
  }
  for (int k0 = kbeg; k0 < kend; k0 += KCX) {
    const int kc = min(KCX, kend - k0);
    const int nsteps = (kc + 3) >> 2;
    // The chunk's right-hand sides, then every operator fragment this wave takes from
    // the chunk, are requested before anything waits, so a lane has NX + NS loads in
    // flight.  The loads are unconditional so that the waits can count them: a
    // right-hand side entry past the chunk is read at a clamped address and zeroed,
    // operator steps past the chunk are loaded but never used.
    double2 xr[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = tid + 256 * i;
      const int k = e % KCX, r = e / KCX;
      const bool ok = k < kc && r < nr;
      xr[i] = X[ok ? (k0 + k) + d.ldx * (long)(r0 + r) : 0];
    }
    C2 af[NS];
    const int c0 = (k0 >> 2) + kw;  // first step of this wave in the chunk
#pragma unroll
    for (int i = 0; i < NS; ++i) af[i] = SkLoad<T>::ld(ra, aoff + (c0 + WK * i) * kstep);
    __syncthreads();  // the previous chunk's right-hand sides have been read
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = tid + 256 * i;
      const int k = e % KCX, r = e / KCX;
      const bool ok = k < kc && r < nr;
      Xs[k][r] = ok ? Cx<T>::mk((T)xr[i].x, (T)xr[i].y) : Cx<T>::mk(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int st = kw + WK * i;
      if (st >= nsteps) break;
      const int kl = 4 * st + lk;
      const C2 a = af[i];
      const T as = a.x + a.y;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const C2 bx = Xs[kl][NRB * j + li];
        accR[j] = MF::op(a.x, bx.x, accR[j]);
        accX[j] = MF::op(a.y, bx.y, accX[j]);
        accI[j] = MF::op(as, bx.x + bx.y, accI[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T t1 = accR[j][v], t2 = accX[j][v];
      accR[j][v] = t1 - t2;
      accI[j][v] = accI[j][v] - t1 - t2;
    }
  if (WK > 1) {
    // waves kw > 0 hand their tiles to the kw = 0 wave of their row group (through the
    // LDS the staged right-hand sides used: every wave is past its last read of them)
    __syncthreads();
    if (kw > 0) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int base = ((((kw - 1) * WR + wr)) * NB + j) * 2;
        red[(base + 0) * 64 + lane] = accR[j];
        red[(base + 1) * 64 + lane] = accI[j];
      }
    }
    __syncthreads();
    if (kw > 0) return;
    for (int q = 1; q < WK; ++q)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int base = ((((q - 1) * WR + wr)) * NB + j) * 2;
        accR[j] += red[(base + 0) * 64 + lane];
        accI[j] += red[(base + 1) * 64 + lane];
      }
  }
  if (partial) {
    // [ks][bb][rhs of the pass][i]
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int rhs = NRB * j + li;
      if (rhs >= nr) continue;
      double2* P = partial + (((long)ks * nbatch(d) + bb) * NC + rhs) * d.M;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + MF::row(lk, v);
        if (i < d.M) P[i] = cmk(accR[j][v], accI[j][v]);
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int rhs = NRB * j + li;
    if (rhs >= nr) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = row0 + MF::row(lk, v);
      if (i >= d.M) continue;
      const long ci = crow ? crow[i] : i;
      double2 val = cmk(d.alpha * accR[j][v], d.alpha * accI[j][v]);
      if (C0 || d.accumulate) val = cadd(val, addend[j][v]);
      C[ci + d.ldc * (long)(r0 + rhs)] = val;
    }
  }
}

__global__ void skinny_reduce_kernel(SkinnyDesc d, int r0, int nr, int nc, int nsplit,
                                     const double2* partial) {
  const int nbt = nbatch(d);
  const long tot = (long)nbt * d.M * nr;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int i = e % d.M;
    const int r = (e / d.M) % nr;
    const long bb = e / ((long)d.M * nr);
    const bool two = has2(d) && bb >= d.batch;
    const long b = two ? bb - d.batch : bb;
    if (d.aper > 0) {
      const int nq = d.nrq[b / d.aper];
      if (nq > 0 && r0 + r >= nq) continue;  // a column the factor does not have
    }
    double2 acc = cmk(0, 0);
    for (int s = 0; s < nsplit; ++s)
      acc = cadd(acc, partial[(((long)s * nbt + bb) * nc + r) * d.M + i]);
    double2* C = reinterpret_cast<double2*>(two ? d.C2 : d.C) +
                 (d.coff ? d.coff[b] - d.cbase : b * d.sC);
    const int* crow = two ? d.crow2 : d.crow;
    const long ci = crow ? crow[i] : i;
    double2 v = cscale(acc, d.alpha);
    double2* p = C + ci + d.ldc * (long)(r0 + r);
    const double* c0p = two ? d.C02 : d.C0;
    if (c0p) {
      const double2* C0 =
          reinterpret_cast<const double2*>(c0p) + (d.c0off ? d.c0off[b] : b * d.s0);
      v = cadd(v, C0[i + d.ld0 * (long)(r0 + r)]);
    } else if (d.accumulate) {
      v = cadd(v, *p);
    }
    *p = v;
  }
}

// rows covered by one workgroup: by the operator's height, at most 64 (four waves of
// 16 rows; shorter operators split K across the waves instead).  Launches of few tall
// operators (the top merge levels: under 256 blocks of 64 rows) take 16-row blocks with
// K split over the four waves, which shortens each workgroup's chain of K steps.
int block_rows(const SkinnyDesc& d) {
  if ((long)cdiv(d.M, 64) * nbatch(d) < 256) return 16;
  return d.M <= 16 ? 16 : d.M <= 32 ? 32 : 64;
}

// K is split across workgroups when the row blocks x batch cannot fill the device: up to
// about kSplitTarget workgroups (with the top levels' 16-row blocks, 512 measured faster
// than 1024 or 2048: fewer, longer K ranges).  Returns the number of splits and the K
// range per split (a multiple of KC).
constexpr long kSplitTarget = 512;
int split_plan(const SkinnyDesc& d, int* kper_out) {
  const int tiles = cdiv(d.M, block_rows(d));
  int nsplit = 1;
  const long blocks = (long)tiles * nbatch(d);
  if (blocks < kSplitTarget && d.K >= 2 * KC) {
    nsplit = (int)std::min<long>((kSplitTarget + blocks - 1) / blocks, (d.K + KC - 1) / KC);
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

// launches of batches beyond the grid's y limit take consecutive slices of it
constexpr long kGridY = 65535;

template <class T, int WK, int NB>
void run_chunk(const SkinnyDesc& d, int r0, int nr, hipStream_t st) {
  const int tiles = cdiv(d.M, 16 * (4 / WK));
  int kper = 0;
  const int nsplit = split_plan(d, &kper);
  const long nbt = nbatch(d);
  if (nsplit == 1) {
    // slices of a multiple of 8 entries; the last is rounded up to one (see the kernel)
    constexpr long kSlice = kGridY / 8 * 8;
    for (long y0 = 0; y0 < nbt; y0 += kSlice) {
      const long ny = std::min(kSlice, (nbt - y0 + 7) / 8 * 8);
      hipLaunchKernelGGL((skinny_kernel<T, WK, NB>), dim3(tiles, ny, 1), dim3(256), 0, st, d, r0,
                         nr, d.K, (double2*)nullptr, y0, true);
      HPS_LAUNCH_CHECK();
    }
    return;
  }
  if (!d.work) throw Error(1, "zgemm_skinny: split-K needs a workspace");
  double2* part = static_cast<double2*>(d.work);
  for (long y0 = 0; y0 < nbt; y0 += kGridY) {
    hipLaunchKernelGGL((skinny_kernel<T, WK, NB>),
                       dim3(tiles, std::min(kGridY, nbt - y0), nsplit), dim3(256), 0, st, d, r0,
                       nr, kper, part, y0, false);
    HPS_LAUNCH_CHECK();
  }
  long tot = (long)nbatch(d) * d.M * nr;
  hipLaunchKernelGGL(skinny_reduce_kernel, dim3(grid1d(tot)), dim3(256), 0, st, d, r0, nr,
                     NRB * NB, nsplit, (const double2*)part);
  HPS_LAUNCH_CHECK();
}

template <class T, int NB>
void run_pass_nb(const SkinnyDesc& d, int r0, int nr, hipStream_t st) {
  switch (block_rows(d)) {
    case 16: run_chunk<T, 4, NB>(d, r0, nr, st); break;
    case 32: run_chunk<T, 2, NB>(d, r0, nr, st); break;
    default: run_chunk<T, 1, NB>(d, r0, nr, st); break;
  }
}

template <class T>
void run_pass_t(const SkinnyDesc& d, int r0, int nr, hipStream_t st) {
  switch (nb_of(nr)) {
    case 1: run_pass_nb<T, 1>(d, r0, nr, st); break;
    case 2: run_pass_nb<T, 2>(d, r0, nr, st); break;
    default: run_pass_nb<T, 4>(d, r0, nr, st); break;
  }
}

void run_pass(const SkinnyDesc& d, int r0, int nr, hipStream_t st) {
  if (d.a_c64) run_pass_t<float>(d, r0, nr, st);
  else run_pass_t<double>(d, r0, nr, st);
}

// bytes of the split-K partial sums of a pass over nr right-hand sides
size_t pass_work_bytes(const SkinnyDesc& d, int nr) {
  const int nb = nb_of(nr);
  int kper = 0;
  const int nsplit = split_plan(d, &kper);
  if (nsplit == 1) return 0;
  return (size_t)nsplit * nbatch(d) * NRB * nb * d.M * sizeof(double2);
}

// ------------------------------------------------------------------ fused up level
constexpr int kUpMaxN3 = 56;  // interface length of the levels the fused kernel takes

// Products Y = A X of one box, A (M x K, column-major lda = M) from memory, X (K x 16,
// LDS, X[k * 16 + r], complex128) a staged block of vectors.  A 16-row tile of A is one
// wave's; its NS 4-deep steps are loaded first (frag_load, through a buffer resource:
// steps past K read as zero) and applied later (frag_apply, 3M MFMA products as in the
// skinny kernel), so a box's next operator can be in flight while the current one is
// applied.  out(v, i, r, y) receives every entry with i < M, r < 16 (v: the lane's
// accumulator slot, i = frag_row(tile, lane, v)).
template <class T, int NS>
struct Frag {
  typename Cx<T>::t a[NS];
};
template <class T, int NS>
__device__ inline void frag_load(Frag<T, NS>& f, const double* Ad, int M, int K, int tile,
                                 int lane) {
  typedef typename Cx<T>::t C2;
  const int li = lane & 15, lk = lane >> 4;
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(Ad), (short)0, (int)((long)M * K * (long)sizeof(C2)), kBufWord3);
  const int aoff = (min(tile * 16 + li, M - 1) + M * lk) * (int)sizeof(C2);
  const int kstep = 4 * M * (int)sizeof(C2);
#pragma unroll
  for (int s = 0; s < NS; ++s) f.a[s] = SkLoad<T>::ld(ra, aoff + s * kstep);
}
template <class T, int NS, class Out>
__device__ inline void frag_apply(const Frag<T, NS>& f, int M, int K, int tile,
                                  const double2* X, int lane, Out out) {
  typedef typename Cx<T>::t C2;
  typedef SkMfma<T> MF;
  typedef typename MF::acc acc_t;
  const int li = lane & 15, lk = lane >> 4;
  const int nsteps = (K + 3) >> 2;
  acc_t accR = acc_t{0, 0, 0, 0}, accX = acc_t{0, 0, 0, 0}, accI = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s < nsteps) {  // (a guard, not a break: the loop stays unrolled, f in registers)
      const int k = 4 * s + lk;
      const double2 xv = k < K ? X[k * 16 + li] : cmk(0, 0);
      const C2 bx = Cx<T>::mk((T)xv.x, (T)xv.y);
      const C2 a = f.a[s];
      accR = MF::op(a.x, bx.x, accR);
      accX = MF::op(a.y, bx.y, accX);
      accI = MF::op(a.x + a.y, bx.x + bx.y, accI);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = tile * 16 + MF::row(lk, v);
    if (i < M)
      out(v, i, li, cmk((double)accR[v] - (double)accX[v],
                        (double)accI[v] - (double)accR[v] - (double)accX[v]));
  }
}
// the rows i = tile * 16 + row(lane, v) that frag_apply hands this lane
template <class T>
__device__ inline int frag_row(int tile, int lane, int v) {
  return tile * 16 + SkMfma<T>::row(lane >> 4, v);
}

// NS = the level's 4-deep steps (n3 <= 4 NS); the n3 x n3 operators have at most 4 row
// tiles, one per wave, and their fragments are loaded one product ahead.
template <class T, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NS <= 4 ? 3 : NS <= 8 ? 2 : 1))) void up_fused_kernel(UpLevelDesc d) {
  constexpr int NR = NRB;  // right-hand sides per pass
  extern __shared__ double2 sv[];
  const int n3 = d.n3, nbc = d.nbc, nbp = d.nbp, n1 = d.n1, n2 = d.n2;
  double2* H3a = sv;            // [n3][16]
  double2* V = sv + n3 * NR;    // v = R33b h3a - h3b
  double2* T3a = V + n3 * NR;   // t~3a
  double2* T3b = T3a + n3 * NR; // t~3b
  // the level's index maps (the same for every box): i3a, i3b, then i1a, i2b, then perm
  int* im = reinterpret_cast<int*>(T3b + n3 * NR);
  int* si3a = im;
  int* si3b = im + n3;
  int* si1a = im + 2 * n3;
  int* si2b = si1a + n1;
  int* sperm = si2b + n2;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const long q = blockIdx.x;
  const int f = (int)(q / d.per), qb = (int)(q % d.per);
  int nrhs = d.nrhs;
  if (d.nrq[f] > 0) nrhs = min(nrhs, d.nrq[f]);
  const long e = d.c64 ? 1 : 2;  // doubles per operator entry
  const double* R33b = d.R33b[f] + qb * (long)n3 * n3 * e;
  const double* Winv = d.Winv[f] + qb * (long)n3 * n3 * e;
  const double* R33a = d.R33a[f] + qb * (long)n3 * n3 * e;
  const double* R13a = d.R13a[f] + qb * (long)n1 * n3 * e;
  const double* R23b = d.R23b[f] + qb * (long)n2 * n3 * e;
  const double2* ha = reinterpret_cast<const double2*>(d.hc) + (2 * q) * (long)nbc * d.nrhs;
  const double2* hb = reinterpret_cast<const double2*>(d.hc) + (2 * q + 1) * (long)nbc * d.nrhs;
  double2* hp = reinterpret_cast<double2*>(d.hp) + q * (long)nbp * d.nrhs;
  double2* tta = reinterpret_cast<double2*>(d.tta) + q * (long)n3 * d.nrhs;
  double2* ttb = reinterpret_cast<double2*>(d.ttb) + q * (long)n3 * d.nrhs;
  const double2* jmp = reinterpret_cast<const double2*>(d.jmp);
  const bool mine = wave * 16 < n3;  // this wave's row tile of the n3 x n3 operators
  Frag<T, NS> fa, fb;
  if (mine) frag_load(fa, R33b, n3, n3, wave, lane);
  for (int x = tid; x < 2 * n3 + n1 + n2 + nbp; x += 256) {
    int v;
    if (x < n3) v = d.i3a[x];
    else if (x < 2 * n3) v = d.i3b[x - n3];
    else if (x < 2 * n3 + n1) v = d.i1a[x - 2 * n3];
    else if (x < 2 * n3 + n1 + n2) v = d.i2b[x - 2 * n3 - n1];
    else v = d.perm[x - 2 * n3 - n1 - n2];
    im[x] = v;
  }
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    const int nr = min(NR, nrhs - r0);
    if (r0 > 0 && mine) frag_load(fa, R33b, n3, n3, wave, lane);
    __syncthreads();  // index maps staged; the previous pass's vectors have been read
    // gather: h3a, and v = -h3b (jumps subtracted), zero past the pass's columns
    for (int x = tid; x < n3 * NR; x += 256) {
      const int k = x / NR, r = x % NR;
      double2 a = cmk(0, 0), b = cmk(0, 0);
      if (r < nr) {
        const long c = (long)nbc * (r0 + r);
        a = ha[si3a[k] + c];
        b = hb[si3b[k] + c];
        if (jmp) {
          const long qk = q * (long)n3 + k;
          a = csub(a, jmp[(long)(r0 + r) * d.ldj + d.jb[qk] - d.jbase]);  // h3a - j2
          b = csub(b, jmp[(long)(r0 + r) * d.ldj + d.ja[qk] - d.jbase]);  // h3b - j1
        }
      }
      H3a[x] = a;
      V[x] = cmk(-b.x, -b.y);
    }
    __syncthreads();
    if (mine) {
      frag_load(fb, Winv, n3, n3, wave, lane);
      frag_apply(fa, n3, n3, wave, H3a, lane, [&](int, int i, int r, double2 y) {
        V[i * NR + r] = cadd(V[i * NR + r], y);
      });
    }
    __syncthreads();
    if (mine) {
      frag_load(fa, R33a, n3, n3, wave, lane);
      frag_apply(fb, n3, n3, wave, V, lane, [&](int, int i, int r, double2 y) {
        T3a[i * NR + r] = y;
        if (r < nr) tta[i + (long)n3 * (r0 + r)] = y;
      });
    }
    __syncthreads();
    // this wave's first R13a tile, and the I1 entries of child a it adds to, in flight
    // while t~3b is formed
    const int li = lane & 15;
    const bool rok = li < nr;
    double2 add[4];
    if (wave * 16 < n1) {
      frag_load(fb, R13a, n1, n3, wave, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = min(frag_row<T>(wave, lane, v), n1 - 1);
        add[v] = rok ? ha[si1a[i] + (long)nbc * (r0 + li)] : cmk(0, 0);
      }
    }
    if (mine)
      frag_apply(fa, n3, n3, wave, T3a, lane, [&](int, int i, int r, double2 y) {
        const double2 h = H3a[i * NR + r];
        const double2 w = cmk(-h.x - y.x, -h.y - y.y);
        T3b[i * NR + r] = w;
        if (r < nr) ttb[i + (long)n3 * (r0 + r)] = w;
      });
    __syncthreads();
    // h^tau: R13a t~3a into the parent's I1 rows, R23b t~3b into its I2 rows
    for (int t = wave; t * 16 < n1; t += 4) {
      if (t != wave) {
        frag_load(fb, R13a, n1, n3, t, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = min(frag_row<T>(t, lane, v), n1 - 1);
          add[v] = rok ? ha[si1a[i] + (long)nbc * (r0 + li)] : cmk(0, 0);
        }
      }
      frag_apply(fb, n1, n3, t, T3a, lane, [&](int v, int i, int r, double2 y) {
        if (r < nr) hp[sperm[i] + (long)nbp * (r0 + r)] = cadd(add[v], y);
      });
    }
    for (int t = wave; t * 16 < n2; t += 4) {
      frag_load(fa, R23b, n2, n3, t, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = min(frag_row<T>(t, lane, v), n2 - 1);
        add[v] = rok ? hb[si2b[i] + (long)nbc * (r0 + li)] : cmk(0, 0);
      }
      frag_apply(fa, n2, n3, t, T3b, lane, [&](int v, int i, int r, double2 y) {
        if (r < nr) hp[sperm[n1 + i] + (long)nbp * (r0 + r)] = cadd(add[v], y);
      });
    }
  }
}

// ------------------------------------------------------------------ fused down level
// Work items of a box: (operator, 16-row tile, K part); an operator of one tile splits K
// in two so that the four waves have work.  A wave accumulates an item over its K range
// in chunks of DNS 4-deep steps, the next chunk's fragments loaded while the current one
// is applied, and leaves its tile in LDS; the outputs add the K parts in order.
constexpr int DNS = 8;
template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void down_fused_kernel(DownLevelDesc d) {
  typedef typename Cx<T>::t C2;
  typedef SkMfma<T> MF;
  typedef typename MF::acc acc_t;
  constexpr int NR = NRB;
  extern __shared__ double2 sv[];
  const int n3 = d.n3, nbc = d.nbc, nbp = d.nbp, n1 = d.n1, n2 = d.n2;
  const int ntile = (n3 + 15) / 16;
  const int nk = ntile == 1 ? 2 : 1;
  const int nitem = 2 * ntile * nk;
  const int Kq = ((nbp + nk - 1) / nk + 3) & ~3;  // K range of a part (whole steps)
  double2* X = sv;                      // [nbp][16] the parent's t
  double2* Pt = X + nbp * NR;           // [nitem][16 rows][16 rhs] partial tiles
  int* im = reinterpret_cast<int*>(Pt + nitem * 256);
  int* si1a = im;
  int* si2b = si1a + n1;
  int* si3a = si2b + n2;
  int* si3b = si3a + n3;
  int* sperm = si3b + n3;
  const int tid = threadIdx.x, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const long q = blockIdx.x;
  const int f = (int)(q / d.per), qb = (int)(q % d.per);
  int nrhs = d.nrhs;
  if (d.nrq[f] > 0) nrhs = min(nrhs, d.nrq[f]);
  const long e = d.c64 ? 1 : 2;
  const double* Pa = d.PhiA[f] + qb * (long)n3 * nbp * e;
  const double* Pb = d.PhiB[f] + qb * (long)n3 * nbp * e;
  const double2* tp = reinterpret_cast<const double2*>(d.tp) + q * (long)nbp * d.nrhs;
  double2* tca = reinterpret_cast<double2*>(d.tc) + (2 * q) * (long)nbc * d.nrhs;
  double2* tcb = reinterpret_cast<double2*>(d.tc) + (2 * q + 1) * (long)nbc * d.nrhs;
  const double2* t0a = d.tta ? reinterpret_cast<const double2*>(d.tta) + q * (long)n3 * d.nrhs : nullptr;
  const double2* t0b = d.ttb ? reinterpret_cast<const double2*>(d.ttb) + q * (long)n3 * d.nrhs : nullptr;
  for (int x = tid; x < n1 + n2 + 2 * n3 + nbp; x += 256) {
    int v;
    if (x < n1) v = d.i1a[x];
    else if (x < n1 + n2) v = d.i2b[x - n1];
    else if (x < n1 + n2 + n3) v = d.i3a[x - n1 - n2];
    else if (x < n1 + n2 + 2 * n3) v = d.i3b[x - n1 - n2 - n3];
    else v = d.perm[x - n1 - n2 - 2 * n3];
    im[x] = v;
  }
  // an item's operator, row tile and K range
  struct Item {
    __amdgpu_buffer_rsrc_t ra;
    int tile, kbeg, kend, aoff;
  };
  auto item = [&](int it) {
    const int op = it / (ntile * nk), rem = it % (ntile * nk);
    Item m;
    m.tile = rem / nk;
    const int kq = rem % nk;
    m.kbeg = kq * Kq;
    m.kend = min(nbp, m.kbeg + Kq);
    m.ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(op ? Pb : Pa), (short)0,
                                             (int)((long)n3 * nbp * (long)sizeof(C2)), kBufWord3);
    m.aoff = (min(m.tile * 16 + li, n3 - 1) + n3 * lk) * (int)sizeof(C2);
    return m;
  };
  const int kstep = 4 * n3 * (int)sizeof(C2);
  C2 fa[DNS], fb[DNS];
  auto load = [&](const Item& m, C2* fr, int s0) {
#pragma unroll
    for (int i = 0; i < DNS; ++i) fr[i] = SkLoad<T>::ld(m.ra, m.aoff + (s0 + i) * kstep);
  };
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    const int nr = min(NR, nrhs - r0);
    // the operators do not depend on t: this wave's first chunk is requested before it
    if (wave < nitem) {
      const Item m = item(wave);
      load(m, fa, m.kbeg >> 2);
    }
    __syncthreads();  // index maps staged; the previous pass's LDS has been read
    for (int x = tid; x < nbp * NR; x += 256) {
      const int k = x / NR, r = x % NR;
      X[x] = r < nr ? tp[k + (long)nbp * (r0 + r)] : cmk(0, 0);
    }
    __syncthreads();
    // the children's outer rows: copies of the parent's I1 and I2 entries
    for (int x = tid; x < (n1 + n2) * nr; x += 256) {
      const int k = x % (n1 + n2), r = x / (n1 + n2);
      const double2 v = X[sperm[k] * NR + r];
      if (k < n1) tca[si1a[k] + (long)nbc * (r0 + r)] = v;
      else tcb[si2b[k - n1] + (long)nbc * (r0 + r)] = v;
    }
    for (int it = wave; it < nitem; it += 4) {
      const Item m = item(it);
      const int s_end = (m.kend + 3) >> 2;
      acc_t accR = acc_t{0, 0, 0, 0}, accX = acc_t{0, 0, 0, 0}, accI = acc_t{0, 0, 0, 0};
      auto apply = [&](const C2* fr, int s0) {
#pragma unroll
        for (int i = 0; i < DNS; ++i) {
          if (s0 + i < s_end) {
            const int k = 4 * (s0 + i) + lk;
            const double2 xv = k < m.kend ? X[k * NR + li] : cmk(0, 0);
            const C2 bx = Cx<T>::mk((T)xv.x, (T)xv.y);
            const C2 a = fr[i];
            accR = MF::op(a.x, bx.x, accR);
            accX = MF::op(a.y, bx.y, accX);
            accI = MF::op(a.x + a.y, bx.x + bx.y, accI);
          }
        }
      };
      int s = m.kbeg >> 2;
      if (it != wave) load(m, fa, s);  // (the first item's first chunk is in flight)
      for (; s < s_end; s += 2 * DNS) {
        if (s + DNS < s_end) load(m, fb, s + DNS);
        apply(fa, s);
        if (s + DNS >= s_end) break;
        if (s + 2 * DNS < s_end) load(m, fa, s + 2 * DNS);
        apply(fb, s + DNS);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Pt[it * 256 + MF::row(lk, v) * NR + li] =
            cmk((double)accR[v] - (double)accX[v],
                (double)accI[v] - (double)accR[v] - (double)accX[v]);
    }
    __syncthreads();
    // the children's interface rows: the K parts in order, plus t~3
    for (int x = tid; x < 2 * n3 * nr; x += 256) {
      const int op = x / (n3 * nr), rem = x % (n3 * nr);
      const int i = rem % n3, r = rem / n3;
      const int tile = i / 16, row = i % 16;
      double2 y = cmk(0, 0);
      for (int kq = 0; kq < nk; ++kq) y = cadd(y, Pt[((op * ntile + tile) * nk + kq) * 256 + row * NR + r]);
      const double2* t0 = op ? t0b : t0a;
      if (t0) y = cadd(y, t0[i + (long)n3 * (r0 + r)]);
      if (op == 0) tca[si3a[i] + (long)nbc * (r0 + r)] = y;
      else tcb[si3b[i] + (long)nbc * (r0 + r)] = y;
    }
  }
}

}  // namespace

size_t skinny_work_bytes(const SkinnyDesc& d) {
  if (d.M <= 0 || d.batch <= 0 || d.K <= 0 || d.nrhs <= 0) return 0;
  constexpr int NCMAX = NRB * MAXNB;
  size_t b = pass_work_bytes(d, std::min(d.nrhs, NCMAX));
  if (d.nrhs > NCMAX && d.nrhs % NCMAX) b = std::max(b, pass_work_bytes(d, d.nrhs % NCMAX));
  return b;
}

void zgemm_skinny(const SkinnyDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.batch <= 0 || d.nrhs <= 0) return;
  if (has2(d) && !d.C2) throw Error(1, "zgemm_skinny: second operator without output");
  if (d.X2 && !has2(d)) throw Error(1, "zgemm_skinny: second right-hand side block without operator");
  if (d.aper > 0) {
    if ((long)d.batch > (long)d.aper * SkinnyDesc::kMaxTab || d.batch % d.aper)
      throw Error(1, "zgemm_skinny: batch is not a whole number of tabled factors");
    for (int q = 0; q < d.batch / d.aper; ++q)
      if (!d.Atab[q] || (d.Atab2[0] && !d.Atab2[q]))
        throw Error(1, "zgemm_skinny: missing operator of a tabled factor");
  }
  if (d.K <= 0) throw Error(1, "zgemm_skinny: K must be positive");
  // operator byte offsets (rows, steps past K by up to one chunk) stay below 2^31
  const long esz = d.a_c64 ? 8 : 16;
  if (d.lda < d.M || ((long)d.lda * (d.K + 2 * KC) + d.M) * esz >= (1L << 31))
    throw Error(1, "zgemm_skinny: operator of more than 2 GiB or lda below M");
  // passes of up to 64 right-hand sides; the last takes the rest
  constexpr int NCMAX = NRB * MAXNB;
  for (int r0 = 0; r0 < d.nrhs; r0 += NCMAX) run_pass(d, r0, std::min(NCMAX, d.nrhs - r0), st);
}

// LDS of a box of the fused upward kernel: four vectors of the pass, then the index maps
static size_t up_fused_lds(int n1, int n2, int n3, int nbp) {
  return (size_t)4 * n3 * NRB * sizeof(double2) + (size_t)(2 * n3 + n1 + n2 + nbp) * sizeof(int);
}

bool up_fused_fits(int n1, int n2, int n3, int nbp) {
  return n3 > 0 && n3 <= kUpMaxN3 && n1 + n2 == nbp && up_fused_lds(n1, n2, n3, nbp) <= 64 * 1024;
}

// LDS of a box of the fused downward kernel: the parent's t, the partial tiles, the maps
size_t down_fused_lds(int n1, int n2, int n3, int nbp) {
  const int ntile = (n3 + 15) / 16, nitem = 2 * ntile * (ntile == 1 ? 2 : 1);
  return (size_t)nbp * NRB * sizeof(double2) + (size_t)nitem * 256 * sizeof(double2) +
         (size_t)(n1 + n2 + 2 * n3 + nbp) * sizeof(int);
}
// LDS limit of a fused downward box: above 64 KB (the two n3 = 56 levels at p = 16, one
// workgroup per CU) the fused form was slower than the separate launches
constexpr size_t kDynLds = 64 * 1024;

bool down_fused_fits(int n1, int n2, int n3, int nbp) {
  return n3 > 0 && n3 <= kUpMaxN3 && n1 + n2 == nbp && down_fused_lds(n1, n2, n3, nbp) <= kDynLds;
}

void down_fused(const DownLevelDesc& d, hipStream_t st) {
  if (d.nbox <= 0 || d.nrhs <= 0) return;
  if (!down_fused_fits(d.n1, d.n2, d.n3, d.nbp))
    throw Error(1, "down_fused: a level the fused kernel does not take");
  if (d.per <= 0 || (d.nbox + d.per - 1) / d.per > SkinnyDesc::kMaxTab)
    throw Error(1, "down_fused: boxes per factor");
  const size_t lds = down_fused_lds(d.n1, d.n2, d.n3, d.nbp);
  if (d.c64)
    hipLaunchKernelGGL(down_fused_kernel<float>, dim3(d.nbox), dim3(256), lds, st, d);
  else
    hipLaunchKernelGGL(down_fused_kernel<double>, dim3(d.nbox), dim3(256), lds, st, d);
  HPS_LAUNCH_CHECK();
}

void up_fused(const UpLevelDesc& d, hipStream_t st) {
  if (d.nbox <= 0 || d.nrhs <= 0) return;
  if (!up_fused_fits(d.n1, d.n2, d.n3, d.nbp))
    throw Error(1, "up_fused: a level the fused kernel does not take");
  if (d.per <= 0 || (d.nbox + d.per - 1) / d.per > SkinnyDesc::kMaxTab)
    throw Error(1, "up_fused: boxes per factor");
  const size_t lds = up_fused_lds(d.n1, d.n2, d.n3, d.nbp);
  const int ns = (d.n3 + 3) / 4;
#define HPS_UPF(T, NS) \
  hipLaunchKernelGGL((up_fused_kernel<T, NS>), dim3(d.nbox), dim3(256), lds, st, d)
  if (d.c64) {
    if (ns <= 4) HPS_UPF(float, 4);
    else if (ns <= 8) HPS_UPF(float, 8);
    else HPS_UPF(float, 14);
  } else {
    if (ns <= 4) HPS_UPF(double, 4);
    else if (ns <= 8) HPS_UPF(double, 8);
    else HPS_UPF(double, 14);
  }
#undef HPS_UPF
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
