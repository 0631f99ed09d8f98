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
  double2* C = reinterpret_cast<double2*>(two ? d.C2 : d.C) +
               (d.coff ? d.coff[b] - d.cbase : b * d.sC);
  const double* c0p = two ? d.C02 : d.C0;
  const double2* C0 =
      c0p ? reinterpret_cast<const double2*>(c0p) + (d.c0off ? d.c0off[b] : b * d.s0) : nullptr;
  const int* crow = two ? d.crow2 : d.crow;
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
      double2* p = C + ci + d.ldc * (long)(r0 + rhs);
      if (C0) val = cadd(val, C0[i + d.ld0 * (long)(r0 + rhs)]);
      else if (d.accumulate) val = cadd(val, *p);
      *p = val;
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
// 16 rows; shorter operators split K across the waves instead)
int block_rows(const SkinnyDesc& d) { return d.M <= 16 ? 16 : d.M <= 32 ? 32 : 64; }

// K is split across workgroups when the row blocks x batch cannot fill the device.
// Returns the number of splits and the K range per split (a multiple of KC).
int split_plan(const SkinnyDesc& d, int* kper_out) {
  const int tiles = cdiv(d.M, block_rows(d));
  int nsplit = 1;
  const long blocks = (long)tiles * nbatch(d);
  if (blocks < 1024 && d.K >= 2 * KC) {
    nsplit = (int)std::min<long>((1024 + blocks - 1) / blocks, (d.K + KC - 1) / KC);
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

}  // namespace hps
