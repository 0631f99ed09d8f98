// Batched complex GEMM on the FP64 matrix cores of gfx950 (v_mfma_f64_16x16x4f64).
//
// A complex product is formed from three real products where the tile's third
// accumulator fits in registers (the 3M method, Higham 1992: T1 = Ar Br, T2 = Ai Bi,
// T3 = (Ar + Ai)(Br + Bi), Cr = T1 - T2, Ci = T3 - T1 - T2; the operand sums are formed
// as the MFMA operands are read), else from four (Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br); a real operand needs two.  A workgroup of WR x WC
// waves computes a BM x BN tile of C; K is staged through LDS in chunks of 16, double
// buffered, with each chunk's global loads issued two chunks ahead (two register
// stages).  Large tiles take K in chunks of 8, which halves their LDS footprint so that
// two workgroups share a compute unit, with the loads one chunk ahead.  LDS rows are padded so that the four 16-lane groups of an MFMA operand read
// fall on alternating halves of the 64 banks.  Used by the leaf stage (Sec. 2.1: Psi_i,
// Y_b, Y_i), by every merge product of Sec. 2.2 (W, Phi^a, Phi^b, R^tau) and by the
// block updates of the interface inversion.
//
// MFMA 16x16x4 lane layouts (measured on gfx950): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element v of lane l is D[l/16 + 4 v][l%16] for the f64
// instruction and D[4 (l/16) + v][l%16] for the f32 one.  Complex64 operands (the
// reduced-precision merge levels) run on the f32 instruction with FP32 accumulation.
#include <cstdio>
#include <map>
#include <mutex>
#include <type_traits>

#include "kernels.hpp"
#include "serve_hooks.hpp"

namespace hps {
namespace {

// element type traits: MFMA, accumulator and output row of accumulator slot v
template <class T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4v acc;
  typedef double2 cplx;
  static __device__ inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ inline cplx mk(double r, double i) { return make_double2(r, i); }
};
template <> struct Mfma<float> {
  typedef f4v acc;
  typedef float2 cplx;
  static __device__ inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ inline cplx mk(float r, float i) { return make_float2(r, i); }
};

constexpr int lds_pad(int w) { return (w % 32 == 16) ? 0 : 16; }

template <class T, int BM, int BN, int WR, int WC, bool AR, bool BR, int BK>
__global__ __launch_bounds__(64 * WR * WC) void zgemm_kernel(GemmDesc d) {
  typedef Mfma<T> MF;
  typedef typename MF::acc acc_t;
  typedef typename MF::cplx cplx_t;
  constexpr int NT = 64 * WR * WC;
  constexpr int NPA = AR ? 1 : 2;  // planes (re, im) of A
  constexpr int NPB = BR ? 1 : 2;
  constexpr int WM = BM / WR, WN = BN / WC;  // per-wave tile
  constexpr int MB = WM / 16, NB = WN / 16;
  constexpr bool M3 = !AR && !BR && MB * NB <= 4;  // three real products per complex one
  constexpr int LA = BM + lds_pad(BM), LB = BN + lds_pad(BN);
  static_assert(MB >= 1 && NB >= 1 && WM % 16 == 0 && WN % 16 == 0, "bad tile");
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile/threads mismatch");
  static_assert(NT % BN == 0, "B tile: whole columns per thread group");
  __shared__ T As[2][NPA][BK][LA];
  __shared__ T Bs[2][NPB][BK][LB];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles = tiles_m * ((d.N + BN - 1) / BN);
  // keep neighbouring tiles on one XCD (workgroups are dealt to the 8 XCDs in turn)
  int t = blockIdx.x;
  if (tiles % 8 == 0 && tiles >= 64) t = (t % 8) * (tiles / 8) + t / 8;
  const int tm = t % tiles_m, tn = t / tiles_m;
  const int i0 = tm * BM, j0 = tn * BN;
  const long b = blockIdx.y;

  const T* A = reinterpret_cast<const T*>(d.A) + b * d.sA * NPA;
  const T* B = reinterpret_cast<const T*>(d.B) + b * d.sB * NPB;

  // 3M: accR, accX, accI hold T1, T2, T3 until the epilogue
  acc_t accR[MB][NB], accI[MB][NB], accX[M3 ? MB : 1][M3 ? NB : 1];
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      accR[x][y] = acc_t{0, 0, 0, 0};
      accI[x][y] = acc_t{0, 0, 0, 0};
      if (M3) accX[M3 ? x : 0][M3 ? y : 0] = acc_t{0, 0, 0, 0};
    }

  constexpr int EA = BM * BK / NT;  // A elements per thread per chunk
  constexpr int EB = BN * BK / NT;
  // register stages of the global loads: two for the small tiles (a chunk's loads are
  // issued two chunks before its LDS store), one for the large tiles (whose registers
  // are taken by their accumulators); the stage index is a constant at every use
  constexpr int NS = BK == 16 ? 2 : 1;
  T ra[NS][EA][NPA], rb[NS][EB][NPB];

  auto gload = [&](auto stage, int k0) {
    constexpr int S = decltype(stage)::value;
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + NT * e;
      const int i = idx % BM, k = idx / BM;
      const int gi = i0 + i, gk = k0 + k;
      const bool ok = gi < d.M && gk < d.K;
      const long off = (long)gi + d.lda * (long)gk;
      if (AR) {
        ra[S][e][0] = ok ? A[off] : T(0);
      } else {
        const cplx_t v = ok ? reinterpret_cast<const cplx_t*>(A)[off] : MF::mk(0, 0);
        ra[S][e][0] = v.x;
        ra[S][e][NPA - 1] = v.y;
      }
    }
    // B: each thread reads EB consecutive k of one column (contiguous in memory), and
    // neighbouring threads take neighbouring columns, so that the stores into the
    // [k][j] LDS layout below are contiguous across lanes (no bank conflicts)
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int j = tid % BN, k = (tid / BN) * EB + e;
      const int gk = k0 + k, gj = j0 + j;
      const bool ok = gk < d.K && gj < d.N;
      const long off = (long)gk + d.ldb * (long)gj;
      if (BR) {
        rb[S][e][0] = ok ? B[off] : T(0);
      } else {
        const cplx_t v = ok ? reinterpret_cast<const cplx_t*>(B)[off] : MF::mk(0, 0);
        rb[S][e][0] = v.x;
        rb[S][e][NPB - 1] = v.y;
      }
    }
  };
  auto sstore = [&](auto stage, int buf) {
    constexpr int S = decltype(stage)::value;
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + NT * e;
      const int i = idx % BM, k = idx / BM;
#pragma unroll
      for (int pl = 0; pl < NPA; ++pl) As[buf][pl][k][i] = ra[S][e][pl];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int j = tid % BN, k = (tid / BN) * EB + e;
#pragma unroll
      for (int pl = 0; pl < NPB; ++pl) Bs[buf][pl][k][j] = rb[S][e][pl];
    }
  };

  // the MFMAs of one K chunk, from LDS buffer buf
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kl = kk + (lane >> 4);
      T ar[MB], ai[MB], br[NB], bi[NB];
#pragma unroll
      for (int x = 0; x < MB; ++x) {
        const int r = wr * WM + 16 * x + (lane & 15);
        ar[x] = As[buf][0][kl][r];
        ai[x] = AR ? T(0) : As[buf][NPA - 1][kl][r];
      }
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        const int c = wc * WN + 16 * y + (lane & 15);
        br[y] = Bs[buf][0][kl][c];
        bi[y] = BR ? T(0) : Bs[buf][NPB - 1][kl][c];
      }
      if constexpr (M3) {
        T as[MB], bs[NB];
#pragma unroll
        for (int x = 0; x < MB; ++x) as[x] = ar[x] + ai[x];
#pragma unroll
        for (int y = 0; y < NB; ++y) bs[y] = br[y] + bi[y];
#pragma unroll
        for (int x = 0; x < MB; ++x)
#pragma unroll
          for (int y = 0; y < NB; ++y) {
            accR[x][y] = MF::op(ar[x], br[y], accR[x][y]);
            accX[M3 ? x : 0][M3 ? y : 0] = MF::op(ai[x], bi[y], accX[M3 ? x : 0][M3 ? y : 0]);
            accI[x][y] = MF::op(as[x], bs[y], accI[x][y]);
          }
      } else {
#pragma unroll
        for (int x = 0; x < MB; ++x)
#pragma unroll
          for (int y = 0; y < NB; ++y) {
            accR[x][y] = MF::op(ar[x], br[y], accR[x][y]);
            if (!AR && !BR) accR[x][y] = MF::op(-ai[x], bi[y], accR[x][y]);
            if (!BR) accI[x][y] = MF::op(ar[x], bi[y], accI[x][y]);
            if (!AR) accI[x][y] = MF::op(ai[x], br[y], accI[x][y]);
          }
      }
    }
  };

  constexpr std::integral_constant<int, 0> s0{};
  constexpr std::integral_constant<int, NS - 1> s1{};
  const int nk = (d.K + BK - 1) / BK;
  if constexpr (NS == 2) {
    // Chunk c lives in register stage c % 2 and LDS buffer c % 2.  Its global loads are
    // issued while chunk c - 2 is computed; it is stored to LDS after chunk c - 1 is.
    gload(s0, 0);
    if (nk > 1) gload(s1, BK);
    sstore(s0, 0);
    __syncthreads();
    for (int kc = 0; kc < nk; kc += 2) {
      // even chunk kc (buffer 0); stage 1 holds chunk kc + 1
      if (kc + 2 < nk) gload(s0, (kc + 2) * BK);
      compute(0);
      if (kc + 1 < nk) sstore(s1, 1);
      __syncthreads();
      if (kc + 1 >= nk) break;
      // odd chunk kc + 1 (buffer 1); stage 0 holds chunk kc + 2
      if (kc + 3 < nk) gload(s1, (kc + 3) * BK);
      compute(1);
      if (kc + 2 < nk) sstore(s0, 0);
      __syncthreads();
    }
  } else {
    // chunk c + 1's global loads are issued before chunk c's MFMAs
    gload(s0, 0);
    sstore(s0, 0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nk) gload(s0, (kc + 1) * BK);
      compute(buf);
      if (kc + 1 < nk) sstore(s0, buf ^ 1);
      __syncthreads();
    }
  }

  if constexpr (M3) {
#pragma unroll
    for (int x = 0; x < MB; ++x)
#pragma unroll
      for (int y = 0; y < NB; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T t1 = accR[x][y][v], t2 = accX[M3 ? x : 0][M3 ? y : 0][v];
          accR[x][y][v] = t1 - t2;
          accI[x][y][v] = accI[x][y][v] - t1 - t2;
        }
  }

  // epilogue
  cplx_t* C = reinterpret_cast<cplx_t*>(d.C) + b * d.sC;
  const T alpha = (T)d.alpha, beta = (T)d.beta;
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * WM + 16 * x + MF::row(lane, v);
        const int j = j0 + wc * WN + 16 * y + (lane & 15);
        if (i < d.M && j < d.N) {
          const long ri = d.crow ? d.crow[i] : i;
          const long cj = d.ccol ? d.ccol[j] : j;
          cplx_t* p = C + ri + d.ldc * cj;
          cplx_t val = MF::mk(alpha * accR[x][y][v], alpha * accI[x][y][v]);
          if (d.C0r) val.x += (T)d.C0r[b * d.s0 + i + d.ld0 * (long)j];
          if (d.beta != 0.0) {
            const cplx_t old = *p;
            val.x += beta * old.x;
            val.y += beta * old.y;
          }
          *p = val;
        }
      }
}

template <int BM, int BN, int WR, int WC, int BK>
void launch_tile(const GemmDesc& d, hipStream_t st) {
  const int tiles = cdiv(d.M, BM) * cdiv(d.N, BN);
  const dim3 grid(tiles, d.batch);
  const dim3 block(64 * WR * WC);
  if (d.c64) {
    // the reduced-precision merges are complex x complex only
    if (d.a_real || d.b_real) throw Error(1, "zgemm: complex64 operands must be complex");
    hipLaunchKernelGGL((zgemm_kernel<float, BM, BN, WR, WC, false, false, BK>), grid, block, 0, st, d);
  } else if (d.a_real && d.b_real) {
    hipLaunchKernelGGL((zgemm_kernel<double, BM, BN, WR, WC, true, true, BK>), grid, block, 0, st, d);
  } else if (d.a_real) {
    hipLaunchKernelGGL((zgemm_kernel<double, BM, BN, WR, WC, true, false, BK>), grid, block, 0, st, d);
  } else if (d.b_real) {
    hipLaunchKernelGGL((zgemm_kernel<double, BM, BN, WR, WC, false, true, BK>), grid, block, 0, st, d);
  } else {
    hipLaunchKernelGGL((zgemm_kernel<double, BM, BN, WR, WC, false, false, BK>), grid, block, 0, st,
                       d);
  }
}

// ------------------------------------------------------------------ tile choice
// Tile variants (BM x BN, waves WR x WC).  The default choice follows the operand shape
// (thin tiles for thin operands, 64 x 64 otherwise); the autotuner replaces it per GEMM
// shape with the variant measured fastest on the device.
enum Tile { T16x64, T64x16, T32x32, T32x64, T64x32, T64x64, T128x64, T64x128, T128x128, NTILE };
const char* const kTileName[NTILE] = {"16x64", "64x16", "32x32", "32x64", "64x32",
                                      "64x64", "128x64", "64x128", "128x128"};

Tile heuristic_tile(const GemmDesc& d) {
  if (d.M <= 16) return T16x64;
  if (d.N <= 16) return T64x16;
  if (d.M <= 32 && d.N <= 32) return T32x32;
  if (d.M <= 32) return T32x64;
  if (d.N <= 32) return T64x32;
  return T64x64;
}

struct TuneKey {
  int M, N, K, batch, flags;
  bool operator<(const TuneKey& o) const {
    if (M != o.M) return M < o.M;
    if (N != o.N) return N < o.N;
    if (K != o.K) return K < o.K;
    if (batch != o.batch) return batch < o.batch;
    return flags < o.flags;
  }
};

TuneKey key_of(const GemmDesc& d) {
  const int flags = (d.a_real ? 1 : 0) | (d.b_real ? 2 : 0) | (d.c64 ? 4 : 0) |
                    (d.beta != 0.0 ? 8 : 0) | ((d.crow || d.ccol) ? 16 : 0) | (d.C0r ? 32 : 0);
  return TuneKey{d.M, d.N, d.K, d.batch, flags};
}

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;  // GEMM shape -> measured best tile

Tile pick_tile(const GemmDesc& d) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key_of(d));
  return it == g_tune.end() ? heuristic_tile(d) : (Tile)it->second;
}

void launch_variant(Tile t, const GemmDesc& d, hipStream_t st) {
  switch (t) {
    case T16x64: launch_tile<16, 64, 1, 4, 16>(d, st); break;
    case T64x16: launch_tile<64, 16, 4, 1, 16>(d, st); break;
    case T32x32: launch_tile<32, 32, 2, 2, 16>(d, st); break;
    case T32x64: launch_tile<32, 64, 2, 2, 16>(d, st); break;
    case T64x32: launch_tile<64, 32, 2, 2, 16>(d, st); break;
    case T128x64: launch_tile<128, 64, 4, 2, 8>(d, st); break;
    case T64x128: launch_tile<64, 128, 2, 4, 8>(d, st); break;
    case T128x128: launch_tile<128, 128, 4, 2, 8>(d, st); break;
    default: launch_tile<64, 64, 2, 2, 8>(d, st); break;
  }
}

}  // namespace

std::string zgemm_variant(const GemmDesc& d) {
  std::string v = kTileName[pick_tile(d)];
  v += d.a_real ? "r" : "c";
  v += d.b_real ? "r" : "c";
  if (d.c64) v += "s";  // complex64
  return v;
}

void zgemm_check(const GemmDesc& d) {
  if (d.K <= 0) throw Error(1, "zgemm: K must be positive");
  if (d.C0r && d.c64) throw Error(1, "zgemm: the real addend is for complex128 outputs");
}

// Batches beyond the grid's y limit run as consecutive slices (operands advanced by
// their batch strides; doubles per element: 1 for real or complex64, 2 for complex128).
void zgemm(const GemmDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  zgemm_check(d);
  const Tile tile = pick_tile(d);
  const long ea = (d.a_real || d.c64) ? 1 : 2, eb = (d.b_real || d.c64) ? 1 : 2;
  const long ec = d.c64 ? 1 : 2;
  for (long b0 = 0; b0 < d.batch; b0 += 65535) {
    GemmDesc s = d;
    s.batch = (int)std::min<long>(65535, d.batch - b0);
    s.A = d.A + b0 * d.sA * ea;
    s.B = d.B + b0 * d.sB * eb;
    s.C = d.C + b0 * d.sC * ec;
    if (d.C0r) s.C0r = d.C0r + b0 * d.s0;
    launch_variant(tile, s, st);
    HPS_LAUNCH_CHECK();
  }
}

// Time every tile variant on d's operands (output to a dense scratch matrix, beta = 0,
// no scatter maps: the variants differ in their main loop) and record the fastest for
// d's shape.  Synchronizes the stream.  A shape already in the table is left alone.
void zgemm_tune(const GemmDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  zgemm_check(d);
  const TuneKey key = key_of(d);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.count(key)) return;
  }
  const size_t esz = d.c64 ? 8 : 16;
  const int tb = std::min(d.batch, 65535);  // timed on the first grid-sized slice
  void* scratch = dev_alloc((size_t)tb * d.M * d.N * esz);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = heuristic_tile(d);
  float best_ms = 0.0f;
  try {
    HPS_HIP(hipEventCreate(&e0));
    HPS_HIP(hipEventCreate(&e1));
    GemmDesc t = d;
    t.batch = tb;
    t.C = static_cast<double*>(scratch);
    t.ldc = d.M;
    t.sC = (long)d.M * d.N;
    t.crow = t.ccol = nullptr;
    t.beta = 0.0;
    bool first = true;
    for (int v = 0; v < NTILE; ++v) {
      launch_variant((Tile)v, t, st);  // warm-up run
      HPS_LAUNCH_CHECK();
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {
        HPS_HIP(hipEventRecord(e0, st));
        launch_variant((Tile)v, t, st);
        HPS_LAUNCH_CHECK();
        HPS_HIP(hipEventRecord(e1, st));
        HPS_HIP(hipEventSynchronize(e1));
        float m = 0.0f;
        HPS_HIP(hipEventElapsedTime(&m, e0, e1));
        ms = rep == 0 ? m : std::min(ms, m);
      }
      if (first || ms < best_ms) {
        best = v;
        best_ms = ms;
        first = false;
      }
    }
  } catch (...) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(scratch);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dev_free(scratch);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = best;
}

int zgemm_tune_entries() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tune.size();
}

void zgemm_tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

// Table as text: one line per shape, "M N K batch flags variant".
std::string zgemm_tune_dump() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::string out;
  for (const auto& kv : g_tune) {
    const TuneKey& k = kv.first;
    out += std::to_string(k.M) + " " + std::to_string(k.N) + " " + std::to_string(k.K) + " " +
           std::to_string(k.batch) + " " + std::to_string(k.flags) + " " + kTileName[kv.second] +
           "\n";
  }
  return out;
}

// Merge lines of zgemm_tune_dump's format into the table; returns the entries read or
// throws on a malformed line.
int zgemm_tune_load(const std::string& text) {
  std::map<TuneKey, int> add;
  size_t pos = 0;
  while (pos < text.size()) {
    size_t end = text.find('\n', pos);
    if (end == std::string::npos) end = text.size();
    const std::string line = text.substr(pos, end - pos);
    pos = end + 1;
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    TuneKey k{};
    char name[32] = {0};
    if (std::sscanf(line.c_str(), "%d %d %d %d %d %31s", &k.M, &k.N, &k.K, &k.batch, &k.flags,
                    name) != 6)
      throw Error(1, "autotune table: malformed line: " + line);
    int v = -1;
    for (int i = 0; i < NTILE; ++i)
      if (std::string(name) == kTileName[i]) v = i;
    if (v < 0) throw Error(1, std::string("autotune table: unknown variant ") + name);
    add[k] = v;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : add) g_tune[kv.first] = kv.second;
  return (int)add.size();
}

}  // namespace hps
