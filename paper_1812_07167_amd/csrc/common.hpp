// Shared device/host helpers of the HPS library (complex arithmetic on double2,
// error plumbing).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace hps {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- complex on double2
__host__ __device__ inline double2 cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
// a += b * c
__host__ __device__ inline double2 cfma(double2 b, double2 c, double2 a) {
  return cmk(a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x);
}
// 1 / a, scaled to avoid overflow in |a|^2 (Smith's method)
__host__ __device__ inline double2 crcp(double2 a) {
  if (fabs(a.x) >= fabs(a.y)) {
    double r = a.y / a.x, d = a.x + a.y * r;
    return cmk(1.0 / d, -r / d);
  } else {
    double r = a.x / a.y, d = a.y + a.x * r;
    return cmk(r / d, -1.0 / d);
  }
}
// 1 / a with one division (|a|^2 must stay inside the double range: used for pivots of
// matrices with entries of moderate size, where |a| is the column's largest entry)
__host__ __device__ inline double2 crcp_fast(double2 a) {
  const double d = 1.0 / fma(a.x, a.x, a.y * a.y);
  return cmk(a.x * d, -a.y * d);
}
// 1 / a with one division when |a|^2 is comfortably inside the double range, else by
// Smith's method (callers with a wave-uniform a take one branch only)
__host__ __device__ inline double2 crcp_pivot(double2 a) {
  const double n2 = fma(a.x, a.x, a.y * a.y);
  if (n2 > 1e-280 && n2 < 1e280) {
    const double d = 1.0 / n2;
    return cmk(a.x * d, -a.y * d);
  }
  return crcp(a);
}
__host__ __device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

// the same operations on complex64 (float2), for the reduced-precision merge levels
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cfma(float2 b, float2 c, float2 a) {
  return make_float2(a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x);
}
__host__ __device__ inline float2 crcp(float2 a) {
  if (fabsf(a.x) >= fabsf(a.y)) {
    float r = a.y / a.x, d = a.x + a.y * r;
    return make_float2(1.0f / d, -r / d);
  } else {
    float r = a.x / a.y, d = a.y + a.x * r;
    return make_float2(r / d, -1.0f / d);
  }
}
__host__ __device__ inline float2 crcp_fast(float2 a) {
  const float d = 1.0f / fmaf(a.x, a.x, a.y * a.y);
  return make_float2(a.x * d, -a.y * d);
}
__host__ __device__ inline float2 crcp_pivot(float2 a) {
  const float n2 = fmaf(a.x, a.x, a.y * a.y);
  if (n2 > 1e-35f && n2 < 1e35f) {
    const float d = 1.0f / n2;
    return make_float2(a.x * d, -a.y * d);
  }
  return crcp(a);
}
__host__ __device__ inline float cabs1(float2 a) { return fabsf(a.x) + fabsf(a.y); }

// complex type of a real element type
template <class T> struct Cx;
template <> struct Cx<double> {
  typedef double2 t;
  static __host__ __device__ inline t mk(double r, double i) { return make_double2(r, i); }
};
template <> struct Cx<float> {
  typedef float2 t;
  static __host__ __device__ inline t mk(float r, float i) { return make_float2(r, i); }
};

// ---------------------------------------------------------------- wave reductions
// Maximum of an unsigned value over the 64 lanes of a wave (all lanes active), by DPP
// row shifts (prefix maximum inside each row of 16 lanes) and the row broadcasts of
// lanes 15 and 31; lane 63 then holds the wave maximum.  0 is the neutral element.
__device__ inline unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Value of a double held by lane `lane` (uniform across the wave).
__device__ inline double readlane_f64(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)hi << 32) | lo));
}

// Pivot search over a wave: every lane offers its best candidate (magnitude mag >= 0,
// or a negative mag for "none") and its row index.  Returns the row of the largest
// magnitude, compared in single precision (ties go to the lowest lane), or -1 if no
// lane has a candidate with a positive magnitude.  Must be called by all 64 lanes.
__device__ inline int wave_argmax(double mag, int row) {
  // non-negative floats order like their bit patterns; a positive magnitude below the
  // single-precision range still counts as a candidate
  unsigned key = mag > 0.0 ? max(__float_as_uint((float)mag), 1u) : 0u;
  unsigned best = wave_max_u32(key);
  if (best == 0u) return -1;
  unsigned long long hit = __ballot(key == best);
  int src = __builtin_ctzll(hit);
  return __builtin_amdgcn_readlane(row, src);
}

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HPS_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::hps::Error(4, std::string("HIP error ") + hipGetErrorString(e_) + " at " \
                                + __FILE__ + ":" + std::to_string(__LINE__));         \
  } while (0)

#define HPS_LAUNCH_CHECK() HPS_HIP(hipGetLastError())

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// Blocks of 256 threads for an elementwise kernel over n items with a grid-stride loop:
// a dispatch counts its work-items in 32 bits, so the grid is capped (2^28 threads).
inline unsigned grid1d(long n) { return (unsigned)std::min<long>(cdiv(n, 256), 1L << 20); }
// a grid's y or z extent (at most 65535); kernels launched with it loop over the rest
inline unsigned grid_y(long n) { return (unsigned)std::max<long>(1, std::min<long>(n, 65535)); }

}  // namespace hps
