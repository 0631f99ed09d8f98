// Shared device/host helpers of the HPS library (complex arithmetic on double2,
// error plumbing).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace hps {

typedef double d4v __attribute__((ext_vector_type(4)));

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
__host__ __device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

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

}  // namespace hps
