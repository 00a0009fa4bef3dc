// Shared device/host helpers of the ChASE HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

namespace chase {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct z64 {  // complex128 as stored by the caller: (re, im) interleaved
  double re, im;
};
struct c32 {  // complex64
  float re, im;
};

// Status codes of the C-ABI (LAPACK-like; negative = bad argument index).
enum Status : int {
  kOk = 0,
  kNotConverged = 1,
  kAllocFailed = 2,
  kHipError = 3,
  kBreakdown = 4,
};

// Error plumbing: every HIP call in host code goes through CHK, which turns a
// failure into kHipError and remembers the message for chase_last_error().
void set_last_error(const char* where, hipError_t err);
const char* last_error();

#define CHASE_CHK(expr)                                   \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) {                               \
      ::chase::set_last_error(#expr, e_);                 \
      return ::chase::kHipError;                          \
    }                                                     \
  } while (0)

#define CHASE_CHK_LAUNCH()                                \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) {                               \
      ::chase::set_last_error("kernel launch", e_);       \
      return ::chase::kHipError;                          \
    }                                                     \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace chase
