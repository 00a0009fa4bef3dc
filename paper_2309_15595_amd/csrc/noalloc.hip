// Allocation-free variant of the Chebyshev filter entry point, for callers
// that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid hipMalloc).
//
// The filter's split-K tail needs scratch beyond its inputs and outputs: the
// partial tiles of the K segments and the arrival / queue counters.  Here
// that scratch is one file-scope device array of fixed size, held by every
// GPU the library runs on until the process ends.  Host code never passes the
// array's name to a kernel: its device address is looked up once per device
// with hipGetSymbolAddress and cached.
#include "../../include/chase_hip.h"
#include "common.hpp"
#include "kernels.hpp"

#include <mutex>

namespace {

constexpr int kScratchSegments = CHASE_FILTER_NOALLOC_SEGMENTS;
constexpr size_t kTileBytes = 128 * 128 * 16;  // one partial 128 x 128 complex128 tile
constexpr size_t kTilesBytes = (size_t)kScratchSegments * kTileBytes;
constexpr size_t kScratchBytes = kTilesBytes + sizeof(int) * chase::kTailCounterInts;
static_assert(kScratchSegments <= chase::kTailMaxSegments, "segment cap above the planner's limit");
static_assert(kTilesBytes % 256 == 0, "counters must stay 256-byte aligned");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
int scratch_address(void** out) {
  int dev = -1;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) {
    chase::set_last_error("chase_filter_noalloc: hipGetDevice", err);
    return chase::kHipError;
  }
  if (dev < 0 || dev >= kMaxDevices) return chase::kHipError;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || p == nullptr) {
      chase::set_last_error("chase_filter_noalloc: hipGetSymbolAddress(scratch)", err);
      return chase::kHipError;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return chase::kOk;
}

}  // namespace

extern "C" int chase_filter_noalloc(const void* A, int64_t lda, void* V, int64_t ldv, void* W, int64_t ldw, int64_t N,
                                    int64_t n, const int32_t* degs, double c, double e, double mu_1,
                                    int64_t* matvecs, chase_stream_t stream) {
  if (int bad = chase::filter_check_args(A, lda, V, ldv, W, ldw, N, n, degs, e)) return bad;
  void* base = nullptr;
  if (int st = scratch_address(&base)) return st;
  unsigned char* b = static_cast<unsigned char*>(base);
  return chase::filter_on_scratch(A, lda, V, ldv, W, ldw, N, n, degs, c, e, mu_1, matvecs, b,
                                  reinterpret_cast<int*>(b + kTilesBytes), kScratchSegments,
                                  reinterpret_cast<hipStream_t>(stream));
}

extern "C" int64_t chase_filter_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }
