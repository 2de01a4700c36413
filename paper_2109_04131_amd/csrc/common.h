// Shared device/host helpers of the usFFT library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/usfft.h"

namespace usfft {

// ---- error plumbing: every ABI call returns a status and sets a message ----
void set_error(const std::string& msg);

struct Error {
  usfft_status st;
  std::string msg;
};

#define USFFT_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw ::usfft::Error{USFFT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define USFFT_REQUIRE(cond, code, msg)                  \
  do {                                                  \
    if (!(cond)) throw ::usfft::Error{(code), (msg)};   \
  } while (0)

// ---- device helpers ----
constexpr int kWave = 64;

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide sum in a fixed order: every thread returns the same value
// (wave sums are combined in wave order), so control decisions taken on it
// are uniform and results do not depend on which block runs a sample.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  constexpr int NW = BLOCK / kWave;
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (lane == 0) red[w] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s += red[i];
  return s;
}

template <int BLOCK, typename T>
__device__ __forceinline__ void block_sum2(T& a, T& b, T* red) {
  constexpr int NW = BLOCK / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (lane == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  T sa = red[0], sb = red[1];
#pragma unroll
  for (int i = 1; i < NW; ++i) {
    sa += red[2 * i];
    sb += red[2 * i + 1];
  }
  a = sa;
  b = sb;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Remap so that each XCD works on one contiguous range of work items: writes
// of neighbouring items then meet in the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, rem = nb % 8;
  const int64_t x = b % 8, k = b / 8;
  return x * q + (x < rem ? x : rem) + k;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace usfft
