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

// Cross-lane moves through DPP (data-parallel primitives of GFX9): lanes the
// row/bank mask disables receive 0.
template <int CTRL, int ROW = 0xF, int BANK = 0xF>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW, BANK, false));
}
template <int CTRL, int ROW = 0xF, int BANK = 0xF>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), CTRL, ROW, BANK, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW, BANK, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }
__device__ __forceinline__ double lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Wave sum in registers: pairs, quads (quad_perm), 8 lanes (row_half_mirror),
// 16-lane rows (row_mirror), then row_bcast15 / row_bcast31 carry the row
// sums up so lane 63 holds the total, which is broadcast.  Fixed order, so
// the result is deterministic.
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v) {
  v += dpp_mov<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);       // row_half_mirror
  v += dpp_mov<0x140>(v);       // row_mirror
  v += dpp_mov<0x142, 0xA>(v);  // row_bcast15 into rows 1, 3
  v += dpp_mov<0x143, 0xC>(v);  // row_bcast31 into rows 2, 3
  return lane63(v);
}
__device__ __forceinline__ float wave_sum(float v) { return wave_sum_dpp(v); }
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

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

template <int BLOCK, typename T>
__device__ __forceinline__ void block_sum3(T& a, T& b, T& c, T* red) {
  constexpr int NW = BLOCK / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (lane == 0) {
    red[3 * w] = a;
    red[3 * w + 1] = b;
    red[3 * w + 2] = c;
  }
  __syncthreads();
  T sa = red[0], sb = red[1], sc = red[2];
#pragma unroll
  for (int i = 1; i < NW; ++i) {
    sa += red[3 * i];
    sb += red[3 * i + 1];
    sc += red[3 * i + 2];
  }
  a = sa;
  b = sb;
  c = sc;
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
