// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state += 0x9E3779B97F4A7C15,
// output the variant-13 finalizer of the state.  Keyed per use: key =
// out(seed + gamma (stream + 1)), draw(idx) = out(key + gamma (idx + 1)).
// Usable on the host and on the device.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace usfft {
namespace rng {
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
__host__ __device__ inline uint64_t fin(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t stream(int kind, int t, int a, int b) {
  return ((uint64_t)(kind & 0xFF) << 56) | ((uint64_t)(t & 0xFFFF) << 40) | ((uint64_t)(a & 0xFFFFFF) << 16) |
         (uint64_t)(b & 0xFFFF);
}
__host__ __device__ inline uint64_t draw(uint64_t seed, uint64_t st, uint64_t idx) {
  const uint64_t key = fin(seed + kGamma * (st + 1));
  return fin(key + kGamma * (idx + 1));
}
__host__ __device__ inline double uniform01(uint64_t seed, uint64_t st, uint64_t idx) {
  return (double)(draw(seed, st, idx) >> 11) * (1.0 / 9007199254740992.0);
}
// generator of try b of lattice attempt a: z_j = 1 + draw mod (M - 1)
__host__ __device__ inline int32_t lattice_z(uint64_t seed, int kind, int tcode, int a, int b, int j, int M) {
  return (int32_t)(1 + draw(seed, stream(kind, tcode, a, b), (uint64_t)j) % (uint64_t)(M - 1));
}
enum { kTail1 = 1, kTail2 = 2, kLat2 = 3, kLat3 = 4 };
}  // namespace rng
}  // namespace usfft
