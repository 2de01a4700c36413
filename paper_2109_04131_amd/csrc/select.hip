// Per-node selection and uniform union (Alg. 1 step 1&2a and steps 2d/2e).
//
// For node g the candidates are kept whose |coefficient| is among the s~
// largest and at least theta; the detected set is the union over all nodes.
// tau_g^2, the s~-th largest squared magnitude of column g (with
// multiplicity), is found by an exact MSB-first radix select on the bit
// patterns of the non-negative float64 values (their unsigned order is the
// numeric order): 8 passes of 8-bit digits with an LDS histogram.  A
// candidate is kept when v >= max(theta^2, (1 - tie) tau_g^2); each wave ORs
// its 64 keep bits into the global candidate mask with two word atomics.
#include "kernels.h"

namespace usfft {

constexpr int kSelBlock = 256;

__global__ __launch_bounds__(kSelBlock) void select_kernel(const double* __restrict__ v, int64_t G, int64_t n,
                                                           int64_t ld, int s_tilde,
                                                           const double* __restrict__ theta2p, double tie_rel,
                                                           uint32_t* __restrict__ mask, double* __restrict__ thr_out) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int64_t s_rank;
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x);
  const uint64_t* keys = reinterpret_cast<const uint64_t*>(v + g * ld);
  double tau2 = 0.0;
  if (s_tilde > 0 && n >= s_tilde) {
    uint64_t prefix = 0;   // digits fixed so far
    int64_t rank = s_tilde;  // 1-based rank from the top among matching keys
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int i = threadIdx.x; i < 256; i += kSelBlock) hist[i] = 0;
      __syncthreads();
      const uint64_t hmask = (shift == 56) ? 0ull : (~0ull << (shift + 8));
      for (int64_t a = threadIdx.x; a < n; a += kSelBlock) {
        const uint64_t k = keys[a];
        if ((k & hmask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int64_t acc = 0;
        int dsel = 0;
        for (int dgt = 255; dgt >= 0; --dgt) {
          if (acc + hist[dgt] >= rank) {
            dsel = dgt;
            break;
          }
          acc += hist[dgt];
        }
        s_prefix = prefix | ((uint64_t)dsel << shift);
        s_rank = rank - acc;
      }
      __syncthreads();
      prefix = s_prefix;
      rank = s_rank;
      __syncthreads();
    }
    tau2 = __longlong_as_double((long long)prefix);
  }
  const double thr = fmax(*theta2p, (1.0 - tie_rel) * tau2);
  if (thr_out && threadIdx.x == 0) thr_out[g] = thr;
  const double* col = v + g * ld;
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t a0 = (int64_t)(threadIdx.x - lane); a0 < n; a0 += kSelBlock) {
    const int64_t a = a0 + lane;
    const bool keep = a < n && col[a] >= thr;
    const uint64_t bal = __ballot(keep);
    if (lane == 0 && bal) {
      const int64_t w = a0 >> 5;  // a0 is a multiple of 64
      const uint32_t lo = (uint32_t)(bal & 0xffffffffull), hi = (uint32_t)(bal >> 32);
      if (lo) atomicOr(&mask[w], lo);
      if (hi) atomicOr(&mask[w + 1], hi);
    }
  }
}

void launch_select(const double* v, int64_t G, int64_t n, int64_t ld, int s_tilde, const double* theta2,
                   double tie_rel, uint32_t* mask, double* thr, hipStream_t st) {
  if (G <= 0 || n <= 0) return;
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)G), dim3(kSelBlock), 0, st, v, G, n, ld, s_tilde, theta2, tie_rel,
                     mask, thr);
  USFFT_HIP(hipGetLastError());
}

// theta2 = (theta * max |c|)^2 = theta^2 * max v over the stage's G x n values.
__global__ void max_bits_kernel(const double* __restrict__ v, int64_t G, int64_t n, int64_t ld,
                                unsigned long long* __restrict__ out) {
  const int64_t tot = G * n;
  unsigned long long best = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = e / n, a = e % n;
    const unsigned long long k = (unsigned long long)__double_as_longlong(v[g * ld + a]);
    best = k > best ? k : best;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, kWave);
    best = other > best ? other : best;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, best);
}

__global__ void theta_kernel(const unsigned long long* __restrict__ bits, double theta, double* __restrict__ theta2) {
  const double vmax = __longlong_as_double((long long)*bits);
  *theta2 = theta * theta * vmax;
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

void launch_max_to_theta(const double* v, int64_t G, int64_t n, int64_t ld, double theta, double* theta2,
                         uint64_t* scratch, hipStream_t st) {
  unsigned long long* s = reinterpret_cast<unsigned long long*>(scratch);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, st, s);
  const int64_t tot = G * n;
  const unsigned grid = (unsigned)std::min<int64_t>(1024, ceil_div(tot, 256));
  if (tot > 0) hipLaunchKernelGGL(max_bits_kernel, dim3(grid), dim3(256), 0, st, v, G, n, ld, s);
  hipLaunchKernelGGL(theta_kernel, dim3(1), dim3(1), 0, st, s, theta, theta2);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
