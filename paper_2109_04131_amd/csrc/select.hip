// Per-node selection and uniform union (Alg. 1 step 1&2a and steps 2d/2e).
//
// For node g the candidates are kept whose |coefficient| is among the s~
// largest and at least theta; the detected set is the union over all nodes.
// tau_g^2, the s~-th largest squared magnitude of column g (with
// multiplicity), is found by an exact MSB-first radix select on the bit
// patterns of the non-negative float64 values (their unsigned order is the
// numeric order): up to 8 passes of 8-bit digits with an LDS histogram, over
// the column staged once in LDS when it fits.  As soon as at most kSelFew keys
// share the digits fixed so far, they are gathered and ranked pairwise, which
// fixes the remaining bits at once (the digits of the first passes are mostly
// exponent bits; after two or three passes few keys remain).  A column with
// fewer than s~ keys v whose (1 - tie) v reaches theta^2 (counted while it is
// staged) needs no select: its threshold is theta^2 whatever tau_g^2 is.  A
// candidate is kept when v >= max(theta^2, (1 - tie) tau_g^2); each wave ORs
// its 64 keep bits into the global candidate mask, with an atomic only for
// bits not yet set.
#include "kernels.h"

namespace usfft {

constexpr int kSelBlock = 256;

constexpr int kSelLds = 8192;  // columns up to this length are staged in LDS (64 KB)
constexpr int kSelFew = 64;    // candidate count that ends the radix passes

// One column block per launch, or (lineK != null) the step-1 lines in one
// launch: blockIdx.y = line y of coordinate t = y / line_r, its K_t = lineK[t]
// candidates in columns y * line_stride .. of v, its mask words after those
// of the coordinates before t.
template <bool STAGE>
__global__ __launch_bounds__(kSelBlock) void select_kernel(const double* __restrict__ v, int64_t G, int64_t n,
                                                           int64_t ld, int s_tilde,
                                                           const double* __restrict__ theta2p, double tie_rel,
                                                           uint32_t* __restrict__ mask, double* __restrict__ thr_out,
                                                           const int32_t* __restrict__ lineK, int line_r,
                                                           int64_t line_stride) {
  if (!lineK) {
    v += (int64_t)blockIdx.y * line_stride;  // iteration blocks (one block: y = 0)
  } else {
    const int y = blockIdx.y, t = y / line_r;
    int64_t w = 0;
    for (int j = 0; j < t; ++j) w += (lineK[j] + 31) / 32;
    n = lineK[t];
    v += (int64_t)y * line_stride;
    mask += w;
  }
  extern __shared__ uint64_t stage[];
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int64_t s_rank;
  __shared__ uint32_t s_cnt, s_nfew;
  __shared__ uint64_t few[kSelFew];
  __shared__ uint32_t wabove[kSelBlock / kWave];
  // LDS-staged columns: the keep bits of all columns of this workgroup are
  // ORed here first and reach the global mask once at the end, so the G
  // columns do not all contend for the same few mask words
  __shared__ uint32_t lmask[kSelLds / 32];
  const int64_t words = (n + 31) / 32;
  if (STAGE)
    for (int64_t i = threadIdx.x; i < words; i += kSelBlock) lmask[i] = 0u;
  for (int64_t g = xcd_remap(blockIdx.x, gridDim.x); g < G; g += gridDim.x) {
    __syncthreads();  // the previous column is done with the stage and wabove
    const uint64_t* gkeys = reinterpret_cast<const uint64_t*>(v + g * ld);
    // Keys whose tie-scaled value reaches theta^2: when fewer than s~ do, the
    // s~-th largest key tau^2 has (1 - tie) tau^2 < theta^2 (the rounded
    // product is monotone in the key), so the threshold is theta^2 whatever
    // tau^2 is and the radix select is skipped.
    const double theta2 = *theta2p, keepf = 1.0 - tie_rel;
    uint32_t above = 0;
    if (STAGE) {
      // eight loads in flight per thread before their LDS stores: the column
      // comes from HBM, and one load at a time would wait out its latency
      constexpr int U = 8;
      for (int64_t a0 = threadIdx.x; a0 < n; a0 += U * kSelBlock) {
        uint64_t k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t a = a0 + u * kSelBlock;
          k[u] = a < n ? gkeys[a] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t a = a0 + u * kSelBlock;
          if (a < n) {
            stage[a] = k[u];
            above += keepf * __longlong_as_double((long long)k[u]) >= theta2;
          }
        }
      }
    } else {
      for (int64_t a = threadIdx.x; a < n; a += kSelBlock)
        above += keepf * __longlong_as_double((long long)gkeys[a]) >= theta2;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) above += __shfl_xor(above, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) wabove[threadIdx.x / kWave] = above;
    __syncthreads();
    above = 0;
#pragma unroll
    for (int w = 0; w < kSelBlock / kWave; ++w) above += wabove[w];
    const uint64_t* keys = STAGE ? stage : gkeys;
    double tau2 = 0.0;
    if (s_tilde > 0 && n >= s_tilde && above >= (uint32_t)s_tilde) {
      uint64_t prefix = 0;   // digits fixed so far
      int64_t rank = s_tilde;  // 1-based rank from the top among matching keys
      for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += kSelBlock) hist[i] = 0;
        __syncthreads();
        const uint64_t hmask = (shift == 56) ? 0ull : (~0ull << (shift + 8));
        const int lane = threadIdx.x & (kWave - 1);
        for (int64_t a0 = threadIdx.x - lane; a0 < n; a0 += kSelBlock) {
          // wave-aggregated increments: the digits of a column concentrate on a
          // few bins (shared exponent bits), so the wave's most common case
          // (the first active lane's digit) is counted with one atomic
          const int64_t a = a0 + lane;
          const uint64_t k = a < n ? keys[a] : 0ull;
          const bool act = a < n && (k & hmask) == prefix;
          const uint32_t dg = (uint32_t)(k >> shift) & 255u;
          const uint64_t actm = __ballot(act);
          if (actm) {
            const int first = __ffsll((unsigned long long)actm) - 1;
            const uint32_t lead = __shfl(dg, first, kWave);
            const uint64_t same = __ballot(act && dg == lead);
            if (lane == first) atomicAdd(&hist[lead], (uint32_t)__popcll(same));
            if (act && dg != lead) atomicAdd(&hist[dg], 1u);
          }
        }
        __syncthreads();
        if (threadIdx.x < kWave) {
          // wave 0 finds the digit holding the rank-th largest key: lane l owns
          // bins 255-4l .. 252-4l, an inclusive prefix over lanes gives the
          // count of larger keys, exactly one lane contains the rank.
          const int l = threadIdx.x;
          uint32_t h[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) h[i] = hist[255 - 4 * l - i];
          const uint32_t c = h[0] + h[1] + h[2] + h[3];
          uint32_t inc = c;
#pragma unroll
          for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, kWave);
            if (l >= o) inc += t;
          }
          const int64_t exc = (int64_t)(inc - c);
          if (exc < rank && (int64_t)inc >= rank) {
            int64_t acc = exc;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (acc + h[i] >= rank) {
                s_prefix = prefix | ((uint64_t)(255 - 4 * l - i) << shift);
                s_rank = rank - acc;
                s_cnt = h[i];  // keys that match the new prefix, rank <= h[i]
                break;
              }
              acc += h[i];
            }
          }
        }
        __syncthreads();
        prefix = s_prefix;
        rank = s_rank;
        const uint32_t cnt = s_cnt;
        if (threadIdx.x == 0) s_nfew = 0;
        __syncthreads();
        if (shift > 0 && cnt <= (uint32_t)kSelFew) {
          // the cnt keys whose bits from `shift` up equal the prefix; the
          // rank-th largest of them (with multiplicity) is the key k with
          // #{> k} < rank <= #{>= k}
          const uint64_t fmask = ~0ull << shift;
          for (int64_t a = threadIdx.x; a < n; a += kSelBlock) {
            const uint64_t k = keys[a];
            if ((k & fmask) == prefix) {
              const uint32_t i = atomicAdd(&s_nfew, 1u);
              if (i < (uint32_t)kSelFew) few[i] = k;
            }
          }
          __syncthreads();
          if (threadIdx.x < cnt) {
            const uint64_t k = few[threadIdx.x];
            uint32_t gt = 0, ge = 0;
            for (uint32_t j = 0; j < cnt; ++j) {
              const uint64_t o = few[j];
              gt += o > k;
              ge += o >= k;
            }
            if ((int64_t)gt < rank && rank <= (int64_t)ge) s_prefix = k;  // equal keys write the same value
          }
          __syncthreads();
          prefix = s_prefix;
          break;
        }
      }
      tau2 = __longlong_as_double((long long)prefix);
    }
    const double thr = fmax(theta2, keepf * tau2);
    if (thr_out && threadIdx.x == 0) thr_out[g] = thr;
    const double* col = STAGE ? reinterpret_cast<const double*>(stage) : v + g * ld;
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t a0 = (int64_t)(threadIdx.x - lane); a0 < n; a0 += kSelBlock) {
      const int64_t a = a0 + lane;
      const bool keep = a < n && col[a] >= thr;
      const uint64_t bal = __ballot(keep);
      if (STAGE) {
        if (lane == 0 && bal) {
          const int64_t w = a0 >> 5;  // a0 is a multiple of 64
          const uint32_t lo = (uint32_t)(bal & 0xffffffffull), hi = (uint32_t)(bal >> 32);
          if (lo) atomicOr(&lmask[w], lo);
          if (hi) atomicOr(&lmask[w + 1], hi);
        }
      } else if (lane == 0 && bal) {
        // Most nodes keep the same candidates, so most bits are already set by
        // other workgroups: check the word first (bits are only ever set, so a
        // stale read can only cost an unneeded atomic) and skip the atomic --
        // all G workgroups would otherwise serialise on the same few words.
        const int64_t w = a0 >> 5;  // a0 is a multiple of 64
        const uint32_t lo = (uint32_t)(bal & 0xffffffffull), hi = (uint32_t)(bal >> 32);
        if (lo && (__hip_atomic_load(&mask[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & lo) != lo)
          atomicOr(&mask[w], lo);
        if (hi && (__hip_atomic_load(&mask[w + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & hi) != hi)
          atomicOr(&mask[w + 1], hi);
      }
    }
  }  // columns of this workgroup
  if (STAGE) {
    __syncthreads();
    for (int64_t i = threadIdx.x; i < words; i += kSelBlock) {
      const uint32_t b = lmask[i];
      if (b && (__hip_atomic_load(&mask[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & b) != b)
        atomicOr(&mask[i], b);
    }
  }
}

// Workgroups per column set: each takes every gridDim.x-th column, enough of
// them to fill the GPU a few times over.
static unsigned select_blocks(int64_t G, int64_t sets) {
  const int64_t want = std::max<int64_t>(1, 4096 / std::max<int64_t>(sets, 1));
  return (unsigned)std::min<int64_t>(G, want);
}

void launch_select(const double* v, int64_t G, int64_t n, int64_t ld, int s_tilde, const double* theta2,
                   double tie_rel, uint32_t* mask, double* thr, hipStream_t st) {
  if (G <= 0 || n <= 0) return;
  if (n <= kSelLds)
    hipLaunchKernelGGL(select_kernel<true>, dim3(select_blocks(G, 1)), dim3(kSelBlock), (size_t)n * sizeof(uint64_t), st, v,
                       G, n, ld, s_tilde, theta2, tie_rel, mask, thr, nullptr, 1, 0);
  else
    hipLaunchKernelGGL(select_kernel<false>, dim3((unsigned)G), dim3(kSelBlock), 0, st, v, G, n, ld, s_tilde,
                       theta2, tie_rel, mask, thr, nullptr, 1, 0);
  USFFT_HIP(hipGetLastError());
}

void launch_select_iters(const double* v, int64_t G, int64_t n, int64_t ld, int niter, int64_t iter_stride,
                         int s_tilde, const double* theta2, double tie_rel, uint32_t* mask, hipStream_t st) {
  if (G <= 0 || n <= 0 || niter <= 0) return;
  const dim3 grid((unsigned)G, (unsigned)niter);
  if (n <= kSelLds)
    hipLaunchKernelGGL(select_kernel<true>, dim3(select_blocks(G, niter), (unsigned)niter), dim3(kSelBlock), (size_t)n * sizeof(uint64_t), st, v, G, n, ld,
                       s_tilde, theta2, tie_rel, mask, nullptr, nullptr, 1, iter_stride);
  else
    hipLaunchKernelGGL(select_kernel<false>, grid, dim3(kSelBlock), 0, st, v, G, n, ld, s_tilde, theta2, tie_rel,
                       mask, nullptr, nullptr, 1, iter_stride);
  USFFT_HIP(hipGetLastError());
}

void launch_select_lines(const double* v, int64_t G, int64_t ld, int nlines, int line_r, int64_t line_stride,
                         const int32_t* lineK, int Kmax, int s_tilde, const double* theta2, double tie_rel,
                         uint32_t* mask, hipStream_t st) {
  if (G <= 0 || nlines <= 0) return;
  USFFT_REQUIRE(Kmax >= 1 && Kmax <= kSelLds && line_stride >= Kmax, USFFT_EINVAL, "bad line selection shape");
  hipLaunchKernelGGL(select_kernel<true>, dim3(select_blocks(G, nlines), (unsigned)nlines), dim3(kSelBlock),
                     (size_t)Kmax * sizeof(uint64_t), st, v, G, (int64_t)Kmax, ld, s_tilde, theta2, tie_rel, mask,
                     nullptr, lineK, line_r, line_stride);
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
