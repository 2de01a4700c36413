// Integer set work of the usFFT (Alg. 1 step 2): candidate product, detected
// set compaction and the alias tests of the lattice-family planner.  All of it
// is exact integer arithmetic, so results are bit-identical to any correct
// implementation.
#include "kernels.h"
#include "rng.h"

namespace usfft {

// J = parent x child, parent-major: row p*nc + c = (parent[p], child[c]).
__global__ void product_kernel(const int32_t* __restrict__ parent, int64_t np, int t,
                               const int32_t* __restrict__ child, int64_t nc, int32_t* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = t + 1;
  if (e >= np * nc * w) return;
  const int64_t row = e / w;
  const int j = (int)(e % w);
  const int64_t p = row / nc, c = row % nc;
  out[e] = (j < t) ? parent[p * t + j] : child[c];
}

void launch_product(const int32_t* parent, int64_t np, int t, const int32_t* child, int64_t nc, int32_t* out,
                    hipStream_t st) {
  const int64_t tot = np * nc * (t + 1);
  if (tot <= 0) return;
  hipLaunchKernelGGL(product_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, st, parent, np, t, child, nc,
                     out);
  USFFT_HIP(hipGetLastError());
}

// Order-keeping compaction with one workgroup: chunks of 1024 candidates,
// ballot + popcount prefix within waves, wave offsets through LDS.
constexpr int kCompactBlock = 1024;
__global__ __launch_bounds__(kCompactBlock) void compact_kernel(const int32_t* __restrict__ J,
                                                                const uint32_t* __restrict__ mask, int64_t n, int t,
                                                                int32_t* __restrict__ out,
                                                                int64_t* __restrict__ count) {
  __shared__ int wave_cnt[kCompactBlock / kWave];
  __shared__ int64_t base_s;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  for (int64_t a0 = 0; a0 < n; a0 += kCompactBlock) {
    const int64_t a = a0 + threadIdx.x;
    const bool keep = a < n && ((mask[a >> 5] >> (a & 31)) & 1u);
    const uint64_t bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[w] = __popcll(bal);
    __syncthreads();
    int64_t off = base_s;
    for (int i = 0; i < w; ++i) off += wave_cnt[i];
    if (keep) {
      const int64_t dst = off + before;
      for (int j = 0; j < t; ++j) out[dst * t + j] = J[a * t + j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int i = 0; i < kCompactBlock / kWave; ++i) tot += wave_cnt[i];
      base_s += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base_s;
}

void launch_compact(const int32_t* J, const uint32_t* mask, int64_t n, int t, int32_t* out, int64_t* count_dev,
                    hipStream_t st) {
  hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kCompactBlock), 0, st, J, mask, n, t, out, count_dev);
  USFFT_HIP(hipGetLastError());
}

// The T tries of lattice attempt a, one workgroup each: the try's generator
// z_tr (the draw of rng::lattice_z), bins[tr][a] = (k_a . z_tr) mod M of
// every candidate, the alias counts per bin (in LDS, then copied to
// counts[tr][.] for the commit) and the score #{a uncovered :
// counts[tr][bins[tr][a]] == 1}.
constexpr int kTryBlock = 1024;
__global__ __launch_bounds__(kTryBlock) void lattice_try_kernel(uint64_t seed, int kind, int tcode, int a, int t,
                                                                int M, const int32_t* __restrict__ J, int64_t n,
                                                                const uint8_t* __restrict__ covered,
                                                                int32_t* __restrict__ z, int32_t* __restrict__ bins,
                                                                int32_t* __restrict__ counts,
                                                                int32_t* __restrict__ scores) {
  extern __shared__ int32_t cnt[];  // M alias counts
  __shared__ int32_t zs[kMaxD];
  __shared__ int32_t wsum[kTryBlock / kWave];
  const int tr = blockIdx.x;
  for (int i = threadIdx.x; i < M; i += kTryBlock) cnt[i] = 0;
  if (threadIdx.x < t) {
    const int32_t zj = rng::lattice_z(seed, kind, tcode, a, tr, threadIdx.x, M);
    zs[threadIdx.x] = zj;
    z[tr * t + threadIdx.x] = zj;
  }
  __syncthreads();
  int32_t* bt = bins + (int64_t)tr * n;
  for (int64_t e = threadIdx.x; e < n; e += kTryBlock) {
    int64_t acc = 0;
    for (int j = 0; j < t; ++j) acc += (int64_t)J[e * t + j] * (int64_t)zs[j];
    int64_t bn = acc % M;
    if (bn < 0) bn += M;
    bt[e] = (int32_t)bn;
    atomicAdd(&cnt[bn], 1);
  }
  __syncthreads();
  int32_t* ct = counts + (int64_t)tr * M;
  for (int i = threadIdx.x; i < M; i += kTryBlock) ct[i] = cnt[i];
  int c = 0;
  for (int64_t e = threadIdx.x; e < n; e += kTryBlock) c += (!covered[e] && cnt[bt[e]] == 1) ? 1 : 0;
  c = wave_sum(c);
  if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < kTryBlock / kWave; ++w) tot += wsum[w];
    scores[tr] = tot;
  }
}

void launch_lattice_try(uint64_t seed, int kind, int tcode, int a, int T, int t, int M, const int32_t* J, int64_t n,
                        const uint8_t* covered, int32_t* z, int32_t* bins, int32_t* counts, int32_t* scores,
                        hipStream_t st) {
  USFFT_REQUIRE(T >= 1 && t >= 1 && t <= kMaxD && M >= 1 && M <= kMaxLattice && n >= 1, USFFT_EINVAL,
                "bad lattice try shape");
  hipLaunchKernelGGL(lattice_try_kernel, dim3((unsigned)T), dim3(kTryBlock), sizeof(int32_t) * (size_t)M, st, seed,
                     kind, tcode, a, t, M, J, n, covered, z, bins, counts, scores);
  USFFT_HIP(hipGetLastError());
}

// The choice and commit of one attempt on the device: the try that frees
// the most still-uncovered candidates (lowest index on ties).  Every
// workgroup finds it from the T scores.  state_in = (uncovered candidates,
// lattices taken) before the attempt is only read; workgroup 0 writes
// state_out and log = (best, freed), freed = 0 when the attempt takes nothing
// (no candidate freed, or none left).  A candidate is committed to the new
// lattice when it was uncovered and its bin holds no other candidate.
__global__ void lattice_pick_take_kernel(const int32_t* __restrict__ scores, int T,
                                         const int64_t* __restrict__ state_in, int64_t* __restrict__ state_out,
                                         int32_t* __restrict__ log, const int32_t* __restrict__ bins,
                                         const int32_t* __restrict__ counts, uint8_t* __restrict__ covered,
                                         int64_t n, int M, int32_t* __restrict__ assign,
                                         int32_t* __restrict__ bin_out) {
  int best = 0;
  for (int b = 1; b < T; ++b)
    if (scores[b] > scores[best]) best = b;
  const int64_t uncovered = state_in[0], taken = state_in[1];
  const int freed = uncovered > 0 ? scores[best] : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    log[0] = best;
    log[1] = freed;
    state_out[0] = uncovered - freed;
    state_out[1] = taken + (freed > 0 ? 1 : 0);
  }
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n || freed == 0) return;
  const int32_t b = bins[(int64_t)best * n + a];
  if (!covered[a] && counts[(int64_t)best * M + b] == 1) {
    covered[a] = 1;
    assign[a] = (int32_t)taken;  // index of the lattice this attempt adds
    bin_out[a] = b;
  }
}

void launch_lattice_pick_take(const int32_t* scores, int T, const int64_t* state_in, int64_t* state_out,
                              int32_t* log, const int32_t* bins, const int32_t* counts, uint8_t* covered, int64_t n,
                              int M, int32_t* assign, int32_t* bin_out, hipStream_t st) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, ceil_div(n, 256));
  hipLaunchKernelGGL(lattice_pick_take_kernel, dim3(grid), dim3(256), 0, st, scores, T, state_in, state_out, log,
                     bins, counts, covered, n, M, assign, bin_out);
  USFFT_HIP(hipGetLastError());
}

__global__ void ungroup_mask_kernel(const uint32_t* __restrict__ in, const int32_t* __restrict__ pos, int64_t n,
                                    uint32_t* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  if ((in[q >> 5] >> (q & 31)) & 1u) {
    const int32_t a = pos[q];
    atomicOr(&out[a >> 5], 1u << (a & 31));
  }
}

void launch_ungroup_mask(const uint32_t* mask_in, const int32_t* pos, int64_t n, uint32_t* mask_out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(ungroup_mask_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, mask_in, pos, n,
                     mask_out);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
