// Evaluation of the approximant (Sec. 3.1, eq. (3.1)):
// out[j, g] = Re sum_{k in I} c_k(u_{x_g}) exp(2 pi i k . phi^{-1}(y_j)),
// with phi^{-1} the inverse periodization of the model (Sec. 3.2): the
// identity (periodic), (y - alpha) / (2 (beta - alpha)) (affine) or
// erf(y / sqrt(2)) / 4 + delta + 1/4 (lognormal).
// One workgroup per evaluation point; the phases of a chunk of frequencies
// are staged in LDS, coefficients are read k-major so a wave reads 64
// consecutive nodes.  Not on the timed path.
#include "kernels.h"

namespace usfft {

constexpr int kEvalChunk = 1024;

__global__ __launch_bounds__(256) void eval_kernel(const int32_t* __restrict__ I, int64_t nI, int d,
                                                   const double* __restrict__ C, int64_t G,
                                                   const double* __restrict__ Y, int model, double alpha,
                                                   double beta, double delta, double* __restrict__ out) {
  __shared__ double cs[kEvalChunk];
  __shared__ double sn[kEvalChunk];
  __shared__ double y[kMaxD];
  const int64_t j = blockIdx.x;
  for (int q = threadIdx.x; q < d; q += 256) {
    const double v = Y[j * d + q];
    y[q] = model == USFFT_MODEL_AFFINE      ? (v - alpha) / (2.0 * (beta - alpha))
           : model == USFFT_MODEL_LOGNORMAL ? 0.25 * erf(v * 0.7071067811865476) + delta + 0.25
                                            : v;
  }
  __syncthreads();
  for (int64_t g0 = 0; g0 < G; g0 += 256) {
    const int64_t g = g0 + threadIdx.x;
    double acc = 0.0;
    for (int64_t a0 = 0; a0 < nI; a0 += kEvalChunk) {
      const int na = (int)min<int64_t>(kEvalChunk, nI - a0);
      __syncthreads();
      for (int a = threadIdx.x; a < na; a += 256) {
        double ph = 0.0;
        for (int q = 0; q < d; ++q) ph += (double)I[(a0 + a) * d + q] * y[q];
        ph -= floor(ph);
        sincospi(2.0 * ph, &sn[a], &cs[a]);
      }
      __syncthreads();
      if (g < G)
        for (int a = 0; a < na; ++a) {
          const double* c = C + ((a0 + a) * G + g) * 2;
          acc += c[0] * cs[a] - c[1] * sn[a];
        }
    }
    if (g < G) out[j * G + g] = acc;
  }
}

void launch_eval(const int32_t* I, int64_t nI, int d, const double* C, int64_t G, const double* Y, int64_t n,
                 int model, double alpha, double beta, double delta, double* out, hipStream_t st) {
  if (n <= 0 || G <= 0) return;
  hipLaunchKernelGGL(eval_kernel, dim3((unsigned)n), dim3(256), 0, st, I, nI, d, C, G, Y, model, alpha, beta,
                     delta, out);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
