// Evaluation and post-processing of a usFFT result.
//
// Evaluation (Sec. 3.1, eq. (3.1) at the model's inverse periodization,
// Sec. 3.2):  u(x_g, y_j) ~ Re sum_{k in I} c_{k,g} e^{2 pi i k . phi^{-1}(y_j)}.
// For many points this is a dense contraction: with K = 2 |I| rows
//     B[2a][j] = cos(2 pi k_a . t_j),  B[2a+1][j] = -sin(2 pi k_a . t_j),
//     A[g][2a] = Re c_{a,g},           A[g][2a+1] = Im c_{a,g},
// the values are the float64 product A B (G x n).  It runs on the matrix
// cores (v_mfma_f64_16x16x4f64) in 64 x 64 tiles: A comes straight from the
// k-major coefficient array (the real and imaginary parts of one frequency
// are adjacent, so a K-slice of 16 is 8 frequencies x 64 nodes, 1 KB runs),
// B from a phase matrix computed once per chunk of points.  Two epilogues:
// write the values (usfft_eval), or fold them into the error measures of
// Sec. 4 against float64 finite-element solutions at the same parameters
// (usfft_errors): per node the sum of |u_FE - u_usFFT|^p and the maximum,
// reduced over the tile's 64 points in registers and LDS and written per
// (point tile, node); a second pass adds the tiles in a fixed order.
//
// Statistics (Sec. 4, Sec. 4.1), one thread per node, frequencies in order:
//     E     = sum_k c_k D_k  (D_k: 1 at k = 0 for the periodic model; a
//             product of 2i/(pi k_j) (odd k_j), 1 (k_j = 0), 0 (other) for the
//             affine one, times e^{2 pi i k_j Delta} for the lognormal one),
//     var   = sum_{k != 0} |c_k|^2,
//     gsi_l = sum_{||k||_0 = l} |c_k|^2 / var   (0 where var = 0).
#include "kernels.h"

namespace usfft {

typedef double double4v __attribute__((ext_vector_type(4)));

constexpr int kTileG = 64;  // nodes per tile
constexpr int kTileJ = 64;  // points per tile
constexpr int kSlice = 16;  // contraction rows staged per step
constexpr int kLdA = kTileG + 2;
constexpr int kLdB = kTileJ + 2;

// parameter y -> point of the torus (inverse periodization, Sec. 3.2)
__device__ __forceinline__ double param_to_node(int model, double alpha, double beta, double delta, double v) {
  if (model == USFFT_MODEL_AFFINE) return (v - alpha) / (2.0 * (beta - alpha));
  if (model == USFFT_MODEL_LOGNORMAL) return 0.25 * erf(v * 0.7071067811865476) + delta + 0.25;
  return v;
}

// T[q * ldt + j] = phi^{-1}(Y[j * d + q]), j < n
__global__ void node_map_kernel(const double* __restrict__ Y, int64_t n, int d, int model, double alpha, double beta,
                                double delta, double* __restrict__ T, int64_t ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  const int64_t j = e / d;
  const int q = (int)(e % d);
  T[q * ldt + j] = param_to_node(model, alpha, beta, delta, Y[e]);
}

// B[(2a) ldb + j] = cos(2 pi k_a . t_j), B[(2a+1) ldb + j] = -sin(2 pi k_a . t_j);
// blockIdx.y walks the frequencies in steps of gridDim.y.
__global__ __launch_bounds__(256) void phase_kernel(const int32_t* __restrict__ I, int64_t nI, int d,
                                                    const double* __restrict__ T, int64_t ldt, int64_t n,
                                                    double* __restrict__ B, int64_t ldb) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  for (int64_t a = blockIdx.y; a < nI; a += gridDim.y) {
    double ph = 0.0;
    for (int q = 0; q < d; ++q) ph += (double)I[a * d + q] * T[q * ldt + j];
    ph -= floor(ph);
    double s, c;
    sincospi(2.0 * ph, &s, &c);
    B[(2 * a) * ldb + j] = c;
    B[(2 * a + 1) * ldb + j] = -s;
  }
}

// Out = A B over one 64 x 64 tile per workgroup (see the file comment).
// Wave w covers nodes 32 (w >> 1) .. +31 and points 32 (w & 1) .. +31 as
// 2 x 2 blocks of 16 x 16.  MODE 0 writes out[j * ldo + g]; MODE 1 writes
// the per-tile error partials psum / pmax[jt * G + g].
template <int MODE>
__global__ __launch_bounds__(256) void evgemm_kernel(const double* __restrict__ C, int64_t G, int64_t nI,
                                                     const double* __restrict__ B, int64_t ldb, int64_t n,
                                                     int64_t ntg, double* __restrict__ out, int64_t ldo,
                                                     const double* __restrict__ U, int64_t ldu, double p, int pkind,
                                                     double* __restrict__ psum, double* __restrict__ pmax) {
  __shared__ double As[kSlice][kLdA];
  __shared__ double Bs[kSlice][kLdB];
  __shared__ double rs[2][kTileG];
  __shared__ double rm[2][kTileG];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the node tiles of one point tile are neighbouring items, and xcd_remap
  // keeps neighbouring items on one XCD: they share that tile's phases in L2
  const int64_t item = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t jt = item / ntg, gt = item % ntg;
  const int64_t g0 = gt * kTileG, j0 = jt * kTileJ;
  const int64_t K = 2 * nI;
  const int gw = 32 * (w >> 1), jw = 32 * (w & 1), l16 = lane & 15, lq = lane >> 4;
  double4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = double4v{0.0, 0.0, 0.0, 0.0};
  // staging roles: A slice = 8 frequencies x 64 nodes x (re, im): thread ->
  // frequency tid >> 5, nodes 2 (tid & 31) + h; B slice = 16 rows x 64
  // points: thread -> row tid >> 4, points 4 (tid & 15) + h
  const int sa = tid >> 5, sg = 2 * (tid & 31), sr = tid >> 4, sj = 4 * (tid & 15);
  for (int64_t k0 = 0; k0 < K; k0 += kSlice) {
    const int64_t a = k0 / 2 + sa;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t g = g0 + sg + h;
      double re = 0.0, im = 0.0;
      if (a < nI && g < G) {
        const double2 v = *reinterpret_cast<const double2*>(C + (a * G + g) * 2);
        re = v.x;
        im = v.y;
      }
      As[2 * sa][sg + h] = re;
      As[2 * sa + 1][sg + h] = im;
    }
    const int64_t kr = k0 + sr;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int64_t j = j0 + sj + h;
      Bs[sr][sj + h] = (kr < K && j < n) ? B[kr * ldb + j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSlice / 4; ++s) {
      const int r = 4 * s + lq;
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        av[i] = As[r][gw + 16 * i + l16];
        bv[i] = Bs[r][jw + 16 * i + l16];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[jj], acc[i][jj], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element v of block (i, jj): node gw + 16 i + lq + 4 v,
  // point jw + 16 jj + l16 (the float64 16x16 result holds rows lq, lq + 4,
  // lq + 8, lq + 12 in one lane)
  if constexpr (MODE == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t g = g0 + gw + 16 * i + lq + 4 * v, j = j0 + jw + 16 * jj + l16;
          if (g < G && j < n) out[j * ldo + g] = acc[i][jj][v];
        }
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t g = g0 + gw + 16 * i + lq + 4 * v;
        double s = 0.0, m = 0.0;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int64_t j = j0 + jw + 16 * jj + l16;
          if (g < G && j < n) {
            const double e = fabs(U[g * ldu + j] - acc[i][jj][v]);
            s += pkind == 2 ? e * e : (pkind == 1 ? e : pow(e, p));
            m = fmax(m, e);
          }
        }
        // the 16 lanes of a row group hold the same node
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) {
          s += __shfl_xor(s, o, 16);
          m = fmax(m, __shfl_xor(m, o, 16));
        }
        if (l16 == 0) {
          rs[w & 1][gw + 16 * i + lq + 4 * v] = s;
          rm[w & 1][gw + 16 * i + lq + 4 * v] = m;
        }
      }
    __syncthreads();
    if (tid < kTileG && g0 + tid < G) {
      psum[jt * G + g0 + tid] = rs[0][tid] + rs[1][tid];
      pmax[jt * G + g0 + tid] = fmax(rm[0][tid], rm[1][tid]);
    }
  }
}

// acc_s[g] (+)= sum over point tiles of psum, acc_m[g] = max(...), tiles in order
__global__ void err_accum_kernel(const double* __restrict__ psum, const double* __restrict__ pmax, int64_t njt,
                                 int64_t G, int first, double* __restrict__ acc_s, double* __restrict__ acc_m) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  double s = first ? 0.0 : acc_s[g], m = first ? 0.0 : acc_m[g];
  for (int64_t t = 0; t < njt; ++t) {
    s += psum[t * G + g];
    m = fmax(m, pmax[t * G + g]);
  }
  acc_s[g] = s;
  acc_m[g] = m;
}

// err_p = (sum / n)^(1/p) in place
__global__ void err_final_kernel(double* __restrict__ errp, int64_t G, int64_t n, double p, int pkind) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const double mean = errp[g] / (double)n;
  errp[g] = pkind == 2 ? sqrt(mean) : (pkind == 1 ? mean : pow(mean, 1.0 / p));
}

// D_k (complex) and ||k||_0 of every frequency
__global__ void dfactor_kernel(const int32_t* __restrict__ I, int64_t nI, int d, int model, double delta,
                               double* __restrict__ D, int32_t* __restrict__ ord) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nI) return;
  double re = 1.0, im = 0.0;
  int o = 0;
  for (int q = 0; q < d; ++q) {
    const int k = I[a * d + q];
    if (k == 0) continue;
    ++o;
    if (model == USFFT_MODEL_PERIODIC || (k % 2) == 0) {
      re = im = 0.0;
      continue;
    }
    // 2i / (pi k), times e^{2 pi i k delta} for the lognormal model
    const double r = 2.0 / (3.141592653589793 * (double)k);
    double fr = 0.0, fi = r;
    if (model == USFFT_MODEL_LOGNORMAL) {
      double sn, cs;
      sincospi(2.0 * (double)k * delta, &sn, &cs);
      fr = -r * sn;
      fi = r * cs;
    }
    const double nr = re * fr - im * fi, ni = re * fi + im * fr;
    re = nr;
    im = ni;
  }
  D[2 * a] = re;
  D[2 * a + 1] = im;
  ord[a] = o;
}

// one node per thread, frequencies in order; per-order sums in LDS
__global__ __launch_bounds__(64) void stats_kernel(const double* __restrict__ C, int64_t nI, int64_t G, int d,
                                                   const double* __restrict__ D, const int32_t* __restrict__ ord,
                                                   double* __restrict__ mean, double* __restrict__ var,
                                                   double* __restrict__ gsi) {
  __shared__ double acc[kMaxD][64];
  const int t = threadIdx.x;
  const int64_t g = (int64_t)blockIdx.x * 64 + t;
  for (int l = 0; l < d; ++l) acc[l][t] = 0.0;
  if (g >= G) return;
  double mr = 0.0, mi = 0.0;
  for (int64_t a = 0; a < nI; ++a) {
    const double2 c = *reinterpret_cast<const double2*>(C + (a * G + g) * 2);
    const double dr = D[2 * a], di = D[2 * a + 1];
    mr += c.x * dr - c.y * di;
    mi += c.x * di + c.y * dr;
    const int o = ord[a];
    if (o > 0) acc[o - 1][t] += c.x * c.x + c.y * c.y;
  }
  double v = 0.0;
  for (int l = 0; l < d; ++l) v += acc[l][t];
  if (mean) {
    mean[2 * g] = mr;
    mean[2 * g + 1] = mi;
  }
  if (var) var[g] = v;
  if (gsi)
    for (int l = 0; l < d; ++l) gsi[l * G + g] = v > 0.0 ? acc[l][t] / v : 0.0;
}

// ---------------------------------------------------------------- host side
void launch_node_map(const double* Y, int64_t n, int d, int model, double alpha, double beta, double delta,
                     double* T, int64_t ldt, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(node_map_kernel, dim3((unsigned)ceil_div(n * d, 256)), dim3(256), 0, st, Y, n, d, model, alpha,
                     beta, delta, T, ldt);
  USFFT_HIP(hipGetLastError());
}

void launch_phases(const int32_t* I, int64_t nI, int d, const double* T, int64_t ldt, int64_t n, double* B,
                   int64_t ldb, hipStream_t st) {
  if (n <= 0 || nI <= 0) return;
  const unsigned gy = (unsigned)std::min<int64_t>(nI, 256);
  hipLaunchKernelGGL(phase_kernel, dim3((unsigned)ceil_div(n, 256), gy), dim3(256), 0, st, I, nI, d, T, ldt, n, B,
                     ldb);
  USFFT_HIP(hipGetLastError());
}

void launch_evgemm_values(const double* C, int64_t G, int64_t nI, const double* B, int64_t ldb, int64_t n,
                          double* out, int64_t ldo, hipStream_t st) {
  if (n <= 0 || G <= 0) return;
  const int64_t ntg = ceil_div(G, kTileG), ntj = ceil_div(n, kTileJ);
  hipLaunchKernelGGL(evgemm_kernel<0>, dim3((unsigned)(ntg * ntj)), dim3(256), 0, st, C, G, nI, B, ldb, n, ntg, out,
                     ldo, nullptr, 0, 0.0, 0, nullptr, nullptr);
  USFFT_HIP(hipGetLastError());
}

int64_t evgemm_tiles_j(int64_t n) { return ceil_div(n, kTileJ); }

void launch_evgemm_errors(const double* C, int64_t G, int64_t nI, const double* B, int64_t ldb, int64_t n,
                          const double* U, int64_t ldu, double p, double* psum, double* pmax, int first,
                          double* acc_s, double* acc_m, hipStream_t st) {
  if (n <= 0 || G <= 0) return;
  const int pkind = p == 2.0 ? 2 : (p == 1.0 ? 1 : 0);
  const int64_t ntg = ceil_div(G, kTileG), ntj = ceil_div(n, kTileJ);
  hipLaunchKernelGGL(evgemm_kernel<1>, dim3((unsigned)(ntg * ntj)), dim3(256), 0, st, C, G, nI, B, ldb, n, ntg,
                     nullptr, 0, U, ldu, p, pkind, psum, pmax);
  USFFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(err_accum_kernel, dim3((unsigned)ceil_div(G, 256)), dim3(256), 0, st, psum, pmax, ntj, G, first,
                     acc_s, acc_m);
  USFFT_HIP(hipGetLastError());
}

void launch_err_final(double* errp, int64_t G, int64_t n, double p, hipStream_t st) {
  if (G <= 0) return;
  const int pkind = p == 2.0 ? 2 : (p == 1.0 ? 1 : 0);
  hipLaunchKernelGGL(err_final_kernel, dim3((unsigned)ceil_div(G, 256)), dim3(256), 0, st, errp, G, n, p, pkind);
  USFFT_HIP(hipGetLastError());
}

void launch_stats(const int32_t* I, int64_t nI, int d, const double* C, int64_t G, int model, double delta,
                  double* D, int32_t* ord, double* mean, double* var, double* gsi, hipStream_t st) {
  if (G <= 0) return;
  if (nI > 0) {
    hipLaunchKernelGGL(dfactor_kernel, dim3((unsigned)ceil_div(nI, 256)), dim3(256), 0, st, I, nI, d, model, delta,
                       D, ord);
    USFFT_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(stats_kernel, dim3((unsigned)ceil_div(G, 64)), dim3(64), 0, st, C, nI, G, d, D, ord, mean, var,
                     gsi);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
