// Black-box sampler of the usFFT (Sec. 2.1, Alg. 1 steps 1&2a, 2c, 3) on gfx950.
//
// One workgroup solves one PDE sample.  The P1 system of eq. (1.1)/(1.2) on
// the uniform mesh is a 5-point operator whose off-diagonal weights are edge
// weights w_e = (a_T1 + a_T2)/2 of the two right triangles sharing an
// axis-parallel edge (the hypotenuse couplings vanish), with diagonal equal to
// the sum of the four edge weights of a node and load h^2 for f = 1.  The
// workgroup assembles those weights from the centroid tables in registers,
// keeps x, r, p and the weights of its nodes in registers and only the search
// direction p in LDS (with a zero halo that carries the Dirichlet data), and
// runs Jacobi-preconditioned CG.  All reductions combine wave partials in a
// fixed order, so a sample's result does not depend on which block or batch
// runs it.
#include "kernels.h"

namespace usfft {

// ---------------------------------------------------------------- nodes
// Sampling nodes of one stage, one thread per (sample, coordinate).
__global__ void nodes_kernel(int d, int line, int t, int nlat, const int64_t* __restrict__ off,
                             const int32_t* __restrict__ Ms, const int32_t* __restrict__ zs,
                             const double* __restrict__ tail, double* __restrict__ Y, int64_t ns) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ns * d) return;
  const int64_t s = e / d;
  const int j = (int)(e % d);
  double y;
  if (line >= 0) {
    const int K = Ms[0];
    y = (j == line) ? (double)s / (double)K : tail[j];
  } else if (j >= t) {
    y = tail[j];
  } else {
    int l = 0;
    while (l + 1 < nlat && off[l + 1] <= s) ++l;
    const int64_t M = Ms[l];
    const int64_t m = s - off[l];
    const int64_t r = (m * (int64_t)zs[(int64_t)l * t + j]) % M;
    y = (double)r / (double)M;
  }
  Y[e] = y;
}

// ---------------------------------------------------------------- weights
// Centroid value of a on the lower (q=0) / upper (q=1) triangle of cell (ci, cj).
// tab holds sin(m1 pi x1), sin(m2 pi x2) at the centroid abscissae:
// [0] x1 of lower, [1] x1 of upper, [2] x2 of lower, [3] x2 of upper; each d x n.
__device__ __forceinline__ double tri_coef(const PdeDev& P, const double* coef, int q, int ci, int cj) {
  const double* tx = P.tab + (size_t)(q) * P.d * P.n;
  const double* ty = P.tab + (size_t)(2 + q) * P.d * P.n;
  double a = P.a0;
  for (int k = 0; k < P.d; ++k) a += coef[k] * tx[k * P.n + ci] * ty[k * P.n + cj];
  return a;
}

// The four edge weights of interior node (i, j), 1 <= i, j <= n-1.
__device__ __forceinline__ void node_weights(const PdeDev& P, const double* coef, int i, int j,
                                             double& wE, double& wW, double& wN, double& wS) {
  const double aL_ij = tri_coef(P, coef, 0, i, j);
  const double aU_ij = tri_coef(P, coef, 1, i, j);
  const double aU_ijm = tri_coef(P, coef, 1, i, j - 1);
  const double aL_imj = tri_coef(P, coef, 0, i - 1, j);
  const double aU_imjm = tri_coef(P, coef, 1, i - 1, j - 1);
  const double aL_imjm = tri_coef(P, coef, 0, i - 1, j - 1);
  wE = 0.5 * (aL_ij + aU_ijm);    // edge (i,j)-(i+1,j): lower of cell (i,j), upper of (i,j-1)
  wW = 0.5 * (aL_imj + aU_imjm);  // edge (i-1,j)-(i,j)
  wN = 0.5 * (aU_ij + aL_imj);    // edge (i,j)-(i,j+1): upper of cell (i,j), lower of (i-1,j)
  wS = 0.5 * (aU_ijm + aL_imjm);  // edge (i,j-1)-(i,j)
}

__device__ __forceinline__ void load_coef(const PdeDev& P, const double* __restrict__ Y, int64_t s,
                                          double* coef) {
  for (int k = threadIdx.x; k < P.d; k += blockDim.x) coef[k] = P.amp[k] * sinpi(2.0 * Y[s * P.d + k]);
}

template <typename T>
__device__ __forceinline__ void store_sample(void* out, int out_fp32, int64_t idx, T v) {
  if (out_fp32)
    static_cast<float*>(out)[idx] = (float)v;
  else
    static_cast<double*>(out)[idx] = (double)v;
}

// ---------------------------------------------------------------- FP64 PCG
template <int BLOCK, int NPT>
__global__ __launch_bounds__(BLOCK) void pcg64_kernel(PdeDev P, const double* __restrict__ Y, int64_t ns,
                                                      double rtol, int maxit, void* __restrict__ out,
                                                      int out_fp32, int64_t ld, int64_t col0,
                                                      int* __restrict__ iters) {
  extern __shared__ double sp[];  // (n+1)^2, zero halo = Dirichlet data
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  const int64_t s = xcd_remap(blockIdx.x, gridDim.x);
  const int n = P.n, m = n - 1, G = m * m, P1 = n + 1;
  load_coef(P, Y, s, coef);
  for (int e = threadIdx.x; e < P1 * P1; e += BLOCK) sp[e] = 0.0;
  __syncthreads();

  double x[NPT], r[NPT], p[NPT], wE[NPT], wW[NPT], wN[NPT], wS[NPT], di[NPT];
  int li[NPT];
  double rz = 0.0, bb = 0.0;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int g = threadIdx.x + k * BLOCK;
    x[k] = 0.0;
    if (g < G) {
      const int i = g % m + 1, j = g / m + 1;
      node_weights(P, coef, i, j, wE[k], wW[k], wN[k], wS[k]);
      di[k] = 1.0 / (wE[k] + wW[k] + wN[k] + wS[k]);
      li[k] = j * P1 + i;
      r[k] = P.h2;
      p[k] = di[k] * r[k];
      rz += r[k] * p[k];
      bb += r[k] * r[k];
    } else {
      wE[k] = wW[k] = wN[k] = wS[k] = di[k] = 0.0;
      r[k] = p[k] = 0.0;
      li[k] = P1 + 1;  // any interior slot: keeps the unused neighbour reads in bounds
    }
  }
  block_sum2<BLOCK>(rz, bb, red1);
  const double stop = rtol * rtol * bb;
  int it = 0;
  bool conv = false;
  while (it < maxit) {
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      if (threadIdx.x + k * BLOCK < G) sp[li[k]] = p[k];
    __syncthreads();
    double q[NPT];
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int l = li[k];
      q[k] = (wE[k] + wW[k] + wN[k] + wS[k]) * p[k] -
             (wE[k] * sp[l + 1] + wW[k] * sp[l - 1] + wN[k] * sp[l + P1] + wS[k] * sp[l - P1]);
      if (threadIdx.x + k * BLOCK >= G) q[k] = 0.0;
      pq += p[k] * q[k];
    }
    pq = block_sum<BLOCK>(pq, red0);
    const double alpha = rz / pq;
    double rz2 = 0.0, rr = 0.0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      x[k] += alpha * p[k];
      r[k] -= alpha * q[k];
      rz2 += r[k] * (di[k] * r[k]);
      rr += r[k] * r[k];
    }
    block_sum2<BLOCK>(rz2, rr, red1);
    ++it;
    if (rr <= stop) {
      conv = true;
      break;
    }
    const double beta = rz2 / rz;
    rz = rz2;
#pragma unroll
    for (int k = 0; k < NPT; ++k) p[k] = di[k] * r[k] + beta * p[k];
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int g = threadIdx.x + k * BLOCK;
    if (g < G) store_sample(out, out_fp32, (int64_t)g * ld + col0 + s, x[k]);
  }
  if (threadIdx.x == 0 && iters) iters[s] = conv ? it : -1;
}

// ------------------------------------------ FP32 PCG with FP64 refinement
// Outer loop in float64: r = b - A(y) x with weights recomputed in float64;
// inner loop: float32 Jacobi-PCG on A d = r / |r| to inner_rtol; x += |r| d.
template <int BLOCK, int NPT>
__global__ __launch_bounds__(BLOCK) void pcg32r_kernel(PdeDev P, const double* __restrict__ Y, int64_t ns,
                                                       double rtol, int maxit, double inner_rtol,
                                                       int max_refine, void* __restrict__ out,
                                                       int out_fp32, int64_t ld, int64_t col0,
                                                       int* __restrict__ iters) {
  extern __shared__ double lds[];
  const int n = P.n, m = n - 1, G = m * m, P1 = n + 1;
  double* sx = lds;                                   // (n+1)^2 float64: x for the residual
  float* sp = reinterpret_cast<float*>(lds + P1 * P1);  // (n+1)^2 float32: p of the inner loop
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  __shared__ float fred0[2 * (BLOCK / kWave)];
  __shared__ float fred1[2 * (BLOCK / kWave)];
  const int64_t s = xcd_remap(blockIdx.x, gridDim.x);
  load_coef(P, Y, s, coef);
  for (int e = threadIdx.x; e < P1 * P1; e += BLOCK) {
    sx[e] = 0.0;
    sp[e] = 0.0f;
  }
  __syncthreads();

  double x[NPT];
  float r[NPT], p[NPT], dx[NPT], wE[NPT], wW[NPT], wN[NPT], wS[NPT], di[NPT];
  int li[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int g = threadIdx.x + k * BLOCK;
    x[k] = 0.0;
    if (g < G) {
      const int i = g % m + 1, j = g / m + 1;
      double e, w, nn, so;
      node_weights(P, coef, i, j, e, w, nn, so);
      wE[k] = (float)e;
      wW[k] = (float)w;
      wN[k] = (float)nn;
      wS[k] = (float)so;
      di[k] = (float)(1.0 / (e + w + nn + so));
      li[k] = j * P1 + i;
    } else {
      wE[k] = wW[k] = wN[k] = wS[k] = di[k] = 0.0f;
      li[k] = P1 + 1;  // any interior slot: keeps the unused neighbour reads in bounds
    }
  }
  double bb = 0.0;
#pragma unroll
  for (int k = 0; k < NPT; ++k)
    if (threadIdx.x + k * BLOCK < G) bb += P.h2 * P.h2;
  bb = block_sum<BLOCK>(bb, red0);
  const double stop = rtol * rtol * bb;
  int total = 0;
  bool conv = false;
  for (int ref = 0; ref <= max_refine; ++ref) {
    // float64 residual r = b - A x
    double r64[NPT];
    double rr64 = 0.0;
    if (ref == 0) {
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        r64[k] = (threadIdx.x + k * BLOCK < G) ? P.h2 : 0.0;
        rr64 += r64[k] * r64[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (threadIdx.x + k * BLOCK < G) sx[li[k]] = x[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int g = threadIdx.x + k * BLOCK;
        r64[k] = 0.0;
        if (g < G) {
          const int i = g % m + 1, j = g / m + 1, l = li[k];
          double e, w, nn, so;
          node_weights(P, coef, i, j, e, w, nn, so);
          const double ax = (e + w + nn + so) * x[k] -
                            (e * sx[l + 1] + w * sx[l - 1] + nn * sx[l + P1] + so * sx[l - P1]);
          r64[k] = P.h2 - ax;
        }
        rr64 += r64[k] * r64[k];
      }
    }
    rr64 = block_sum<BLOCK>(rr64, red1);
    if (rr64 <= stop) {
      conv = true;
      break;
    }
    if (ref == max_refine) break;
    // inner float32 PCG on the scaled residual
    const double rn = sqrt(rr64);
    const float inv = (float)(1.0 / rn);
    float rz = 0.0f, rr0 = 0.0f;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      r[k] = (float)r64[k] * inv;
      dx[k] = 0.0f;
      p[k] = di[k] * r[k];
      rz += r[k] * p[k];
      rr0 += r[k] * r[k];
    }
    block_sum2<BLOCK>(rz, rr0, fred1);
    const float istop = (float)(inner_rtol * inner_rtol) * rr0;
    int it = 0;
    while (it < maxit) {
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (threadIdx.x + k * BLOCK < G) sp[li[k]] = p[k];
      __syncthreads();
      float q[NPT];
      float pq = 0.0f;
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int l = li[k];
        q[k] = (wE[k] + wW[k] + wN[k] + wS[k]) * p[k] -
               (wE[k] * sp[l + 1] + wW[k] * sp[l - 1] + wN[k] * sp[l + P1] + wS[k] * sp[l - P1]);
        if (threadIdx.x + k * BLOCK >= G) q[k] = 0.0f;
        pq += p[k] * q[k];
      }
      pq = block_sum<BLOCK>(pq, fred0);
      const float alpha = rz / pq;
      float rz2 = 0.0f, rr = 0.0f;
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        dx[k] += alpha * p[k];
        r[k] -= alpha * q[k];
        rz2 += r[k] * (di[k] * r[k]);
        rr += r[k] * r[k];
      }
      block_sum2<BLOCK>(rz2, rr, fred1);
      ++it;
      if (rr <= istop) break;
      const float beta = rz2 / rz;
      rz = rz2;
#pragma unroll
      for (int k = 0; k < NPT; ++k) p[k] = di[k] * r[k] + beta * p[k];
    }
    total += it;
#pragma unroll
    for (int k = 0; k < NPT; ++k) x[k] += rn * (double)dx[k];
    __syncthreads();  // sx may be rewritten only after every thread left the last residual
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int g = threadIdx.x + k * BLOCK;
    if (g < G) store_sample(out, out_fp32, (int64_t)g * ld + col0 + s, x[k]);
  }
  if (threadIdx.x == 0 && iters) iters[s] = conv ? total : -1;
}

// ---------------------------------------------------------------- trig poly
// u_g(y) = Re sum_a c[a,g] exp(2 pi i k_a . y); phases of one sample staged in LDS.
constexpr int kPolyChunk = 1024;
__global__ __launch_bounds__(256) void trigpoly_kernel(int d, const double* __restrict__ Y, int64_t ns,
                                                       const int32_t* __restrict__ K, int64_t np,
                                                       const double* __restrict__ C, int64_t G,
                                                       void* __restrict__ out, int out_fp32, int64_t ld,
                                                       int64_t col0) {
  __shared__ double cs[kPolyChunk];
  __shared__ double sn[kPolyChunk];
  const int64_t s = xcd_remap(blockIdx.x, gridDim.x);
  const double* y = Y + s * d;
  for (int64_t g0 = 0; g0 < G; g0 += 256) {
    const int64_t g = g0 + threadIdx.x;
    double acc = 0.0;
    for (int64_t a0 = 0; a0 < np; a0 += kPolyChunk) {
      const int na = (int)min<int64_t>(kPolyChunk, np - a0);
      __syncthreads();
      for (int a = threadIdx.x; a < na; a += 256) {
        double ph = 0.0;
        for (int j = 0; j < d; ++j) ph += (double)K[(a0 + a) * d + j] * y[j];
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
    if (g < G) store_sample(out, out_fp32, g * ld + col0 + s, acc);
  }
}

// ---------------------------------------------------------------- launchers
void launch_nodes(int d, int line, int t, int nlat, const int64_t* off, const int32_t* Ms,
                  const int32_t* zs, const double* tail, double* Y, int64_t ns, hipStream_t st) {
  if (ns <= 0) return;
  const int64_t tot = ns * d;
  hipLaunchKernelGGL(nodes_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, st, d, line, t, nlat,
                     off, Ms, zs, tail, Y, ns);
  USFFT_HIP(hipGetLastError());
}

using Pcg64Fn = void (*)(PdeDev, const double*, int64_t, double, int, void*, int, int64_t, int64_t, int*);
using Pcg32Fn = void (*)(PdeDev, const double*, int64_t, double, int, double, int, void*, int, int64_t,
                         int64_t, int*);

struct SolverCfg {
  int block, npt;
  Pcg64Fn f64;
  Pcg32Fn f32;
};

#define USFFT_CFG(B, N) SolverCfg{B, N, pcg64_kernel<B, N>, pcg32r_kernel<B, N>}
static const SolverCfg kSolverCfgs[] = {
    USFFT_CFG(64, 1),   USFFT_CFG(64, 2),   USFFT_CFG(128, 1),  USFFT_CFG(128, 2),
    USFFT_CFG(128, 4),  USFFT_CFG(256, 1),  USFFT_CFG(256, 2),  USFFT_CFG(256, 4),
    USFFT_CFG(256, 8),  USFFT_CFG(256, 16), USFFT_CFG(512, 2),  USFFT_CFG(512, 4),
    USFFT_CFG(512, 8),  USFFT_CFG(1024, 4), USFFT_CFG(1024, 2),
};
#undef USFFT_CFG

int solver_config_count() { return (int)(sizeof(kSolverCfgs) / sizeof(kSolverCfgs[0])); }

bool solver_config_fits(int c, int G) {
  const SolverCfg& k = kSolverCfgs[c];
  const int cap = k.block * k.npt;
  return cap >= G && cap < 2 * G + 2 * k.block && cap <= 4 * G + k.block;
}

void solver_config_shape(int c, int* block, int* npt) {
  *block = kSolverCfgs[c].block;
  *npt = kSolverCfgs[c].npt;
}

int solver_default_config(int G) {
  // smallest block whose capacity covers G with at most 8 nodes per thread
  int best = -1;
  for (int c = 0; c < solver_config_count(); ++c) {
    const SolverCfg& k = kSolverCfgs[c];
    if (k.block * k.npt < G || k.npt > 8) continue;
    if (best < 0 || k.block * k.npt < kSolverCfgs[best].block * kSolverCfgs[best].npt ||
        (k.block * k.npt == kSolverCfgs[best].block * kSolverCfgs[best].npt && k.npt > kSolverCfgs[best].npt))
      best = c;
  }
  return best;
}

void launch_pde_solve(int cfg, const PdeDev& P, int precision, const double* Y, int64_t ns, double rtol,
                      int maxit, double inner_rtol, int max_refine, void* out, int out_fp32, int64_t ld,
                      int64_t col0, int* iters, hipStream_t st) {
  if (ns <= 0) return;
  const SolverCfg& k = kSolverCfgs[cfg];
  const size_t P1 = (size_t)(P.n + 1) * (P.n + 1);
  if (precision == USFFT_FP64) {
    hipLaunchKernelGGL(k.f64, dim3((unsigned)ns), dim3(k.block), P1 * sizeof(double), st, P, Y, ns, rtol,
                       maxit, out, out_fp32, ld, col0, iters);
  } else {
    hipLaunchKernelGGL(k.f32, dim3((unsigned)ns), dim3(k.block), P1 * (sizeof(double) + sizeof(float)), st,
                       P, Y, ns, rtol, maxit, inner_rtol, max_refine, out, out_fp32, ld, col0, iters);
  }
  USFFT_HIP(hipGetLastError());
}

void launch_trigpoly(int d, const double* Y, int64_t ns, const int32_t* K, int64_t np, const double* C,
                     int64_t G, void* out, int out_fp32, int64_t ld, int64_t col0, hipStream_t st) {
  if (ns <= 0) return;
  hipLaunchKernelGGL(trigpoly_kernel, dim3((unsigned)ns), dim3(256), 0, st, d, Y, ns, K, np, C, G, out,
                     out_fp32, ld, col0);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
