// Device-side P1 assembly of the parametric diffusion problem (eq. (1.1),
// (1.2)) on the uniform mesh, shared by the PCG solvers.
#pragma once
#include "kernels.h"

namespace usfft {

// Centroid value of a on the lower (q=0) / upper (q=1) triangle of cell (ci, cj).
// tab holds sin(m1 pi x1), sin(m2 pi x2) at the centroid abscissae:
// [0] x1 of lower, [1] x1 of upper, [2] x2 of lower, [3] x2 of upper; each d x n;
// then [2] and [3] again, each d x row_tab_pitch(n) with padded rows.
// The lognormal model exponentiates the sum (Sec. 1).
__device__ __forceinline__ double tri_coef(const PdeDev& P, const double* coef, int q, int ci, int cj) {
  const double* tx = P.tab + (size_t)(q) * P.d * P.n;
  const double* ty = P.tab + (size_t)(2 + q) * P.d * P.n;
  const bool logn = P.model == USFFT_MODEL_LOGNORMAL;
  double a = logn ? 0.0 : P.a0;
#pragma unroll 1
  for (int k = 0; k < P.d; ++k) a += coef[k] * tx[k * P.n + ci] * ty[k * P.n + cj];
  return logn ? P.a0 + exp(a) : a;
}

// Weight of horizontal edge (i,j)-(i+1,j), 0 <= i <= n-1: lower triangle of
// cell (i,j) and upper triangle of cell (i,j-1).
__device__ __forceinline__ double edge_h(const PdeDev& P, const double* coef, int i, int j) {
  return 0.5 * (tri_coef(P, coef, 0, i, j) + tri_coef(P, coef, 1, i, j - 1));
}
// Weight of vertical edge (i,j)-(i,j+1), 0 <= j <= n-1: upper triangle of
// cell (i,j) and lower triangle of cell (i-1,j).
__device__ __forceinline__ double edge_v(const PdeDev& P, const double* coef, int i, int j) {
  return 0.5 * (tri_coef(P, coef, 1, i, j) + tri_coef(P, coef, 0, i - 1, j));
}

// Fill the edge grids of one sample: eh[j*P1 + i] = edge_h(i, j) for
// 0 <= i <= n-1, 1 <= j <= n-1 and ev[j*P1 + i] = edge_v(i, j) for
// 1 <= i <= n-1, 0 <= j <= n-1 (every edge touching an interior node); the
// row pitch P1 is n + 1 unless given.
template <typename T>
__device__ void fill_edges(const PdeDev& P, const double* coef, T* eh, T* ev, int pitch = 0) {
  const int n = P.n, P1 = pitch > 0 ? pitch : n + 1, cnt = n * (n - 1);
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int i = e % n, j = e / n + 1;  // horizontal: i in [0, n-1], j in [1, n-1]
    eh[j * P1 + i] = (T)edge_h(P, coef, i, j);
    const int vi = e / n + 1, vj = e % n;  // vertical: i in [1, n-1], j in [0, n-1]
    ev[vj * P1 + vi] = (T)edge_v(P, coef, vi, vj);
  }
}

// Per-dimension factor of the coefficient at the sampling node t = Y[s]:
// amp_k Theta_k(t) with Theta = sin(2 pi t) (periodic), the tent image phi(t)
// (affine, eq. (3.2)) or sqrt(2) erf^-1(2 tau(t)) with tau the tent shifted
// by delta (lognormal, eq. (3.3)).  Not inlined: a few lanes evaluate it once
// per sample, and inlined into a solver its polynomial constants are hoisted
// out of the sample loop and spilled.
// With raw set, t is already the parameter y (the affine and lognormal
// factors are y itself, the periodic one sin(2 pi y)).  Its arguments are
// scalars: a reference to the kernel's problem structure would make the
// callers keep a private copy of it.
__device__ __noinline__ double model_theta(int model, int raw, double alpha, double beta, double delta, double t) {
  if (raw && model != USFFT_MODEL_PERIODIC) return t;
  if (model == USFFT_MODEL_AFFINE) return beta - fabs((beta - alpha) * (1.0 - 2.0 * t));
  if (model == USFFT_MODEL_LOGNORMAL) {
    const double dl = delta;
    const double v = t < dl ? -0.5 - 2.0 * (t - dl) : (t < 0.5 + dl ? -0.5 + 2.0 * (t - dl) : 1.5 - 2.0 * (t - dl));
    return 1.4142135623730951 * erfinv(2.0 * v);
  }
  return sinpi(2.0 * t);
}

__device__ __forceinline__ void load_coef(const PdeDev& P, const double* __restrict__ Y, int64_t s,
                                          double* coef) {
  for (int k = threadIdx.x; k < P.d; k += blockDim.x)
    coef[k] = P.amp[k] * model_theta(P.model, P.raw, P.alpha, P.beta, P.delta, Y[s * P.d + k]);
}

template <typename T>
__device__ __forceinline__ void store_sample(void* out, int out_fp32, int64_t idx, T v) {
  if (out_fp32)
    static_cast<float*>(out)[idx] = (float)v;
  else
    static_cast<double*>(out)[idx] = (double)v;
}

}  // namespace usfft
