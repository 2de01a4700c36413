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
#include "pde_device.h"

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

// ---------------------------------------------------------------- FP64 PCG
// WPE: requested waves per SIMD (0 = compiler's choice); WPE = 2 * BLOCK / 256
// asks for two resident workgroups per CU.
template <int BLOCK, int NPT, int WPE, int NC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1))) void pcg64_kernel(PdeDev P, const double* __restrict__ Y, int64_t ns,
                                                      double rtol, int maxit, void* __restrict__ out,
                                                      int out_fp32, int64_t ld, int64_t col0,
                                                      int* __restrict__ iters) {
  extern __shared__ double sp[];  // (n+1)^2, zero halo = Dirichlet data
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  const int64_t s = xcd_remap(blockIdx.x, gridDim.x);
  const int n = NC > 0 ? NC : P.n, m = n - 1, G = m * m, P1 = n + 1;
  load_coef(P, Y, s, coef);
  for (int e = threadIdx.x; e < P1 * P1; e += BLOCK) sp[e] = 0.0;
  __syncthreads();

  double x[NPT], r[NPT], p[NPT], wE[NPT], wW[NPT], wN[NPT], wS[NPT], di[NPT];
  int li[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int g = threadIdx.x + k * BLOCK;
    li[k] = (g < G) ? (g / m + 1) * P1 + (g % m + 1) : P1 + 1;  // padding slots read in bounds
  }
  // edge weights through LDS, one direction at a time (the p buffer holds one grid)
  {
    const int cnt = n * (n - 1);
    for (int e = threadIdx.x; e < cnt; e += BLOCK) {
      const int i = e % n, j = e / n + 1;
      sp[j * P1 + i] = edge_h(P, coef, i, j);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      wE[k] = sp[li[k]];
      wW[k] = sp[li[k] - 1];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += BLOCK) {
      const int i = e / n + 1, j = e % n;
      sp[j * P1 + i] = edge_v(P, coef, i, j);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      wN[k] = sp[li[k]];
      wS[k] = sp[li[k] - P1];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < P1 * P1; e += BLOCK) sp[e] = 0.0;
    __syncthreads();
  }
  double rz = 0.0, bb = 0.0;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int g = threadIdx.x + k * BLOCK;
    x[k] = 0.0;
    if (g < G) {
      di[k] = 1.0 / (wE[k] + wW[k] + wN[k] + wS[k]);
      r[k] = P.h2;
      p[k] = di[k] * r[k];
      rz += r[k] * p[k];
      bb += r[k] * r[k];
    } else {
      wE[k] = wW[k] = wN[k] = wS[k] = di[k] = 0.0;
      r[k] = p[k] = 0.0;
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

// One float32 Jacobi-PCG run with "reliable updates" (Sleijpen & van der
// Vorst 1996): the float64 iterate x lives in LDS, the float32 correction dx
// accumulated since the last update lives in registers.  The kernel is
// persistent (one workgroup per resident slot, looping over samples), so each
// workgroup keeps its sample's exact float64 edge grids in a private global
// scratch slot that stays in L2; updates read them instead of recomputing.  Whenever the float32
// recursive residual has dropped by inner_rtol since the last reference (or
// every refine_every iterations, a guard against float32 stagnation), x +=
// dx and the true residual b - A(y) x is formed in float64 (weights
// recomputed in float64 from the centroid tables, edge-difference form) and
// replaces the float32 one; the search direction is kept.  The solve stops on
// the float64 true residual.  Dot products are accumulated in float64.  The
// float32 state is small enough for two resident samples per CU, which hide
// each other's barrier and reduction latency.
// Jacobi scaling of the float32 path: hardware reciprocal (1 ulp), a fixed
// deterministic diagonal preconditioner; padding slots (zero diagonal) get 0.
__device__ __forceinline__ float jacobi_rcp(float dg) { return dg > 0.0f ? __builtin_amdgcn_rcpf(dg) : 0.0f; }

template <int BLOCK, int NPT, int WPE, int NC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1))) void pcg32r_kernel(
    PdeDev P, const double* __restrict__ Y, int64_t ns, double rtol, int maxit, double inner_rtol, int refine_every,
    void* __restrict__ out, int out_fp32, int64_t ld, int64_t col0, int* __restrict__ iters,
    double* __restrict__ wscr, int64_t wstride) {
  extern __shared__ double lds[];
  const int n = NC > 0 ? NC : P.n, m = n - 1, G = m * m, P1 = n + 1;
  double* sx = lds;                                     // (n+1)^2 float64 iterate x (zero halo)
  float* sp = reinterpret_cast<float*>(lds + P1 * P1);  // (n+1)^2 float32 search direction
  double* eh = wscr + (size_t)blockIdx.x * 2 * wstride;  // this workgroup's float64 edge grids
  double* ev = eh + wstride;
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  int li[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int g = threadIdx.x + k * BLOCK;
    li[k] = (g < G) ? (g / m + 1) * P1 + (g % m + 1) : P1 + 1;  // padding slots read in bounds
  }
  // persistent: consecutive samples stay on one XCD within each round
  for (int64_t s = xcd_remap(blockIdx.x, gridDim.x); s < ns; s += gridDim.x) {
    __syncthreads();  // the previous sample is done with LDS, coef and the edge grids
    load_coef(P, Y, s, coef);
    for (int e = threadIdx.x; e < P1 * P1; e += BLOCK) {
      sx[e] = 0.0;
      sp[e] = 0.0f;
    }
    __syncthreads();
    fill_edges<double>(P, coef, eh, ev);
    __syncthreads();
    float r[NPT], p[NPT], dx[NPT], wE[NPT], wW[NPT], wN[NPT], wS[NPT];
    double rz = 0.0, rr = 0.0, bb = 0.0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int g = threadIdx.x + k * BLOCK;
      dx[k] = 0.0f;
      if (g < G) {
        wE[k] = (float)eh[li[k]];
        wW[k] = (float)eh[li[k] - 1];
        wN[k] = (float)ev[li[k]];
        wS[k] = (float)ev[li[k] - P1];
        r[k] = (float)P.h2;
        bb += P.h2 * P.h2;
      } else {
        wE[k] = wW[k] = wN[k] = wS[k] = 0.0f;
        r[k] = 0.0f;
      }
      p[k] = r[k] * jacobi_rcp(wE[k] + wW[k] + wN[k] + wS[k]);
      rz += (double)(r[k] * p[k]);
      rr += (double)(r[k] * r[k]);
    }
    block_sum2<BLOCK>(rz, rr, red1);
    bb = block_sum<BLOCK>(bb, red0);
    const double stop = rtol * rtol * bb;
    const double drop = inner_rtol * inner_rtol;
    double rr_ref = rr;  // float32 residual norm^2 right after the last true residual
    int it = 0, last_update = 0;
    bool conv = false;
    while (it < maxit) {
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (threadIdx.x + k * BLOCK < G) sp[li[k]] = p[k];
      __syncthreads();
      float q[NPT];
      double pq = 0.0;
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int l = li[k];
        q[k] = wE[k] * (p[k] - sp[l + 1]) + wW[k] * (p[k] - sp[l - 1]) + wN[k] * (p[k] - sp[l + P1]) +
               wS[k] * (p[k] - sp[l - P1]);
        if (threadIdx.x + k * BLOCK >= G) q[k] = 0.0f;
        pq += (double)(p[k] * q[k]);
      }
      pq = block_sum<BLOCK>(pq, red0);
      const float alpha = (float)(rz / pq);
      double rz2 = 0.0;
      rr = 0.0;
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        dx[k] += alpha * p[k];
        r[k] -= alpha * q[k];
        rz2 += (double)(r[k] * (r[k] * jacobi_rcp(wE[k] + wW[k] + wN[k] + wS[k])));
        rr += (double)(r[k] * r[k]);
      }
      block_sum2<BLOCK>(rz2, rr, red1);
      ++it;
      if (rr <= drop * rr_ref || it - last_update >= refine_every) {
        // x += dx in float64; the float64 true residual (exact float64 edge
        // grids, edge-difference form) replaces the float32 one
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
          if (threadIdx.x + k * BLOCK < G) sx[li[k]] += (double)dx[k];
          dx[k] = 0.0f;
        }
        __syncthreads();
        // plain pass over the nodes (keeps the per-node register arrays out of
        // it); the float32 residual is staged in sp
        double rr64 = 0.0, rz3 = 0.0, rr3 = 0.0;
        for (int g = threadIdx.x; g < G; g += BLOCK) {
          const int l = (g / m + 1) * P1 + (g % m + 1);
          const double xc = sx[l];
          const double ax = eh[l] * (xc - sx[l + 1]) + eh[l - 1] * (xc - sx[l - 1]) + ev[l] * (xc - sx[l + P1]) +
                            ev[l - P1] * (xc - sx[l - P1]);
          const double r64 = P.h2 - ax;
          rr64 += r64 * r64;
          sp[l] = (float)r64;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
          if (threadIdx.x + k * BLOCK < G) {
            r[k] = sp[li[k]];
            rz3 += (double)(r[k] * (r[k] * jacobi_rcp(wE[k] + wW[k] + wN[k] + wS[k])));
            rr3 += (double)(r[k] * r[k]);
          }
        }
        rr64 = block_sum<BLOCK>(rr64, red0);
        block_sum2<BLOCK>(rz3, rr3, red1);
        last_update = it;
        if (rr64 <= stop) {
          conv = true;
          break;
        }
        rz2 = rz3;
        rr_ref = rr3;
      }
      const float beta = (float)(rz2 / rz);
      rz = rz2;
#pragma unroll
      for (int k = 0; k < NPT; ++k) p[k] = r[k] * jacobi_rcp(wE[k] + wW[k] + wN[k] + wS[k]) + beta * p[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int g = threadIdx.x + k * BLOCK;
      if (g < G) store_sample(out, out_fp32, (int64_t)g * ld + col0 + s, sx[li[k]]);
    }
    if (threadIdx.x == 0 && iters) iters[s] = conv ? it : -1;
  }
}

// ------------------------------------------ streaming FP64 PCG (large meshes)
// For meshes whose per-sample state exceeds one CU (h < 1/64): persistent
// workgroups, each owning a workspace in global memory (iterate, residual,
// search direction with zero halo, A p, edge grids, Jacobi scaling), loop over
// samples s = blockIdx.x + k gridDim.x.  Same Jacobi-PCG and fixed-order
// reductions as the on-chip kernels; bound by L2 / Infinity Cache / HBM
// traffic, not by ALU.
constexpr int kStreamBlock = 1024;
constexpr int kStreamArrays = 7;

__global__ __launch_bounds__(kStreamBlock) void pcg_stream_kernel(PdeDev P, const double* __restrict__ Y,
                                                                  int64_t ns, double rtol, int maxit,
                                                                  void* __restrict__ out, int out_fp32,
                                                                  int64_t ld, int64_t col0,
                                                                  int* __restrict__ iters,
                                                                  double* __restrict__ ws, int64_t gp) {
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (kStreamBlock / kWave)];
  __shared__ double red1[2 * (kStreamBlock / kWave)];
  const int n = P.n, m = n - 1, G = m * m, P1 = n + 1;
  double* x = ws + (size_t)blockIdx.x * kStreamArrays * gp;
  double* r = x + gp;
  double* p = r + gp;   // (n+1)^2 grid, zero halo
  double* q = p + gp;
  double* eh = q + gp;  // (n+1)^2 horizontal edge grid
  double* ev = eh + gp; // (n+1)^2 vertical edge grid
  double* di = ev + gp;
  for (int64_t s = blockIdx.x; s < ns; s += gridDim.x) {
    __syncthreads();  // previous sample finished with coef and the workspace
    load_coef(P, Y, s, coef);
    for (int e = threadIdx.x; e < P1 * P1; e += kStreamBlock) p[e] = 0.0;
    __syncthreads();
    fill_edges<double>(P, coef, eh, ev);
    __syncthreads();
    double rz = 0.0, bb = 0.0;
    for (int g = threadIdx.x; g < G; g += kStreamBlock) {
      const int l = (g / m + 1) * P1 + (g % m + 1);
      const double dinv = 1.0 / (eh[l] + eh[l - 1] + ev[l] + ev[l - P1]);
      di[g] = dinv;
      x[g] = 0.0;
      r[g] = P.h2;
      p[l] = dinv * P.h2;
      rz += P.h2 * dinv * P.h2;
      bb += P.h2 * P.h2;
    }
    block_sum2<kStreamBlock>(rz, bb, red1);
    const double stop = rtol * rtol * bb;
    int it = 0;
    bool conv = false;
    while (it < maxit) {
      double pq = 0.0;
      for (int g = threadIdx.x; g < G; g += kStreamBlock) {
        const int l = (g / m + 1) * P1 + (g % m + 1);
        const double pc = p[l];
        const double qq = eh[l] * (pc - p[l + 1]) + eh[l - 1] * (pc - p[l - 1]) + ev[l] * (pc - p[l + P1]) +
                          ev[l - P1] * (pc - p[l - P1]);
        q[g] = qq;
        pq += pc * qq;
      }
      pq = block_sum<kStreamBlock>(pq, red0);
      const double alpha = rz / pq;
      double rz2 = 0.0, rr = 0.0;
      for (int g = threadIdx.x; g < G; g += kStreamBlock) {
        const int l = (g / m + 1) * P1 + (g % m + 1);
        x[g] += alpha * p[l];
        const double rg = r[g] - alpha * q[g];
        r[g] = rg;
        rz2 += rg * (di[g] * rg);
        rr += rg * rg;
      }
      block_sum2<kStreamBlock>(rz2, rr, red1);
      ++it;
      if (rr <= stop) {
        conv = true;
        break;
      }
      const double beta = rz2 / rz;
      rz = rz2;
      for (int g = threadIdx.x; g < G; g += kStreamBlock) {
        const int l = (g / m + 1) * P1 + (g % m + 1);
        p[l] = di[g] * r[g] + beta * p[l];
      }
      __syncthreads();
    }
    for (int g = threadIdx.x; g < G; g += kStreamBlock) store_sample(out, out_fp32, (int64_t)g * ld + col0 + s, x[g]);
    if (threadIdx.x == 0 && iters) iters[s] = conv ? it : -1;
  }
}

int64_t stream_workspace_doubles(int n, int blocks) {
  const int64_t gp = ((int64_t)(n + 1) * (n + 1) + 63) / 64 * 64;
  return gp * kStreamArrays * blocks;
}

void launch_pde_solve_stream(const PdeDev& P, const double* Y, int64_t ns, double rtol, int maxit, void* out,
                             int out_fp32, int64_t ld, int64_t col0, int* iters, double* ws, int blocks,
                             hipStream_t st) {
  if (ns <= 0) return;
  const int64_t gp = ((int64_t)(P.n + 1) * (P.n + 1) + 63) / 64 * 64;
  const unsigned grid = (unsigned)std::min<int64_t>(blocks, ns);
  hipLaunchKernelGGL(pcg_stream_kernel, dim3(grid), dim3(kStreamBlock), 0, st, P, Y, ns, rtol, maxit, out,
                     out_fp32, ld, col0, iters, ws, gp);
  USFFT_HIP(hipGetLastError());
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
// All d x r detection lines of step 1 in one launch: line L = t r + i covers
// samples [loff[L], loff[L + 1]) with coordinate t on l / K_t and tail L.
__global__ void line_nodes_kernel(int d, int r, int nlines, const int64_t* __restrict__ loff,
                                  const int32_t* __restrict__ Kt, const double* __restrict__ tails,
                                  double* __restrict__ Y, int64_t ns) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ns * d) return;
  const int64_t s = e / d;
  const int j = (int)(e % d);
  int lo = 0, hi = nlines - 1;  // last line with loff <= s
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (loff[mid] <= s) lo = mid; else hi = mid - 1;
  }
  const int t = lo / r;
  Y[e] = j == t ? (double)(s - loff[lo]) / (double)Kt[t] : tails[(int64_t)lo * d + j];
}

void launch_line_nodes(int d, int r, const int64_t* loff, const int32_t* Kt, const double* tails, double* Y,
                       int64_t ns, hipStream_t st) {
  if (ns <= 0) return;
  hipLaunchKernelGGL(line_nodes_kernel, dim3((unsigned)ceil_div(ns * d, 256)), dim3(256), 0, st, d, r, d * r, loff,
                     Kt, tails, Y, ns);
  USFFT_HIP(hipGetLastError());
}

// nrep copies of a lattice family's nodes, copy b with tail b: the r~
// iterations of one step-2 stage in one launch.
__global__ void lattice_nodes_rep_kernel(int d, int t, int nlat, const int64_t* __restrict__ off,
                                         const int32_t* __restrict__ Ms, const int32_t* __restrict__ zs,
                                         const double* __restrict__ tails, double* __restrict__ Y, int64_t ns,
                                         int nrep) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ns * nrep * d) return;
  const int64_t sg = e / d;
  const int j = (int)(e % d);
  const int b = (int)(sg / ns);
  const int64_t s = sg % ns;
  double y;
  if (j >= t) {
    y = tails[(int64_t)b * d + j];
  } else {
    int l = 0;
    while (l + 1 < nlat && off[l + 1] <= s) ++l;
    const int64_t M = Ms[l];
    const int64_t m = s - off[l];
    y = (double)((m * (int64_t)zs[(int64_t)l * t + j]) % M) / (double)M;
  }
  Y[e] = y;
}

void launch_lattice_nodes_rep(int d, int t, int nlat, const int64_t* off, const int32_t* Ms, const int32_t* zs,
                              const double* tails, double* Y, int64_t ns, int nrep, hipStream_t st) {
  if (ns <= 0 || nrep <= 0) return;
  hipLaunchKernelGGL(lattice_nodes_rep_kernel, dim3((unsigned)ceil_div(ns * nrep * d, 256)), dim3(256), 0, st, d, t,
                     nlat, off, Ms, zs, tails, Y, ns, nrep);
  USFFT_HIP(hipGetLastError());
}

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
                         int64_t, int*, double*, int64_t);

struct SolverCfg {
  int block, npt, wpe, nc;  // nc: mesh size compiled in (0 = any)
  Pcg64Fn f64;
  Pcg32Fn f32;
};

#define USFFT_CFG(B, N, W, NC) SolverCfg{B, N, W, NC, pcg64_kernel<B, N, W, NC>, pcg32r_kernel<B, N, W, NC>}
static const SolverCfg kSolverCfgs[] = {
    // any mesh size
    USFFT_CFG(64, 1, 0, 0), USFFT_CFG(64, 2, 0, 0), USFFT_CFG(128, 1, 0, 0), USFFT_CFG(128, 2, 0, 0),
    USFFT_CFG(128, 4, 0, 0), USFFT_CFG(256, 1, 0, 0), USFFT_CFG(256, 2, 0, 0), USFFT_CFG(256, 4, 0, 0),
    USFFT_CFG(256, 8, 0, 0), USFFT_CFG(256, 16, 0, 0), USFFT_CFG(512, 2, 0, 0), USFFT_CFG(512, 4, 0, 0),
    USFFT_CFG(512, 8, 0, 0), USFFT_CFG(1024, 4, 0, 0), USFFT_CFG(1024, 2, 0, 0),
    // h = 1/64 (G = 3969)
    USFFT_CFG(512, 8, 0, 64), USFFT_CFG(512, 8, 4, 64), USFFT_CFG(256, 16, 0, 64), USFFT_CFG(256, 16, 2, 64),
    USFFT_CFG(1024, 4, 0, 64),
    // h = 1/32 (G = 961)
    USFFT_CFG(256, 4, 0, 32), USFFT_CFG(128, 8, 0, 32), USFFT_CFG(512, 2, 0, 32), USFFT_CFG(128, 8, 2, 32),
    // h = 1/16 (G = 225)
    USFFT_CFG(256, 1, 0, 16), USFFT_CFG(128, 2, 0, 16), USFFT_CFG(64, 4, 0, 16), USFFT_CFG(64, 4, 2, 16),
};
#undef USFFT_CFG

int solver_config_count() { return (int)(sizeof(kSolverCfgs) / sizeof(kSolverCfgs[0])); }

bool solver_config_fits(int c, int n) {
  const SolverCfg& k = kSolverCfgs[c];
  const int G = (n - 1) * (n - 1);
  if (k.nc != 0 && k.nc != n) return false;
  const int cap = k.block * k.npt;
  return cap >= G && cap < 2 * G + 2 * k.block && cap <= 4 * G + k.block;
}

void solver_config_shape(int c, int* block, int* npt) {
  *block = kSolverCfgs[c].block;
  *npt = kSolverCfgs[c].npt * 100 + kSolverCfgs[c].wpe * 10 + (kSolverCfgs[c].nc ? 1 : 0);
}

int solver_default_config(int n) {
  // smallest generic block whose capacity covers G with at most 8 nodes per thread
  const int G = (n - 1) * (n - 1);
  int best = -1;
  for (int c = 0; c < solver_config_count(); ++c) {
    const SolverCfg& k = kSolverCfgs[c];
    if (k.block * k.npt < G || k.npt > 8 || k.wpe != 0 || k.nc != 0) continue;
    if (best < 0 || k.block * k.npt < kSolverCfgs[best].block * kSolverCfgs[best].npt ||
        (k.block * k.npt == kSolverCfgs[best].block * kSolverCfgs[best].npt && k.npt > kSolverCfgs[best].npt))
      best = c;
  }
  return best;
}

// Workgroups of the persistent float32 kernel: CUs x resident workgroups per CU.
int persistent_blocks(int cfg, int n) {
  static int cache[64] = {0};
  if (cfg < 0 || cfg >= 64) return 256;
  if (cache[cfg] > 0) return cache[cfg];
  const SolverCfg& k = kSolverCfgs[cfg];
  const size_t P1 = (size_t)(n + 1) * (n + 1);
  int per_cu = 0, cus = 0, dev = 0;
  USFFT_HIP(hipGetDevice(&dev));
  USFFT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  USFFT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k.f32), k.block,
                                                         P1 * (sizeof(double) + sizeof(float))));
  cache[cfg] = std::max(1, per_cu) * std::max(1, cus);
  return cache[cfg];
}

int64_t edge_scratch_doubles(int n, int blocks) {
  const int64_t ws = ((int64_t)(n + 1) * (n + 1) + 31) / 32 * 32;
  return 2 * ws * blocks;
}

void launch_pde_solve(int cfg, const PdeDev& P, int precision, const double* Y, int64_t ns, double rtol,
                      int maxit, double inner_rtol, int refine_every, void* out, int out_fp32, int64_t ld,
                      int64_t col0, int* iters, double* wscr, int wblocks, hipStream_t st) {
  if (ns <= 0) return;
  const SolverCfg& k = kSolverCfgs[cfg];
  const size_t P1 = (size_t)(P.n + 1) * (P.n + 1);
  if (precision == USFFT_FP64) {
    hipLaunchKernelGGL(k.f64, dim3((unsigned)ns), dim3(k.block), P1 * sizeof(double), st, P, Y, ns, rtol,
                       maxit, out, out_fp32, ld, col0, iters);
  } else {
    const int64_t ws = ((int64_t)(P.n + 1) * (P.n + 1) + 31) / 32 * 32;
    const unsigned grid = (unsigned)std::min<int64_t>(ns, wblocks);
    hipLaunchKernelGGL(k.f32, dim3(grid), dim3(k.block), P1 * (sizeof(double) + sizeof(float)), st, P, Y, ns,
                       rtol, maxit, inner_rtol, refine_every, out, out_fp32, ld, col0, iters, wscr, ws);
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

// ---------------------------------------------------------------- node set
// u(x_g) = sum_a w[3 g + a] u_mesh(v_a) for every point g and sample s: three
// rows of the mesh-vertex samples per point (neighbouring points share
// vertices, so the rows mostly come from L2), one coalesced output row.
template <typename T>
__global__ __launch_bounds__(256) void interp_kernel(const T* __restrict__ um, int64_t ldm,
                                                     const int32_t* __restrict__ idx, const double* __restrict__ w,
                                                     int64_t G, int64_t ns, T* __restrict__ out, int64_t ld,
                                                     int64_t col0) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= ns) return;
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int r = idx[3 * g + a];
      if (r >= 0) v += w[3 * g + a] * (double)um[(int64_t)r * ldm + s];
    }
    out[g * ld + col0 + s] = (T)v;
  }
}

void launch_interp(const void* um, int fp32, int64_t ldm, const int32_t* idx, const double* w, int64_t G, int64_t ns,
                   void* out, int64_t ld, int64_t col0, hipStream_t st) {
  if (G <= 0 || ns <= 0) return;
  const dim3 grid((unsigned)ceil_div(ns, 256), (unsigned)std::min<int64_t>(G, 65535));
  if (fp32)
    hipLaunchKernelGGL(interp_kernel<float>, grid, dim3(256), 0, st, (const float*)um, ldm, idx, w, G, ns,
                       (float*)out, ld, col0);
  else
    hipLaunchKernelGGL(interp_kernel<double>, grid, dim3(256), 0, st, (const double*)um, ldm, idx, w, G, ns,
                       (double*)out, ld, col0);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
