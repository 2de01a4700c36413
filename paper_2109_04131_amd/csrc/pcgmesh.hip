// Batched PDE solves on a general triangulation.
//
// The sampler of the usFFT (Sec. 2.1) on an unstructured P1 mesh, the
// discretisation the paper itself uses (Sec. 4: an unstructured mesh of the
// unit square).  The nodes T_G are the inner vertices; for one parameter the
// stiffness matrix on the fixed CSR pattern of inner-vertex couplings is
//     A_ij = sum over the triangles T containing edge ij (or vertex i, for
//            the diagonal) of a_T * |T| grad(phi_i) . grad(phi_j),
// with a_T the coefficient at the centroid, and the load is b_i = sum |T|/3
// (f = 1).  The plan stores, per CSR entry, the list of (triangle, geometric
// weight) pairs that add up to it, so a sample's matrix is a gather over
// triangle coefficients with no atomics, in a fixed order.
//
// One persistent workgroup of 256 threads per sample (meshes up to 2048
// inner vertices; larger ones use pcgmesh_global_kernel below): the matrix
// values and
// one vector live in LDS (the vector overlays the triangle coefficients,
// which are dead once the matrix is assembled); thread t owns rows t,
// t + 256, ... (up to RMAX of them) with their iterate, residual and
// directions in registers.  Float64 conjugate gradients with the Jacobi
// preconditioner in the Chronopoulos-Gear arrangement: per iteration one
// product w = A u of the preconditioned residual u = D^-1 r and one fused
// block reduction of (r.u, w.u); the direction's product s = A p follows
// by recursion, s = w + beta s.  Two barriers per iteration.  Stopped on
// the scaled residual  r . D^-1 r <= rtol^2 b . D^-1 b  (D = diag(A)).  The
// sample of inner vertex g is written to out[g * ld + col0 + s], the layout
// of the uniform-mesh solvers.
#include "kernels.h"
#include "pde_device.h"

namespace usfft {

constexpr int kMeshBlock = 256;

int64_t mesh_lds_bytes(const MeshDev& M) { return 8 * ((int64_t)std::max(M.nt, M.G) + M.nnz); }

template <int RMAX>
__global__ __launch_bounds__(kMeshBlock) void pcgmesh_kernel(PdeDev P, MeshDev M, const double* __restrict__ Y,
                                                             int64_t ns, double rtol, int maxit,
                                                             void* __restrict__ out, int out_fp32, int64_t ld,
                                                             int64_t col0, int* __restrict__ iters) {
  extern __shared__ double lds[];
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (kMeshBlock / kWave)];
  double* val = lds;           // matrix values, CSR order
  double* aT = val + M.nnz;    // triangle coefficients (assembly)
  double* su = aT;             // preconditioned residual (iterations)
  const int tid = threadIdx.x;
  const bool logn = P.model == USFFT_MODEL_LOGNORMAL;
  for (int64_t s = xcd_remap(blockIdx.x, gridDim.x); s < ns; s += gridDim.x) {
    __syncthreads();  // the previous sample is done with LDS and coef
    load_coef(P, Y, s, coef);
    __syncthreads();
    for (int t = tid; t < M.nt; t += kMeshBlock) {
      double z = 0.0;
      for (int k = 0; k < P.d; ++k) z += coef[k] * M.psi[(int64_t)k * M.nt + t];
      aT[t] = logn ? P.a0 + exp(z) : P.a0 + z;
    }
    __syncthreads();
    for (int e = tid; e < M.nnz; e += kMeshBlock) {
      double v = 0.0;
      for (int c = M.cptr[e]; c < M.cptr[e + 1]; ++c) v += aT[M.ctri[c]] * M.cw[c];
      val[e] = v;
    }
    __syncthreads();
    double x[RMAX], r[RMAX], p[RMAX], sq[RMAX], dinv[RMAX];
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const int i = tid + kMeshBlock * q;
      x[q] = r[q] = p[q] = sq[q] = dinv[q] = 0.0;
      if (i < M.G) {
        dinv[q] = 1.0 / val[M.diag[i]];
        r[q] = M.load[i];
      }
    }
    double stop = 0.0, gamma_old = 1.0, alpha_old = 1.0;
    int it = 0;
    bool conv = false;
    while (true) {
      // u = D^-1 r to LDS; w = A u; one reduction of (r.u, w.u)
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        const int i = tid + kMeshBlock * q;
        if (i < M.G) su[i] = dinv[q] * r[q];
      }
      __syncthreads();
      double w[RMAX];
      double gamma = 0.0, delta = 0.0;
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        const int i = tid + kMeshBlock * q;
        double acc = 0.0;
        if (i < M.G)
          for (int e = M.rowptr[i]; e < M.rowptr[i + 1]; ++e) acc += val[e] * su[M.col[e]];
        w[q] = acc;
        const double u = dinv[q] * r[q];
        gamma += r[q] * u;
        delta += acc * u;
      }
      block_sum2<kMeshBlock>(gamma, delta, red0);
      if (it == 0) stop = rtol * rtol * gamma;
      if (!(gamma > stop)) {
        conv = true;
        break;
      }
      if (it >= maxit) break;
      const double beta = it == 0 ? 0.0 : gamma / gamma_old;
      const double alpha = gamma / (delta - (it == 0 ? 0.0 : beta * gamma / alpha_old));
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        p[q] = dinv[q] * r[q] + beta * p[q];
        sq[q] = w[q] + beta * sq[q];
        x[q] += alpha * p[q];
        r[q] -= alpha * sq[q];
      }
      gamma_old = gamma;
      alpha_old = alpha;
      ++it;
      // the next iteration's u overwrites su: every lane is past its reads
      // (block_sum2 above)
    }
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const int i = tid + kMeshBlock * q;
      if (i < M.G) store_sample(out, out_fp32, (int64_t)i * ld + col0 + s, x[q]);
    }
    if (tid == 0 && iters) iters[s] = conv ? it : -1;
  }
}

// The same iteration for meshes whose values and vectors do not fit LDS
// (more than 2048 inner vertices, or 8 (nt + nnz + G) bytes above the LDS
// budget): every workgroup keeps its sample's state in its own slot of a
// global scratch, [values nnz | triangle coefficients nt | x r p s u w
// D^-1, G each], doubles, and owns rows tid, tid + 256, ... of every vector.
// Only u is read across rows (by the product); the barrier after its write
// orders it for the workgroup, whose threads share one CU and its L1.
int64_t mesh_scratch_doubles(const MeshDev& M) { return ((int64_t)M.nnz + M.nt + 7 * (int64_t)M.G + 31) / 32 * 32; }

__global__ __launch_bounds__(kMeshBlock) void pcgmesh_global_kernel(PdeDev P, MeshDev M, const double* __restrict__ Y,
                                                                    int64_t ns, double rtol, int maxit,
                                                                    void* __restrict__ out, int out_fp32, int64_t ld,
                                                                    int64_t col0, int* __restrict__ iters,
                                                                    double* __restrict__ scr, int64_t stride) {
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (kMeshBlock / kWave)];
  const int G = M.G, tid = threadIdx.x;
  double* val = scr + (int64_t)blockIdx.x * stride;
  double* aT = val + M.nnz;
  double* x = aT + M.nt;
  double* r = x + G;
  double* p = r + G;
  double* sq = p + G;
  double* su = sq + G;
  double* w = su + G;
  double* dinv = w + G;
  const bool logn = P.model == USFFT_MODEL_LOGNORMAL;
  for (int64_t s = xcd_remap(blockIdx.x, gridDim.x); s < ns; s += gridDim.x) {
    __syncthreads();  // the previous sample is done with the slot and coef
    load_coef(P, Y, s, coef);
    __syncthreads();
    for (int t = tid; t < M.nt; t += kMeshBlock) {
      double z = 0.0;
      for (int k = 0; k < P.d; ++k) z += coef[k] * M.psi[(int64_t)k * M.nt + t];
      aT[t] = logn ? P.a0 + exp(z) : P.a0 + z;
    }
    __syncthreads();
    for (int e = tid; e < M.nnz; e += kMeshBlock) {
      double v = 0.0;
      for (int c = M.cptr[e]; c < M.cptr[e + 1]; ++c) v += aT[M.ctri[c]] * M.cw[c];
      val[e] = v;
    }
    __syncthreads();
    for (int i = tid; i < G; i += kMeshBlock) {
      dinv[i] = 1.0 / val[M.diag[i]];
      x[i] = p[i] = sq[i] = 0.0;
      r[i] = M.load[i];
    }
    double stop = 0.0, gamma_old = 1.0, alpha_old = 1.0;
    int it = 0;
    bool conv = false;
    while (true) {
      for (int i = tid; i < G; i += kMeshBlock) su[i] = dinv[i] * r[i];
      __syncthreads();
      double gamma = 0.0, delta = 0.0;
      for (int i = tid; i < G; i += kMeshBlock) {
        double acc = 0.0;
        for (int e = M.rowptr[i]; e < M.rowptr[i + 1]; ++e) acc += val[e] * su[M.col[e]];
        w[i] = acc;
        const double u = su[i];
        gamma += r[i] * u;
        delta += acc * u;
      }
      block_sum2<kMeshBlock>(gamma, delta, red0);
      if (it == 0) stop = rtol * rtol * gamma;
      if (!(gamma > stop)) {
        conv = true;
        break;
      }
      if (it >= maxit) break;
      const double beta = it == 0 ? 0.0 : gamma / gamma_old;
      const double alpha = gamma / (delta - (it == 0 ? 0.0 : beta * gamma / alpha_old));
      for (int i = tid; i < G; i += kMeshBlock) {
        const double pi = su[i] + beta * p[i];
        const double si = w[i] + beta * sq[i];
        p[i] = pi;
        sq[i] = si;
        x[i] += alpha * pi;
        r[i] -= alpha * si;
      }
      gamma_old = gamma;
      alpha_old = alpha;
      ++it;
      // the next iteration's u overwrites su: every thread is past its
      // reads (block_sum2 above)
    }
    for (int i = tid; i < G; i += kMeshBlock) store_sample(out, out_fp32, (int64_t)i * ld + col0 + s, x[i]);
    if (tid == 0 && iters) iters[s] = conv ? it : -1;
  }
}

bool mesh_fits_lds(const MeshDev& M) { return M.G <= kMaxMeshRows && mesh_lds_bytes(M) <= kMaxMeshLds; }

static int mesh_rmax(int G) { return G <= 4 * kMeshBlock ? 4 : 8; }

int mesh_persistent_blocks(const MeshDev& M) {
  int cus = 0, dev = 0, per_cu = 0;
  USFFT_HIP(hipGetDevice(&dev));
  USFFT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // the global-scratch solver streams its state through L2 and HBM: two
  // workgroups per CU keep the memory system busy with a bounded scratch
  if (!mesh_fits_lds(M)) return 2 * std::max(1, cus);
  const void* k = mesh_rmax(M.G) == 4 ? reinterpret_cast<const void*>(pcgmesh_kernel<4>)
                                      : reinterpret_cast<const void*>(pcgmesh_kernel<8>);
  USFFT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kMeshBlock, (size_t)mesh_lds_bytes(M)));
  return std::max(1, per_cu) * std::max(1, cus);
}

void launch_pde_solve_mesh(const PdeDev& P, const MeshDev& M, const double* Y, int64_t ns, double rtol, int maxit,
                           void* out, int out_fp32, int64_t ld, int64_t col0, int* iters, int blocks, double* scr,
                           hipStream_t st) {
  if (ns <= 0) return;
  USFFT_REQUIRE(M.G >= 1, USFFT_EINVAL, "mesh has no inner vertex");
  const unsigned grid = (unsigned)std::min<int64_t>(ns, blocks);
  if (!mesh_fits_lds(M)) {
    USFFT_REQUIRE(scr != nullptr, USFFT_EINVAL, "the global-scratch mesh solver needs its scratch");
    hipLaunchKernelGGL(pcgmesh_global_kernel, dim3(grid), dim3(kMeshBlock), 0, st, P, M, Y, ns, rtol, maxit, out,
                       out_fp32, ld, col0, iters, scr, mesh_scratch_doubles(M));
    USFFT_HIP(hipGetLastError());
    return;
  }
  const size_t lds = (size_t)mesh_lds_bytes(M);
  if (mesh_rmax(M.G) == 4)
    hipLaunchKernelGGL(pcgmesh_kernel<4>, dim3(grid), dim3(kMeshBlock), lds, st, P, M, Y, ns, rtol, maxit, out,
                       out_fp32, ld, col0, iters);
  else
    hipLaunchKernelGGL(pcgmesh_kernel<8>, dim3(grid), dim3(kMeshBlock), lds, st, P, M, Y, ns, rtol, maxit, out,
                       out_fp32, ld, col0, iters);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
