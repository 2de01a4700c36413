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
// One persistent workgroup of 256 threads per sample: triangle coefficients,
// matrix values and the search direction live in LDS; thread t owns rows
// t, t + 256, ... (up to RMAX of them) with their iterate, residual and
// direction in registers.  Float64 conjugate gradients with the Jacobi
// preconditioner, stopped on the scaled residual
//     r . D^-1 r <= rtol^2 b . D^-1 b   (D = diag(A)),
// which CG forms anyway.  The sample of inner vertex g is written to
// out[g * ld + col0 + s], the layout of the uniform-mesh solvers.
#include "kernels.h"
#include "pde_device.h"

namespace usfft {

constexpr int kMeshBlock = 256;

int64_t mesh_lds_bytes(const MeshDev& M) { return 8 * ((int64_t)M.nt + M.nnz + M.G); }

template <int RMAX>
__global__ __launch_bounds__(kMeshBlock) void pcgmesh_kernel(PdeDev P, MeshDev M, const double* __restrict__ Y,
                                                             int64_t ns, double rtol, int maxit,
                                                             void* __restrict__ out, int out_fp32, int64_t ld,
                                                             int64_t col0, int* __restrict__ iters) {
  extern __shared__ double lds[];
  __shared__ double coef[kMaxD];
  __shared__ double red0[kMeshBlock / kWave];
  __shared__ double red1[kMeshBlock / kWave];
  double* aT = lds;            // triangle coefficients
  double* val = aT + M.nt;     // matrix values, CSR order
  double* sp = val + M.nnz;    // search direction
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
    double x[RMAX], r[RMAX], p[RMAX], dinv[RMAX];
    double rz = 0.0;
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const int i = tid + kMeshBlock * q;
      x[q] = r[q] = p[q] = dinv[q] = 0.0;
      if (i < M.G) {
        dinv[q] = 1.0 / val[M.diag[i]];
        r[q] = M.load[i];
        p[q] = dinv[q] * r[q];
        rz += r[q] * p[q];
      }
    }
    rz = block_sum<kMeshBlock>(rz, red0);
    const double stop = rtol * rtol * rz;
    int it = 0;
    bool conv = !(rz > 0.0);
    while (!conv && it < maxit) {
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        const int i = tid + kMeshBlock * q;
        if (i < M.G) sp[i] = p[q];
      }
      __syncthreads();
      double qv[RMAX];
      double pq = 0.0;
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        const int i = tid + kMeshBlock * q;
        double acc = 0.0;
        if (i < M.G)
          for (int e = M.rowptr[i]; e < M.rowptr[i + 1]; ++e) acc += val[e] * sp[M.col[e]];
        qv[q] = acc;
        pq += p[q] * acc;
      }
      pq = block_sum<kMeshBlock>(pq, red0);
      const double alpha = rz / pq;
      double rz2 = 0.0;
#pragma unroll
      for (int q = 0; q < RMAX; ++q) {
        x[q] += alpha * p[q];
        r[q] -= alpha * qv[q];
        rz2 += r[q] * dinv[q] * r[q];
      }
      rz2 = block_sum<kMeshBlock>(rz2, red1);
      ++it;
      if (rz2 <= stop) {
        conv = true;
        break;
      }
      const double beta = rz2 / rz;
      rz = rz2;
#pragma unroll
      for (int q = 0; q < RMAX; ++q) p[q] = dinv[q] * r[q] + beta * p[q];
    }
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const int i = tid + kMeshBlock * q;
      if (i < M.G) store_sample(out, out_fp32, (int64_t)i * ld + col0 + s, x[q]);
    }
    if (tid == 0 && iters) iters[s] = conv ? it : -1;
  }
}

static int mesh_rmax(int G) { return G <= 4 * kMeshBlock ? 4 : 8; }

int mesh_persistent_blocks(const MeshDev& M) {
  int cus = 0, dev = 0, per_cu = 0;
  USFFT_HIP(hipGetDevice(&dev));
  USFFT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const void* k = mesh_rmax(M.G) == 4 ? reinterpret_cast<const void*>(pcgmesh_kernel<4>)
                                      : reinterpret_cast<const void*>(pcgmesh_kernel<8>);
  USFFT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kMeshBlock, (size_t)mesh_lds_bytes(M)));
  return std::max(1, per_cu) * std::max(1, cus);
}

void launch_pde_solve_mesh(const PdeDev& P, const MeshDev& M, const double* Y, int64_t ns, double rtol, int maxit,
                           void* out, int out_fp32, int64_t ld, int64_t col0, int* iters, int blocks,
                           hipStream_t st) {
  if (ns <= 0) return;
  USFFT_REQUIRE(M.G >= 1 && M.G <= kMaxMeshRows, USFFT_EINVAL, "mesh has too many inner vertices");
  const unsigned grid = (unsigned)std::min<int64_t>(ns, blocks);
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
