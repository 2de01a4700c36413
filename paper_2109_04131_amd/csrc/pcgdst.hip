// Batched PDE solves with a fast-Poisson preconditioner on the matrix cores.
//
// The sampler of the usFFT (Sec. 2.1, Alg. 1 steps 1&2a, 2c, 3) solves one
// P1 system A(y) u = b per sampling node.  A(y) is the 5-point operator of
// the uniform mesh whose off-diagonal weights are edge weights
// w_e = (a_T1 + a_T2)/2, with the diagonal equal to the sum of the four edge
// weights of a node and b = h^2 for f = 1.  The paper treats the solver as a
// black box; here it is conjugate gradients on the symmetrically scaled system
//     At = D^-1/2 A D^-1/2,  bt = D^-1/2 b,  u = D^-1/2 ut,  D = diag(A) / 4,
// whose diagonal is exactly 4, preconditioned by the inverse of the
// constant-coefficient 5-point Laplacian L (Dirichlet, m = n-1 nodes per
// line).  L is diagonalised by the orthonormal DST-I matrix
//     S[i][k] = sqrt(2/n) sin(pi (i+1)(k+1) / n),  S S = I,
// with eigenvalues lambda_p + lambda_q, lambda_p = 4 sin^2(pi (p+1) / (2n)),
// so  L^-1 R = S (Lam o (S R S)) S,  Lam[p][q] = 1 / (lambda_p + lambda_q),
// for the grid function R as an m x m matrix.  For the smooth coefficients of
// the workloads the scaled operator is close to L, and CG needs about ten
// iterations to 1e-12 instead of a few hundred with Jacobi scaling.
//
// One workgroup owns one sample at a time (persistent over samples).  The
// grid is padded to MP x MP (MP = 32 or 64); wave w owns the 16-column strip
// c = 16 w + (lane & 15) and lane l holds rows 16 t + 4 (l >> 4) + v of it,
// t < MP/16, v < 4: exactly the accumulator layout of the 16x16 MFMA tiles.
// The four 64x64x64 products of one preconditioner application run as
// v_mfma_f32_16x16x32_f16 in this layout:
//     T1 = R^T S   (the residual registers are the A operand of R^T),
//     Wt = S T1    (T1 moved through LDS to column strips),
//     Yt = Lam o Wt,
//     T3 = Y S     (the accumulators are the A operand of Y),
//     Z  = S T3    (T3 moved through LDS), Z in the residual's layout.
// Inputs are scaled by a power of two from the last residual norm before the
// conversion to fp16, so every operand stays in fp16's range; the
// preconditioner only steers the iteration, the residual that decides
// convergence is formed in the solver's own precision.
//
// Float64 solves keep every vector and the weights in float64.  Float32
// solves keep them in float32 with float64 reliable updates (the float64
// iterate u lives in LDS; whenever the float32 recursive residual has dropped
// by inner_rtol, u += D^-1/2 dx and the true residual b - A u is formed in
// float64 from the exact float64 edge grids).  Both stop on the scaled
// residual |D^-1/2 (b - A u)| <= rtol |D^-1/2 b|; float32 solves stop only on
// a float64 true residual.  Reductions combine wave partials in a fixed order.
#include <type_traits>

#include "kernels.h"
#include "pde_device.h"

namespace usfft {

// Sample scheduling of the persistent solver kernels.  The samples [0, ns)
// are split into one contiguous share per XCD (workgroup b serves share
// b % 8, so consecutive samples, whose strided output rows share cache
// lines, stay in one L2), and a workgroup takes the next sample of its share
// from that share's ticket counter (eight counters, zero at launch):
// workgroups that draw quick solves take more of them, so a launch waits for
// its slowest solve rather than its slowest fixed set of solves.
struct Tickets {
  unsigned long long* ctr;
  int sh;
  int64_t lo, hi;
  __device__ Tickets(unsigned long long* c, int64_t ns) : ctr(c) {
    const int nsh = gridDim.x < 8 ? (int)gridDim.x : 8;
    sh = (int)(blockIdx.x % nsh);
    lo = ns * sh / nsh;
    hi = ns * (sh + 1) / nsh;
  }
  // The workgroup's next sample (>= hi: none left).  Every thread calls it;
  // its first barrier also ends the previous sample's use of LDS.
  __device__ int64_t next(int64_t* slot) const {
    __syncthreads();
    if (threadIdx.x == 0) *slot = lo + (int64_t)atomicAdd(&ctr[sh], 1ull);
    __syncthreads();
    return *slot;
  }
};

// Clears the eight ticket counters of a solver launch.
__global__ void zero_u64x8_kernel(unsigned long long* p) { p[threadIdx.x] = 0ull; }

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Slot j (0..7) of lane group q in a 32-deep contraction block stands for
// index kappa(q, j) of that block: rows 4q..4q+3 of its first and of its
// second 16-row tile, which are the two accumulator fragments a lane holds.
// Any bijection works as long as both operands use the same one.
__host__ __device__ constexpr int kappa(int q, int j) { return j < 4 ? 4 * q + j : 16 + 4 * q + (j - 4); }

int dst_padded(int n) {
  const int m = n - 1;
  return m <= 32 ? 32 : (m <= 64 ? 64 : 0);
}

int64_t dst_frag_bytes(int mp) { return (int64_t)(mp / 32) * (mp / 16) * 64 * (int64_t)sizeof(half8); }

// frag[(kb * NT + t) * 64 + lane][j] = S[32 kb + kappa(q, j)][16 t + (lane & 15)]
// (zero outside the m x m block); lam[p] = lambda_p (1 on padding, where the
// transformed residual is exactly zero).
__global__ void dst_tables_kernel(int n, int mp, half8* __restrict__ frag, float* __restrict__ lam) {
  const int nt = mp / 16, nkb = mp / 32, m = n - 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nkb * nt * 64) {
    const int lane = e & 63, f = e >> 6, kb = f / nt, t = f % nt;
    const int q = lane >> 4, col = 16 * t + (lane & 15);
    const double sc = sqrt(2.0 / n);
    half8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int row = 32 * kb + kappa(q, j);
      const double s = (row < m && col < m) ? sc * sinpi((double)((row + 1) * (col + 1)) / n) : 0.0;
      v[j] = (_Float16)(float)s;
    }
    frag[e] = v;
  }
  if (e < mp) {
    const double sv = sinpi((e + 1) / (2.0 * n));
    lam[e] = e < m ? (float)(4.0 * sv * sv) : 1.0f;
  }
}

void dst_tables_build(int n, void* frag, float* lam, hipStream_t st) {
  const int mp = dst_padded(n);
  const int cnt = (mp / 32) * (mp / 16) * 64;
  hipLaunchKernelGGL(dst_tables_kernel, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, n, mp,
                     static_cast<half8*>(frag), lam);
  USFFT_HIP(hipGetLastError());
}

__device__ __forceinline__ void store_h4(_Float16* p, floatx4 a) {
  half4 h = {(_Float16)a[0], (_Float16)a[1], (_Float16)a[2], (_Float16)a[3]};
  *reinterpret_cast<half4*>(p) = h;
}

// B-operand fragment of a column-major exchange tile: rows r0 + 0..3 and
// r0 + 16..19 of one column.
__device__ __forceinline__ half8 load_h8(const _Float16* p) {
  const half4 lo = *reinterpret_cast<const half4*>(p);
  const half4 hi = *reinterpret_cast<const half4*>(p + 16);
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// z = (L + shift I)^-1 r for the wave's strip (see the file comment).  r and
// z are in the node layout; sc scales r before the fp16 conversion (z is
// scaled back).
// Pitch of the optional table of the diagonal 1 / (lam_a + lam_b + shift)
// (column b, row a: entry b * (MP + 4) + a); rows of one column are
// contiguous for the 4-wide reads, the padding spreads columns over banks.
__host__ __device__ constexpr int dst_ilam_pitch(int mp) { return mp + 4; }

// The transform fragments come from the lane's registers (an array of
// (MP / 32) (MP / 16) half8) or, where they would not fit, from LDS
// (FragLds: fragment f of the lane at p[64 f + lane]).
struct FragLds {
  const half8* p;
  int lane;
  __device__ __forceinline__ half8 operator[](int f) const { return p[f * 64 + lane]; }
};

template <int MP, typename T, bool TAB = false, typename SF>
__device__ __forceinline__ void dst_apply(const T (&r)[MP / 4], float sc, float (&z)[MP / 4], const SF& sf,
                                          _Float16* xa, _Float16* xb, const float* lam, float shift,
                                          const float* ilam = nullptr) {
  constexpr int NT = MP / 16, KB = MP / 32, LDX = MP + 4;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c16 = lane & 15;
  half8 a[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) a[kb][j] = (_Float16)((float)r[4 * (2 * kb + (j >> 2)) + (j & 3)] * sc);
  floatx4 acc[NT];
  // T1 = R^T S: row strip w of T1
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[kb], sf[kb * NT + t], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) store_h4(xa + (16 * t + c16) * LDX + 16 * w + 4 * q, acc[t]);
  __syncthreads();
  // Wt = S T1: column strip w of Wt, then Yt = Lam o Wt
  half8 b[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) b[kb] = load_h8(xa + (16 * w + c16) * LDX + 32 * kb + 4 * q);
  const float lc = lam[16 * w + c16];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(sf[kb * NT + t], b[kb], acc[t], 0, 0, 0);
    if constexpr (TAB) {
      const floatx4 il = *reinterpret_cast<const floatx4*>(ilam + (16 * w + c16) * dst_ilam_pitch(MP) + 16 * t + 4 * q);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][v] *= il[v];
    } else {
      const floatx4 lr = *reinterpret_cast<const floatx4*>(lam + 16 * t + 4 * q);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][v] *= __builtin_amdgcn_rcpf(lr[v] + lc + shift);
    }
  }
  // T3 = Y S: row strip w of T3
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) a[kb][j] = (_Float16)acc[2 * kb + (j >> 2)][j & 3];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[kb], sf[kb * NT + t], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) store_h4(xb + (16 * t + c16) * LDX + 16 * w + 4 * q, acc[t]);
  __syncthreads();
  // Z = S T3: column strip w of Z, the node layout
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) b[kb] = load_h8(xb + (16 * w + c16) * LDX + 32 * kb + 4 * q);
  const float isc = 1.0f / sc;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(sf[kb * NT + t], b[kb], acc[t], 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) z[4 * t + v] = acc[t][v] * isc;
  }
}

// dst_apply for grids whose fragments do not fit in registers (MP = 128):
// the same four products with the fragments read from LDS where they are
// used, the stages whose results go to LDS loop over their tiles without
// unrolling, and the others take one tile at a time behind a scheduling
// fence, so no more than one tile's fragments and accumulators are live.
template <int MP>
__device__ void dst_apply_big(const float (&r)[MP / 4], float sc, float (&z)[MP / 4], const FragLds& sf,
                              _Float16* xa, _Float16* xb, const float* lam, float shift) {
  constexpr int NT = MP / 16, KB = MP / 32, LDX = MP + 4;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c16 = lane & 15;
  half8 a[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) a[kb][j] = (_Float16)(r[4 * (2 * kb + (j >> 2)) + (j & 3)] * sc);
  // T1 = R^T S: row strip w of T1
#pragma unroll 1
  for (int t = 0; t < NT; ++t) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[kb], sf[kb * NT + t], acc, 0, 0, 0);
    store_h4(xa + (16 * t + c16) * LDX + 16 * w + 4 * q, acc);
  }
  __syncthreads();
  // Wt = S T1: column strip w of Wt, then Yt = Lam o Wt, kept as the A
  // operand of the next product
  half8 b[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) b[kb] = load_h8(xa + (16 * w + c16) * LDX + 32 * kb + 4 * q);
  const float lc = lam[16 * w + c16];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(sf[kb * NT + t], b[kb], acc, 0, 0, 0);
    const floatx4 lr = *reinterpret_cast<const floatx4*>(lam + 16 * t + 4 * q);
#pragma unroll
    for (int v = 0; v < 4; ++v) a[t >> 1][4 * (t & 1) + v] = (_Float16)(acc[v] * __builtin_amdgcn_rcpf(lr[v] + lc + shift));
    __builtin_amdgcn_sched_barrier(0);
  }
  // T3 = Y S: row strip w of T3
#pragma unroll 1
  for (int t = 0; t < NT; ++t) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[kb], sf[kb * NT + t], acc, 0, 0, 0);
    store_h4(xb + (16 * t + c16) * LDX + 16 * w + 4 * q, acc);
  }
  __syncthreads();
  // Z = S T3: column strip w of Z, the node layout
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) b[kb] = load_h8(xb + (16 * w + c16) * LDX + 32 * kb + 4 * q);
  const float isc = 1.0f / sc;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(sf[kb * NT + t], b[kb], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) z[4 * t + v] = acc[v] * isc;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// 2^-round(log2 |r|) from |r|^2, so the scaled residual has norm ~1.
__device__ __forceinline__ float pow2_scale(double rr) {
  if (!(rr > 0.0) || !(rr < 1e300)) return 1.0f;
  const int e = ilogb(rr) / 2;
  return ldexpf(1.0f, -(e < -100 ? -100 : (e > 100 ? 100 : e)));
}

// Shift of the preconditioner from the scaled weights of one sample.  For a
// smooth coefficient the scaled operator is close to L + h^2 V with
// V = lap(sqrt(a)) / sqrt(a) (substitute u = a^-1/2 v); its row sums away
// from the boundary are h^2 V at the node, and their mean (clamped at 0, so
// that the preconditioner stays positive definite) is a constant shift that
// keeps the preconditioner diagonal in the DST basis: (L + shift I)^-1.
__device__ __forceinline__ float potential_shift(double rowsum, int m) {
  if (m < 3) return 0.0f;
  const double c = rowsum / ((double)(m - 2) * (double)(m - 2));
  return c > 0.0 ? (float)c : 0.0f;
}

// LDS grids of one workgroup have the compile-time pitch PP = MP + 2 >= n + 1
// (zero halo at rows/columns 0 and n, unused space beyond), so every stencil
// access is a base register plus an immediate offset.
__host__ __device__ constexpr int dst_pitch(int mp) { return mp + 2; }
__host__ __device__ constexpr int64_t dst_grid_elems(int mp) {
  return ((int64_t)dst_pitch(mp) * dst_pitch(mp) + 3) / 4 * 4;
}

// Resident waves per SIMD the register allocation targets: float32 state fits
// two 64-wide strips per SIMD (two samples per CU at MP = 64), float64 state
// one.
template <typename T, int MP, bool LR>
constexpr int dst_waves() {
  return LR ? 1 : (std::is_same<T, float>::value ? (MP == 64 ? 2 : 3) : (MP == 64 ? 1 : 2));
}

// Doubles of one grid of a workgroup's global scratch (pitch PP); the
// scratch holds three per workgroup: eh, ev and D^-1/2.
int64_t dst_edge_stride(int mp) { return ((int64_t)dst_pitch(mp) * dst_pitch(mp) + 31) / 32 * 32; }

// Dynamic LDS bytes of one workgroup.  Variants 0 and 1: [u (float32
// solves), float64][p, T][exchange tiles][variant 1: eh, ev float64,
// D^-1/2 in T].  Variant 2 (float32 only): [overlay, GE doubles][D^-1/2,
// float32][preconditioner diagonal, MP x (MP + 4) float32].
int64_t dst_lds_bytes(int n, int precision, int variant) {
  const int mp = dst_padded(n);
  const int64_t g = dst_grid_elems(mp);
  if (variant == 2) return g * 8 + g * 4 + (int64_t)mp * dst_ilam_pitch(mp) * 4;
  const int64_t grids = precision == USFFT_FP64 ? g * 8 : g * 8 + g * 4;
  return grids + 2 * (int64_t)mp * (mp + 4) * 2 + (variant == 1 ? g * (8 + 8 + (precision == USFFT_FP64 ? 8 : 4)) : 0);
}

// One-lane shift of a wave (DPP wave_shr:1): lane l gets lane l-1's value,
// lane 0 keeps its own.
__device__ __forceinline__ double wave_shr1(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xF, 0xF, false));
}

// Assembly of one sample (eq. (1.2) at the triangle centroids; the lognormal
// model exponentiates the sum per triangle): the edge
// grids eh[j PP + i] = (aL(i,j) + aU(i,j-1))/2 (i < n, 1 <= j < n) and
// ev[j PP + i] = (aU(i,j) + aL(i-1,j))/2 (1 <= i < n, j < n), and the Jacobi
// scaling D^-1/2 of every interior node, written to dg.  Float32 solves keep
// it rounded to float32 (their float64 true residual uses the unscaled
// operator, so the scaled diagonal need not be exactly 4 there); float64
// solves keep it in float64, where the scaled diagonal is 4 to rounding.
// Lane = cell column ci, each wave sweeps blocks of CB cell rows cj (plus
// the row below).  a(ci, cj) = a0 + sum_k (coef_k x_k(ci)) y_k(cj) is
// separable: with k outermost, the per-lane factors are loaded once per k and
// the row factors are wave-uniform (scalar loads).  Column ci-1's
// coefficients come from the neighbouring lane; columns are covered in
// chunks of 64 lanes overlapping by one (lane 0 of a later chunk only
// supplies its neighbour's values).
// Where the assembly puts the edge weights: float64 grids (LDS or global
// scratch), or float32 LDS grids for the float32 iteration plus float64
// copies in global scratch for the float64 true residual.
struct EdgesF64 {
  double* __restrict__ eh;
  double* __restrict__ ev;
  __device__ __forceinline__ void h(int i, double x) const { eh[i] = x; }
  __device__ __forceinline__ void v(int i, double x) const { ev[i] = x; }
};
struct EdgesSplit {
  float* __restrict__ eh;
  float* __restrict__ ev;
  double* __restrict__ geh;
  double* __restrict__ gev;
  __device__ __forceinline__ void h(int i, double x) const { eh[i] = (float)x; geh[i] = x; }
  __device__ __forceinline__ void v(int i, double x) const { ev[i] = (float)x; gev[i] = x; }
};

template <int NWAVE, int CB, typename DT, typename EW>
__device__ void assemble(const PdeDev& P, const double* coef, const EW& ew, DT* __restrict__ dg, int PP, int tid) {
  const int n = P.n, d = P.d, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double* txL = P.tab;                  // x1 factor, lower triangles
  const double* txU = P.tab + (size_t)d * n;  // x1 factor, upper triangles
  // the row factors are wave-uniform and read-only: scalar loads through the
  // constant address space, from the padded copies where the CB + 1 rows of
  // a block are contiguous
  typedef const __attribute__((address_space(4))) double* cdp;
  const int S = row_tab_pitch(n);
  const cdp tyL = (cdp)(P.tab + (size_t)4 * d * n);
  const cdp tyU = tyL + (size_t)d * S;
  for (int c0 = 0; c0 == 0 || c0 + 1 < n; c0 += 63) {
    const int ci = c0 + lane;
    const bool act = ci < n, outp = act && (c0 == 0 || lane >= 1);
    const int cic = min(ci, n - 1);  // clamped: table loads stay unconditional
    for (int cb = wave * CB; cb < n; cb += NWAVE * CB) {
      // row u of the block is cell row cj = cb - 1 + u
      // the lognormal model sums the exponent and exponentiates below
      const bool logn = P.model == USFFT_MODEL_LOGNORMAL;
      double aL[CB + 1], aU[CB + 1];
#pragma unroll
      for (int u = 0; u <= CB; ++u) aL[u] = aU[u] = logn ? 0.0 : P.a0;
      // the per-lane factors of KC consecutive k are loaded together (a
      // scheduling fence keeps the loads ahead of their uses), so one memory
      // latency covers KC terms
      constexpr int KC = 8;
      for (int k0 = 0; k0 < d; k0 += KC) {
        double txl[KC], txu[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          const int kc = min(k0 + j, d - 1);
          txl[j] = txL[kc * n + cic];
          txu[j] = txU[kc * n + cic];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          const int k = k0 + j;
          if (k >= d) break;
          const double ck = coef[k];
          const double xl = act ? ck * txl[j] : 0.0, xu = act ? ck * txu[j] : 0.0;
          // rows cb - 1 .. cb - 1 + CB are entries cb .. cb + CB < S of the
          // padded rows (rows outside [0, n) repeat the end rows; their
          // values are never used); all row factors of one k are loaded
          // before any is used
          const cdp yLk = tyL + k * S + cb, yUk = tyU + k * S + cb;
          double yl[CB + 1], yu[CB + 1];
#pragma unroll
          for (int u = 0; u <= CB; ++u) {
            yl[u] = yLk[u];
            yu[u] = yUk[u];
          }
#pragma unroll
          for (int u = 0; u <= CB; ++u) {
            aL[u] += xl * yl[u];
            aU[u] += xu * yu[u];
          }
        }
      }
      if (logn) {
#pragma unroll
        for (int u = 0; u <= CB; ++u) {
          aL[u] = P.a0 + exp(aL[u]);
          aU[u] = P.a0 + exp(aU[u]);
        }
      }
#pragma unroll
      for (int u = 1; u <= CB; ++u) {
        const int cj = cb - 1 + u;
        const double aLm = wave_shr1(aL[u]), aUm1 = wave_shr1(aU[u - 1]), aLm1 = wave_shr1(aL[u - 1]);
        if (cj >= n || !outp) continue;
        const double ehc = 0.5 * (aL[u] + aU[u - 1]);  // eh(ci, cj)
        const double evc = 0.5 * (aU[u] + aLm);        // ev(ci, cj)
        if (cj >= 1) ew.h(cj * PP + ci, ehc);
        if (ci >= 1) ew.v(cj * PP + ci, evc);
        if (ci >= 1 && cj >= 1) {
          const double ehm = 0.5 * (aLm + aUm1);        // eh(ci-1, cj)
          const double evm = 0.5 * (aU[u - 1] + aLm1);  // ev(ci, cj-1)
          const double dd = 0.25 * (ehc + ehm + evc + evm);
          // float32 scalings: the hardware reciprocal square root refined by
          // one float64 Newton step, then rounded (the float32 iteration
          // takes the scaled diagonal as 4, so the scaling must be the
          // nearest float32, not merely close)
          if constexpr (std::is_same<DT, float>::value) {
            const double y0 = (double)__builtin_amdgcn_rsqf((float)dd);
            dg[cj * PP + ci] = (float)(y0 * (1.5 - 0.5 * dd * y0 * y0));
          } else
            dg[cj * PP + ci] = 1.0 / sqrt(dd);
        }
      }
    }
  }
}

template <typename T, int MP, bool LR>
__global__ __launch_bounds__(4 * MP) __attribute__((amdgpu_waves_per_eu(dst_waves<T, MP, LR>()))) void pcgdst_kernel(
    const SolveSeg* __restrict__ segs, int nseg, int64_t ns, double rtol, int maxit, double inner_rtol,
    int refine_every, int out_fp32,
    double* __restrict__ wscr, int64_t wstride, const half8* __restrict__ sfrag, const float* __restrict__ lamtab,
    unsigned long long* __restrict__ tick) {
  constexpr int NT = MP / 16, KB = MP / 32, E = 4 * NT, BLOCK = 4 * MP, LDX = MP + 4;
  constexpr int PP = dst_pitch(MP);
  constexpr int64_t GE = dst_grid_elems(MP);
  constexpr bool REFINE = std::is_same<T, float>::value;
  extern __shared__ double lds[];
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  __shared__ __attribute__((aligned(16))) float slam[MP];
  const int n = segs[0].pde.n, m = n - 1;  // every segment has this mesh
  double* sx = lds;                                          // float32 path: float64 iterate u
  T* sp = reinterpret_cast<T*>(lds + (REFINE ? GE : 0));    // search direction (zero halo), staging
  _Float16* xa = reinterpret_cast<_Float16*>(sp + GE);      // exchange tiles, column-major
  _Float16* xb = xa + MP * LDX;
  // float64 edge grids and the float32 Jacobi scaling, pitch PP like the
  // LDS grids: in LDS (LR, one workgroup per CU) or in this workgroup's slot
  // of the global scratch
  double* eh;
  double* ev;
  T* dg;
  if constexpr (LR) {
    eh = reinterpret_cast<double*>(xb + MP * LDX);
    ev = eh + GE;
    dg = reinterpret_cast<T*>(ev + GE);
  } else {
    eh = wscr + (size_t)blockIdx.x * 3 * wstride;
    ev = eh + wstride;
    dg = reinterpret_cast<T*>(ev + wstride);
  }

  const int lane = threadIdx.x & 63;
  half8 sf[KB * NT];
#pragma unroll
  for (int f = 0; f < KB * NT; ++f) sf[f] = sfrag[f * 64 + lane];
  for (int i = threadIdx.x; i < MP; i += BLOCK) slam[i] = lamtab[i];
  for (int64_t e = threadIdx.x; e < GE; e += BLOCK) {
    sp[e] = (T)0;
    if (REFINE) sx[e] = 0.0;
    dg[e] = (T)0;  // the halo stays zero: boundary couplings vanish in the scaled weights
  }

  const Tickets tk(tick, ns);
  __shared__ int64_t s_next;
  for (;;) {
    const int64_t s = tk.next(&s_next);  // the previous sample is done with LDS, coef and the edge grids
    if (s >= tk.hi) break;
    // lane coordinates are re-derived per sample (opaque to the optimiser):
    // hoisted out of the sample loop, per-node addresses would spill
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int q = (tid & 63) >> 4, c = 16 * (tid >> 6) + (tid & 15);
    // node e = 4 t + v of this lane: row 16 t + 4 q + v, column c, grid index
    // base + off(e); padding nodes (row or column >= m) carry zeros, their
    // slots lie on the zero halo or beyond it
    const int base = (4 * q + 1) * PP + c + 1;
    T* spl = sp + base;
    auto off = [](int e) { return (16 * (e >> 2) + (e & 3)) * PP; };
    // the job segment of sample s (a fused launch serves several jobs'
    // batches; each segment has its coefficient family, nodes and output)
    int ks = 0;
    for (int a = 1; a < nseg; ++a) ks = segs[a].begin <= s ? a : ks;
    const SolveSeg& sg = segs[ks];
    const int64_t sl = s - sg.begin;
    load_coef(sg.pde, sg.Y, sl, coef);
    __syncthreads();
    assemble<BLOCK / 64, LR ? 16 : 8>(sg.pde, coef, EdgesF64{eh, ev}, dg, PP, tid);
    __syncthreads();
    // scaled weights: wE, wW, wS per node; wN(v) = wS(v + 1) inside a 4-row
    // group, so only the top row of each group keeps its own (wN4)
    // diagonal of the scaled operator: exactly 4 for float64 solves; float32
    // solves with the LDS-resident scratch keep d_i^2 A_ii (their D^-1/2 is
    // rounded to float32), the others use 4 and leave the difference to the
    // float64 true residual
    constexpr bool DIAG = REFINE && LR;
    T wE[E], wW[E], wS[E], wN4[NT], r[E], p[E], dx[E], dd[DIAG ? E : 1];
    double bb = 0.0;
    {
      const T* sdl = dg + base;
      const double* ehl = eh + base;
      const double* evl = ev + base;
      // padding slots read in-bounds garbage (unwritten scratch) that the
      // selects discard; without branches all loads are in flight together
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int t = e >> 2, v = e & 3, row = 16 * t + 4 * q + v, o = off(e);
        const bool ok = row < m && c < m;
        const double di = sdl[o];
        dx[e] = (T)0;
        wE[e] = ok ? (T)(ehl[o] * di * sdl[o + 1]) : (T)0;
        wW[e] = ok ? (T)(ehl[o - 1] * di * sdl[o - 1]) : (T)0;
        wS[e] = ok ? (T)(evl[o - PP] * di * sdl[o - PP]) : (T)0;
        if (v == 3) wN4[t] = ok ? (T)(evl[o] * di * sdl[o + PP]) : (T)0;
        if constexpr (DIAG)
          dd[e] = ok ? (T)(di * di * (ehl[o] + ehl[o - 1] + evl[o] + evl[o - PP])) : (T)0;
        const double bt = ok ? di * sg.pde.h2 : 0.0;
        r[e] = (T)bt;
        bb += bt * bt;
      }
    }
    double rs = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int row = 16 * (e >> 2) + 4 * q + (e & 3);
      const T wn = (e & 3) == 3 ? wN4[e >> 2] : wS[e + 1];
      const T diag = DIAG ? dd[DIAG ? e : 0] : (T)4;
      if (row >= 1 && row <= m - 2 && c >= 1 && c <= m - 2) rs += (double)(diag - (wE[e] + wW[e] + wn + wS[e]));
    }
    block_sum2<BLOCK>(bb, rs, red0);
    const float shift = potential_shift(rs, m);
    if (REFINE)
      for (int g = tid; g < m * m; g += BLOCK) sx[(g / m + 1) * PP + g % m + 1] = 0.0;  // u = 0
    float z[E];
    dst_apply<MP, T>(r, pow2_scale(bb), z, sf, xa, xb, slam, shift);
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      p[e] = (T)z[e];
      rz += (double)r[e] * (double)z[e];
      rr += (double)r[e] * (double)r[e];
    }
    block_sum2<BLOCK>(rz, rr, red1);
    const double stop = rtol * rtol * bb;
    const double drop = inner_rtol * inner_rtol;
    double rr_ref = rr;
    int it = 0, last_update = 0;
    bool conv = !(bb > 0.0);
    while (!conv && it < maxit) {
#pragma unroll
      for (int e = 0; e < E; ++e) spl[off(e)] = p[e];
      __syncthreads();
      T qv[E];
      double pq = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int o = off(e);
        const T wn = (e & 3) == 3 ? wN4[e >> 2] : wS[e + 1];
        const T diag = DIAG ? dd[DIAG ? e : 0] : (T)4;
        qv[e] = diag * p[e] - (wE[e] * spl[o + 1] + wW[e] * spl[o - 1] + wn * spl[o + PP] + wS[e] * spl[o - PP]);
        pq += (double)(p[e] * qv[e]);
      }
      pq = block_sum<BLOCK>(pq, red0);
      const T alpha = (T)(rz / pq);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        dx[e] += alpha * p[e];
        r[e] -= alpha * qv[e];
      }
      dst_apply<MP, T>(r, pow2_scale(rr), z, sf, xa, xb, slam, shift);
      double rz2 = 0.0;
      rr = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        rz2 += (double)r[e] * (double)z[e];
        rr += (double)r[e] * (double)r[e];
      }
      block_sum2<BLOCK>(rz2, rr, red1);
      ++it;
      if (REFINE) {
        if (rr <= drop * rr_ref || it - last_update >= refine_every) {
          // u += D^-1/2 dx in float64, then the float64 true residual
          // (scaled) replaces the float32 one; the search direction is kept.
          // Both in the node layout; the base is opaque here so that the
          // per-node addresses are not hoisted out of the iteration.
          int b2 = base;
          asm volatile("" : "+v"(b2));
          const double* ehl = eh + b2;
          const double* evl = ev + b2;
          const T* dgl = dg + b2;
          double* sxl = sx + b2;
          // (padding slots: unconditional in-bounds loads, results discarded
          // by selects; sx stays zero there)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const bool ok = 16 * (e >> 2) + 4 * q + (e & 3) < m && c < m;
            const double du = dgl[off(e)] * (double)dx[e];
            sxl[off(e)] += ok ? du : 0.0;
            dx[e] = (T)0;
          }
          __syncthreads();
          double rr64 = 0.0;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int o = off(e);
            const bool ok = 16 * (e >> 2) + 4 * q + (e & 3) < m && c < m;
            const double xc = sxl[o];
            const double ax = ehl[o] * (xc - sxl[o + 1]) + ehl[o - 1] * (xc - sxl[o - 1]) +
                              evl[o] * (xc - sxl[o + PP]) + evl[o - PP] * (xc - sxl[o - PP]);
            const double rsv = dgl[o] * (sg.pde.h2 - ax);
            const double rs = ok ? rsv : 0.0;
            rr64 += rs * rs;
            r[e] = (T)rs;
          }
          rr64 = block_sum<BLOCK>(rr64, red0);
          last_update = it;
          if (rr64 <= stop) {
            conv = true;
            break;
          }
          dst_apply<MP, T>(r, pow2_scale(rr64), z, sf, xa, xb, slam, shift);
          rz2 = 0.0;
          rr = 0.0;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            rz2 += (double)r[e] * (double)z[e];
            rr += (double)r[e] * (double)r[e];
          }
          block_sum2<BLOCK>(rz2, rr, red1);
          rr_ref = rr;
        }
      } else if (rr <= stop) {
        conv = true;
        break;
      }
      const T beta = (T)(rz2 / rz);
      rz = rz2;
#pragma unroll
      for (int e = 0; e < E; ++e) p[e] = (T)z[e] + beta * p[e];
    }
    // u = D^-1/2 ut: float64 solves hold ut in dx, float32 solves the
    // correction not yet folded into u (each lane reads only its own nodes
    // of sx)
    {
      const T* dgl = dg + base;
      const double* sxl = sx + base;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int row = 16 * (e >> 2) + 4 * q + (e & 3);
        const double dv = dgl[off(e)] * (double)dx[e];
        const double u = REFINE ? sxl[off(e)] + dv : dv;
        if (row < m && c < m) store_sample(sg.out, out_fp32, ((int64_t)row * m + c) * sg.ld + sg.col0 + sl, u);
      }
    }
    if (tid == 0 && sg.iters) sg.iters[sl] = conv ? it : -1;
  }
}

// Float32 solves in a compact LDS footprint, so that two workgroups (MP = 64)
// share a CU and hide each other's barrier and LDS latency.  LDS holds one
// overlay region of GE doubles, the float32 Jacobi scaling and the
// sample's preconditioner diagonal 1 / (lam_a + lam_b + shift) (one
// reciprocal per entry per sample instead of one per entry per application):
//   assembly:     float32 edge grids eh, ev (the float64 edges go to this
//                 workgroup's slot of the global scratch),
//   iterations:   float32 search direction (zero halo) + exchange tiles,
//   true residual: float64 u = D^-1/2 ut (zero halo).
// The float64 scaled iterate ut stays in registers and takes alpha p every
// iteration.  The float32 recursive residual r - alpha q has its norm from
// one block reduction of (p.q, r.q, q.q) before the preconditioner:
// |r - alpha q|^2 = |r|^2 - 2 alpha r.q + alpha^2 q.q.  When it has dropped
// by inner_rtol (or after refine_every iterations) the float64 true residual
// b - A u, formed from the float64 edges, replaces it before the
// preconditioner runs, so no preconditioner application is spent on a
// residual that is thrown away.  Convergence is decided on the float64 true
// residual only.
template <int MP>
__global__ __launch_bounds__(4 * MP) __attribute__((amdgpu_waves_per_eu(MP == 64 ? 2 : 4))) void pcgdst32c_kernel(
    const SolveSeg* __restrict__ segs, int nseg, int64_t ns, double rtol, int maxit, double inner_rtol,
    int refine_every, int out_fp32,
    double* __restrict__ wscr, int64_t wstride, const half8* __restrict__ sfrag, const float* __restrict__ lamtab,
    unsigned long long* __restrict__ tick) {
  constexpr int NT = MP / 16, KB = MP / 32, E = 4 * NT, BLOCK = 4 * MP, LDX = MP + 4;
  constexpr int PP = dst_pitch(MP);
  constexpr int64_t GE = dst_grid_elems(MP);
  static_assert(GE * 4 + 2 * MP * LDX * 2 <= GE * 8, "exchange tiles must fit the overlay");
  extern __shared__ double lds[];
  __shared__ double coef[kMaxD];
  __shared__ double red0[3 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  __shared__ __attribute__((aligned(16))) float slam[MP];
  const int n = segs[0].pde.n, m = n - 1;  // every segment has this mesh
  double* su = lds;                                        // overlay: float64 u
  float* sp = reinterpret_cast<float*>(lds);               // overlay: search direction
  _Float16* xa = reinterpret_cast<_Float16*>(sp + GE);     // overlay: exchange tiles
  _Float16* xb = xa + MP * LDX;
  float* feh = sp;                                         // overlay: float32 edges
  float* fev = sp + GE;
  float* dg = reinterpret_cast<float*>(lds + GE);          // D^-1/2
  float* ilam = dg + GE;                                   // 1 / (lam_a + lam_b + shift)
  double* geh = wscr + (size_t)blockIdx.x * 2 * wstride;   // float64 edges
  double* gev = geh + wstride;

  const int lane = threadIdx.x & 63;
  half8 sf[KB * NT];
#pragma unroll
  for (int f = 0; f < KB * NT; ++f) sf[f] = sfrag[f * 64 + lane];
  for (int i = threadIdx.x; i < MP; i += BLOCK) slam[i] = lamtab[i];
  for (int64_t e = threadIdx.x; e < GE; e += BLOCK) dg[e] = 0.0f;  // zero halo: boundary couplings vanish
  // zero ring (rows and columns 0 and PP-1) of a grid of pitch PP
  auto zero_ring = [&](auto* g) {
    const int t = threadIdx.x;
    if (t < PP) {
      g[t] = 0;
      g[(PP - 1) * PP + t] = 0;
      g[t * PP] = 0;
      g[t * PP + PP - 1] = 0;
    }
  };

  const Tickets tk(tick, ns);
  __shared__ int64_t s_next;
  for (;;) {
    const int64_t s = tk.next(&s_next);  // the previous sample is done with LDS and coef
    if (s >= tk.hi) break;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int q = (tid & 63) >> 4, c = 16 * (tid >> 6) + (tid & 15);
    const int base = (4 * q + 1) * PP + c + 1;
    auto off = [](int e) { return (16 * (e >> 2) + (e & 3)) * PP; };
    // the job segment of sample s (a fused launch serves several jobs'
    // batches; each segment has its coefficient family, nodes and output)
    int ks = 0;
    for (int a = 1; a < nseg; ++a) ks = segs[a].begin <= s ? a : ks;
    const SolveSeg& sg = segs[ks];
    const int64_t sl = s - sg.begin;
    load_coef(sg.pde, sg.Y, sl, coef);
    __syncthreads();
    assemble<BLOCK / 64, MP / 4>(sg.pde, coef, EdgesSplit{feh, fev, geh, gev}, dg, PP, tid);
    __syncthreads();
    float wE[E], wW[E], wS[E], wN4[NT], r[E], p[E];
    double ux[E];
    double bb = 0.0;
    {
      const float* sdl = dg + base;
      const float* ehl = feh + base;
      const float* evl = fev + base;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int t = e >> 2, v = e & 3, row = 16 * t + 4 * q + v, o = off(e);
        const bool ok = row < m && c < m;
        const float di = sdl[o];
        ux[e] = 0.0;
        wE[e] = ok ? ehl[o] * di * sdl[o + 1] : 0.0f;
        wW[e] = ok ? ehl[o - 1] * di * sdl[o - 1] : 0.0f;
        wS[e] = ok ? evl[o - PP] * di * sdl[o - PP] : 0.0f;
        if (v == 3) wN4[t] = ok ? evl[o] * di * sdl[o + PP] : 0.0f;
        const double bt = ok ? (double)di * sg.pde.h2 : 0.0;
        r[e] = (float)bt;
        bb += bt * bt;
      }
    }
    double rs = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int row = 16 * (e >> 2) + 4 * q + (e & 3);
      const float wn = (e & 3) == 3 ? wN4[e >> 2] : wS[e + 1];
      if (row >= 1 && row <= m - 2 && c >= 1 && c <= m - 2) rs += (double)(4.0f - (wE[e] + wW[e] + wn + wS[e]));
    }
    block_sum2<BLOCK>(bb, rs, red0);  // every lane is done with the edge grids
    const float shift = potential_shift(rs, m);
    // the diagonal of this sample's preconditioner; the first read follows
    // the barrier inside dst_apply
    for (int i = tid; i < MP * MP; i += BLOCK)
      ilam[(i / MP) * dst_ilam_pitch(MP) + i % MP] = __builtin_amdgcn_rcpf(slam[i % MP] + slam[i / MP] + shift);
    zero_ring(sp);
    float z[E];
    dst_apply<MP, float, true>(r, pow2_scale(bb), z, sf, xa, xb, slam, shift, ilam);
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      p[e] = z[e];
      rz += (double)r[e] * (double)z[e];
      rr += (double)r[e] * (double)r[e];
    }
    block_sum2<BLOCK>(rz, rr, red1);
    const double stop = rtol * rtol * bb;
    const double drop = inner_rtol * inner_rtol;
    double rr_ref = rr;
    int it = 0, last_update = 0;
    bool conv = !(bb > 0.0);
    while (!conv && it < maxit) {
      float* spl = sp + base;
#pragma unroll
      for (int e = 0; e < E; ++e) spl[off(e)] = p[e];
      __syncthreads();
      // these sums only steer the float32 recursion (the float64 true
      // residual decides convergence): float32 throughout
      float qv[E], pqf = 0.0f, rqf = 0.0f, qqf = 0.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int o = off(e);
        const float wn = (e & 3) == 3 ? wN4[e >> 2] : wS[e + 1];
        // a lane's rows 4q .. 4q+3 of a tile are consecutive: the row above
        // and below come from its own registers except at the group ends
        // (the same values the lane stored to sp before the barrier)
        const float pN = (e & 3) == 3 ? spl[o + PP] : p[(e & 3) == 3 ? e : e + 1];
        const float pS = (e & 3) == 0 ? spl[o - PP] : p[(e & 3) == 0 ? e : e - 1];
        qv[e] = 4.0f * p[e] - (wE[e] * spl[o + 1] + wW[e] * spl[o - 1] + wn * pN + wS[e] * pS);
        pqf = fmaf(p[e], qv[e], pqf);
        rqf = fmaf(r[e], qv[e], rqf);
        qqf = fmaf(qv[e], qv[e], qqf);
      }
      block_sum3<BLOCK>(pqf, rqf, qqf, reinterpret_cast<float*>(red0));
      const double pq = pqf, rq = rqf, qq = qqf;
      const double alpha = rz / pq;
      const float af = (float)alpha;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        ux[e] += alpha * (double)p[e];
        r[e] -= af * qv[e];
      }
      rr = fmax(rr - 2.0 * alpha * rq + alpha * alpha * qq, 0.0);
      ++it;
      if (rr <= drop * rr_ref || it - last_update >= refine_every) {
        // float64 true residual of u = D^-1/2 ut; every lane is past the
        // stencil reads of sp (block_sum3) and the exchange tiles
        int b2 = base;
        asm volatile("" : "+v"(b2));
        double* sul = su + b2;
        const float* dgl = dg + b2;
        zero_ring(su);
#pragma unroll
        for (int e = 0; e < E; ++e) sul[off(e)] = (double)dgl[off(e)] * ux[e];  // padding: ux = 0
        __syncthreads();
        const double* ehl = geh + b2;
        const double* evl = gev + b2;
        double rr64 = 0.0;
        // the edges of half the lane's nodes are loaded before any is used
        // (a scheduling fence keeps them together), so their global reads
        // overlap instead of queueing behind one another
        constexpr int HE = E / 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double we[HE], ww[HE], wn[HE], ws[HE];
#pragma unroll
          for (int i = 0; i < HE; ++i) {
            const int o = off(h * HE + i);
            we[i] = ehl[o];
            ww[i] = ehl[o - 1];
            wn[i] = evl[o];
            ws[i] = evl[o - PP];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < HE; ++i) {
            const int e = h * HE + i, o = off(e);
            const bool ok = 16 * (e >> 2) + 4 * q + (e & 3) < m && c < m;
            const double xc = sul[o];
            const double ax = we[i] * (xc - sul[o + 1]) + ww[i] * (xc - sul[o - 1]) + wn[i] * (xc - sul[o + PP]) +
                              ws[i] * (xc - sul[o - PP]);
            const double rsv = (double)dgl[o] * (sg.pde.h2 - ax);
            const double rs = ok ? rsv : 0.0;
            rr64 += rs * rs;
            r[e] = (float)rs;
          }
        }
        rr64 = block_sum<BLOCK>(rr64, red1);  // every lane is done with su
        {
          // the transform fragments are read again instead of being held
          // across the residual, whose edge loads need their registers
          const half8* sfr = sfrag;
          asm volatile("" : "+s"(sfr));
#pragma unroll
          for (int f = 0; f < KB * NT; ++f) sf[f] = sfr[f * 64 + lane];
        }
        last_update = it;
        if (rr64 <= stop) {
          conv = true;
          break;
        }
        zero_ring(sp);
        rr = rr_ref = rr64;
      }
      dst_apply<MP, float, true>(r, pow2_scale(rr), z, sf, xa, xb, slam, shift, ilam);
      float rzf = 0.0f, rrf = 0.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        rzf = fmaf(r[e], z[e], rzf);
        rrf = fmaf(r[e], r[e], rrf);
      }
      block_sum2<BLOCK>(rzf, rrf, reinterpret_cast<float*>(red1));
      const double rz2 = rzf, rre = rrf;
      rr = rre;
      const float beta = (float)(rz2 / rz);
      rz = rz2;
#pragma unroll
      for (int e = 0; e < E; ++e) p[e] = z[e] + beta * p[e];
    }
    {
      const float* dgl = dg + base;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int row = 16 * (e >> 2) + 4 * q + (e & 3);
        const double u = (double)dgl[off(e)] * ux[e];
        if (row < m && c < m) store_sample(sg.out, out_fp32, ((int64_t)row * m + c) * sg.ld + sg.col0 + sl, u);
      }
    }
    if (tid == 0 && sg.iters) sg.iters[sl] = conv ? it : -1;
  }
}

// ------------------------------------------ meshes 65 < mesh_n <= 129
// One sample's state no longer fits a CU, so the CG vectors live in a
// per-workgroup global workspace, as in the streaming Jacobi solver, while
// the fast-Poisson preconditioner still runs on the matrix cores: MP = 128,
// 512 threads, wave w owns the node strip of columns 16 w .. 16 w + 15 and a
// lane 32 of its nodes in the accumulator layout (rows 16 t + 4 q + v), the
// DST fragments (32 KB) and the exchange tiles in LDS.  Float64 CG with the
// preconditioner M^-1 = D^-1/2 (L + c I)^-1 D^-1/2 (D = diag(A) / 4, c the
// mean potential shift of the scaled operator, as in the on-chip kernels),
// stopped on |b - A x| <= rtol |b| with b - A x the recursive residual.
// Workspace per workgroup, slots of gp doubles: x, r, D^-1/2 (node arrays,
// index row NP + col, NP = m rounded up to 16), then one slot of floats: the
// direction p (halo grid, zero border) and D^-1/2 rounded to float, then eh,
// ev (edge grids); A p stays in registers.  The direction is stored in float:
// A p and the step x += alpha p take the same rounded values, so the
// recursive residual still tracks b - A x in float64, and only the search
// direction (already built from an fp16 preconditioner) is perturbed.  The halo grids have MP + 2 rows of PP >= 144 doubles, node
// (row, col) at (row + 1) PP + col + 16: every wave's 16-column strip starts
// on a 128-byte line, and every lane's 32 nodes and their neighbours lie
// inside the grid whether or not they are mesh nodes, so the passes load
// unconditionally (values of padding nodes are discarded by selects, their
// stores skipped) and issue a chunk's loads before its stores.  Before the
// edges exist, the x and r slots hold the two triangle grids.
constexpr int kDstStreamMP = 128;
constexpr int kDstStreamArrays = 6;
constexpr int kDstStreamOff = 15;  // halo index of node (row, col): (row + 1) PP + col + 1 + 15

__host__ __device__ constexpr int dst_stream_rowpitch(int n) {
  return ((n - 1 > kDstStreamMP - 1 ? n - 1 : kDstStreamMP - 1) + 17 + 15) / 16 * 16;
}

// LDS: the DST fragments, then either the two fp16 exchange tiles of the
// preconditioner or (during the assembly) one padded row-factor table
// (d rows of n + 16 doubles)
int64_t dst_stream_lds_bytes() {
  constexpr int MP = kDstStreamMP;
  const int64_t tiles = 2 * (int64_t)MP * (MP + 4) * 2, table = (int64_t)kMaxD * row_tab_pitch(MP + 1) * 8;
  return (int64_t)(MP / 32) * (MP / 16) * 64 * (int64_t)sizeof(half8) + std::max(tiles, table);
}

// a slot holds the halo grid (MP + 2 rows of PP) and the node arrays (MP
// rows of at most MP), rounded to 512 bytes; the float slot holds the float
// halo grid in its first half and the float node array in its second
int64_t dst_stream_pitch(int n) {
  const int64_t grid = (int64_t)(kDstStreamMP + 2) * dst_stream_rowpitch(n),
                nodes = (int64_t)kDstStreamMP * kDstStreamMP;
  return (std::max(grid, nodes) + 127) / 128 * 128;
}

// the per-workgroup slots, then eight ticket counters
int64_t dst_stream_workspace_doubles(int n, int blocks) {
  return dst_stream_pitch(n) * kDstStreamArrays * (int64_t)blocks + 8;
}

__global__ __launch_bounds__(4 * kDstStreamMP) void pcgdst_stream_kernel(
    PdeDev P, const double* __restrict__ Y, int64_t ns, double rtol, int maxit, void* __restrict__ out, int out_fp32,
    int64_t ld, int64_t col0, int* __restrict__ iters, double* __restrict__ ws, int64_t gp,
    const half8* __restrict__ sfrag, const float* __restrict__ lamtab, unsigned long long* __restrict__ tick) {
  constexpr int MP = kDstStreamMP, NT = MP / 16, KB = MP / 32, E = 4 * NT, BLOCK = 4 * MP, LDX = MP + 4;
  constexpr int EH = 8;  // nodes per load chunk of the update passes
  extern __shared__ double lds[];
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  __shared__ __attribute__((aligned(16))) float slam[MP];
  half8* sfl = reinterpret_cast<half8*>(lds);
  _Float16* xa = reinterpret_cast<_Float16*>(sfl + KB * NT * 64);
  _Float16* xb = xa + MP * LDX;
  const int n = P.n, m = n - 1, PP = dst_stream_rowpitch(n);
  // node array row pitch: m rounded up to 16 (a run-time value: with the
  // constant 128 the compiler folds the 32 nodes' offsets and holds their
  // addresses, 55 more registers)
  const int NP = (m + 15) / 16 * 16;
  double* x = ws + (size_t)blockIdx.x * kDstStreamArrays * gp;
  double* r = x + gp;
  double* dh = r + gp;  // written once per sample (the shift reads neighbours)
  float* p = reinterpret_cast<float*>(dh + gp);  // direction, halo grid, zero border
  float* dhf = p + gp;                            // D^-1/2 rounded to float, node index
  double* eh = dh + 2 * gp;
  double* ev = eh + gp;
  const int lane = threadIdx.x & 63, qq = lane >> 4, c = 16 * (threadIdx.x >> 6) + (lane & 15);
  for (int f = threadIdx.x; f < KB * NT * 64; f += BLOCK) sfl[f] = sfrag[f];
  for (int i = threadIdx.x; i < MP; i += BLOCK) slam[i] = lamtab[i];
  const FragLds sf{sfl, lane};
  // node e of the lane: row 4 qq + o(e), o(e) = 16 (e >> 2) + (e & 3) (the
  // accumulator layout), column c; its halo-grid index is bl + o PP and its
  // node-array index bg + o NP, with wave-uniform offsets o PP, o NP.  The
  // bases pass through an empty asm in every loop, so the 32 nodes' addresses
  // are not precomputed and held (they would not fit the registers).
  auto bases = [&](int& bl, int& bg) {
    bl = (4 * qq + 1) * PP + c + 1 + kDstStreamOff;
    bg = 4 * qq * NP + c;
    asm volatile("" : "+v"(bl), "+v"(bg));
  };
  auto ofs = [](int e) { return 16 * (e >> 2) + (e & 3); };
  const bool colok = c < m;
  auto node_ok = [&](int e) { return 4 * qq + ofs(e) < m && colok; };
  // the direction grid's border (and its padding nodes) is never written
  // afterwards: cleared once per launch
  for (int e = threadIdx.x; e < (MP + 2) * PP; e += BLOCK) p[e] = 0.0f;
  const Tickets tk(tick, ns);
  __shared__ int64_t s_next;
  for (;;) {
    const int64_t s = tk.next(&s_next);  // the previous sample is done with coef and the workspace
    if (s >= tk.hi) break;
    load_coef(P, Y, s, coef);
    __syncthreads();
    // the coefficient at the centroids of both triangles of every cell
    // (eq. (1.2)), each evaluated once: triangle q of cell (ci, cj) into
    // T_q[cj PP + ci] (T_0 in the x slot, T_1 in the r slot).  A lane takes
    // one cell column and a wave-uniform block of rows, so the row factors are
    // scalar loads and the column factor coef_k tab_k(ci) one vector load per
    // term; the sum runs over k in order, as in the other solvers' assembly.
    // The row factors come from the padded copies (rows of n + 16, row cj at
    // 1 + cj), staged in LDS over the exchange tiles, so a chunk of 16 rows
    // is one unconditional broadcast read even where it runs past the last
    // row (those sums are not stored); the column factors are loaded eight
    // terms at a time.
    {
      constexpr int RC = 16;  // rows per chunk
      const int S = row_tab_pitch(n);
      const int rpg = (n + 3) / 4;
      const int cj0 = __builtin_amdgcn_readfirstlane((threadIdx.x >> 7) * rpg);
      const int rows = min(rpg, n - cj0);
      const bool logn = P.model == USFFT_MODEL_LOGNORMAL;
      double* tyl = reinterpret_cast<double*>(xa);
#pragma unroll 1
      for (int qt = 0; qt < 2; ++qt) {
        double* T = qt == 0 ? x : r;
        __syncthreads();  // the previous table's readers are done
        {
          const double* tq = P.tab + (size_t)4 * P.d * n + (size_t)qt * P.d * S;
          for (int e = threadIdx.x; e < P.d * S; e += BLOCK) tyl[e] = tq[e];
        }
        __syncthreads();
        // column blocks of 128 with a wave-uniform trip count (a lane's
        // column clamped for the loads, its stores skipped past the last)
#pragma unroll 1
        for (int cb = 0; cb < n; cb += 128) {
          const int ci = min(cb + (int)(threadIdx.x & 127), n - 1);
          const bool cok = cb + (int)(threadIdx.x & 127) < n;
          const double* tx = P.tab + (size_t)qt * P.d * n + ci;
#pragma unroll 1
          for (int u0 = 0; u0 < rows; u0 += RC) {
            const double* ty = tyl + 1 + cj0 + u0;
            double acc[RC];
#pragma unroll
            for (int u = 0; u < RC; ++u) acc[u] = logn ? 0.0 : P.a0;
#pragma unroll 1
            for (int k0 = 0; k0 < P.d; k0 += 8) {
              double t8[8];
#pragma unroll
              for (int kk = 0; kk < 8; ++kk) t8[kk] = tx[(size_t)min(k0 + kk, P.d - 1) * n];
#pragma unroll
              for (int kk = 0; kk < 8; ++kk) {
                if (k0 + kk < P.d) {
                  const double w = coef[k0 + kk] * t8[kk];
                  const double* tyk = ty + (k0 + kk) * S;
#pragma unroll
                  for (int u = 0; u < RC; ++u) acc[u] += w * tyk[u];
                }
              }
            }
#pragma unroll
            for (int u = 0; u < RC; ++u)
              if (u0 + u < rows && cok) T[(cj0 + u0 + u) * PP + ci] = logn ? P.a0 + exp(acc[u]) : acc[u];
          }
        }
      }
    }
    __syncthreads();
    // edge weights (mean of the two triangles beside the edge), at halo
    // index j PP + i + 15: horizontal edge (i, j)-(i + 1, j), 1 <= j < n,
    // from T_0(i, j) and T_1(i, j - 1); vertical edge (i, j)-(i, j + 1),
    // 1 <= i < n, from T_1(i, j) and T_0(i - 1, j).  A lane walks its column
    // i through its block of rows (T_1 of the row below carried), eight rows
    // of loads before their stores.
    {
      const int rpg = (n + 3) / 4;
      const int j0 = (threadIdx.x >> 7) * rpg, j1 = min(j0 + rpg, n);
#pragma unroll 1
      for (int cb = 0; cb < n; cb += 128) {
        const int i = min(cb + (int)(threadIdx.x & 127), n - 1);
        const bool cok = cb + (int)(threadIdx.x & 127) < n;
        double t1b = j0 > 0 ? r[(j0 - 1) * PP + i] : 0.0;
#pragma unroll 1
        for (int jb = j0; jb < j1; jb += 8) {
          double a0[8], a1[8], aw[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = min(jb + u, n - 1);
            a0[u] = x[j * PP + i];
            a1[u] = r[j * PP + i];
            aw[u] = x[j * PP + max(i - 1, 0)];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = jb + u;
            if (j < j1 && cok) {
              if (j >= 1) eh[j * PP + i + kDstStreamOff] = 0.5 * (a0[u] + t1b);
              if (i >= 1) ev[j * PP + i + kDstStreamOff] = 0.5 * (a1[u] + aw[u]);
            }
            t1b = a1[u];
          }
        }
      }
    }
    __syncthreads();
    int bl, bg;
    // D^-1/2 and b
    double bb = 0.0, rs = 0.0;
    bases(bl, bg);
#pragma unroll
    for (int h = 0; h < E; h += 8) {
      double w4[8][4];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int l = bl + ofs(h + j) * PP;
        w4[j][0] = eh[l];
        w4[j][1] = eh[l - 1];
        w4[j][2] = ev[l];
        w4[j][3] = ev[l - PP];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = h + j;
        if (node_ok(e)) {
          const int g = bg + ofs(e) * NP;
          const double dg = 2.0 / sqrt(w4[j][0] + w4[j][1] + w4[j][2] + w4[j][3]);
          dh[g] = dg;
          dhf[g] = (float)dg;
          x[g] = 0.0;
          r[g] = P.h2;
          bb += P.h2 * P.h2;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // D^-1/2 of the neighbours
    // row sums of the scaled operator away from the boundary: the potential
    // shift of the preconditioner
    bases(bl, bg);
#pragma unroll
    for (int h = 0; h < E; h += 4) {
      double v9[4][9];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int o = ofs(h + j), l = bl + o * PP, g = bg + o * NP;
        v9[j][0] = dh[g];
        v9[j][1] = eh[l];
        v9[j][2] = dh[g + 1];
        v9[j][3] = eh[l - 1];
        v9[j][4] = dh[g - 1];
        v9[j][5] = ev[l];
        v9[j][6] = dh[g + NP];
        v9[j][7] = ev[l - PP];
        v9[j][8] = dh[g - NP];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 4 * qq + ofs(h + j);
        const double t = 4.0 - v9[j][0] * (v9[j][1] * v9[j][2] + v9[j][3] * v9[j][4] + v9[j][5] * v9[j][6] +
                                           v9[j][7] * v9[j][8]);
        rs += row >= 1 && row <= m - 2 && c >= 1 && c <= m - 2 ? t : 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    block_sum2<BLOCK>(bb, rs, red0);
    const float shift = potential_shift(rs, m);
    const double stop = rtol * rtol * bb;
    // z = M^-1 r into p (first direction), rz = r . M^-1 r.  The iteration
    // reads D^-1/2 rounded to float: the scaled residual and the new
    // direction both take these values, so M^-1 = D^-1/2 (L + cI)^-1 D^-1/2
    // stays symmetric.
    float rin[E], z[E];
    double rr_s = 0.0;
    bases(bl, bg);
#pragma unroll
    for (int h = 0; h < E; h += EH) {
      float dv[EH];
#pragma unroll
      for (int j = 0; j < EH; ++j) dv[j] = dhf[bg + ofs(h + j) * NP];
#pragma unroll
      for (int j = 0; j < EH; ++j) {
        const int e = h + j;
        const float df = node_ok(e) ? dv[j] : 0.0f;
        rin[e] = (float)((double)df * P.h2);
        rr_s += (double)rin[e] * (double)rin[e];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    rr_s = block_sum<BLOCK>(rr_s, red1);
    dst_apply_big<MP>(rin, pow2_scale(rr_s), z, sf, xa, xb, slam, shift);
    double rz = 0.0;
    bases(bl, bg);
#pragma unroll
    for (int h = 0; h < E; h += EH) {
      float dv[EH];
#pragma unroll
      for (int j = 0; j < EH; ++j) dv[j] = dhf[bg + ofs(h + j) * NP];
#pragma unroll
      for (int j = 0; j < EH; ++j) {
        const int e = h + j;
        if (node_ok(e)) p[bl + ofs(e) * PP] = (float)((double)dv[j] * (double)z[e]);
        rz += (double)rin[e] * (double)z[e];  // padding: rin = 0
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    rz = block_sum<BLOCK>(rz, red0);
    int it = 0;
    bool conv = !(bb > 0.0);
    // Per iteration the workspace sees the direction and both edge arrays
    // (A p, kept in registers: its live range ends before the preconditioner's
    // begins), the residual, then the iterate and the direction together: the
    // step x += alpha p is taken when p is read for the next direction (and
    // once more after the last iteration).
    double alpha = 0.0;
    while (!conv && it < maxit) {
      __syncthreads();  // every direction value is written
      double pq = 0.0, qa[E];
      bases(bl, bg);
      // A p by column groups of four rows (16 t + 4 qq + v, v = 0..3): their
      // north and south neighbours are the group's own values, so a group
      // takes 27 loads instead of 36
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int l0 = bl + 16 * t * PP;
        float pn[6], pe[4], pw[4];
        double eo[4], ew[4], eu[4];
#pragma unroll
        for (int v = 0; v < 6; ++v) pn[v] = p[l0 + (v - 1) * PP];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          pe[v] = p[l0 + v * PP + 1];
          pw[v] = p[l0 + v * PP - 1];
          eo[v] = eh[l0 + v * PP];
          ew[v] = eh[l0 + v * PP - 1];
          eu[v] = ev[l0 + v * PP];
        }
        const double es = ev[l0 - PP];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double pc = pn[v + 1];
          const double qv = eo[v] * (pc - (double)pe[v]) + ew[v] * (pc - (double)pw[v]) +
                            eu[v] * (pc - (double)pn[v + 2]) + (v > 0 ? eu[v - 1] : es) * (pc - (double)pn[v]);
          const bool ok = node_ok(4 * t + v);
          qa[4 * t + v] = ok ? qv : 0.0;
          pq += ok ? pc * qv : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      pq = block_sum<BLOCK>(pq, red1);
      alpha = rz / pq;
      double rr = 0.0;
      rr_s = 0.0;
      bases(bl, bg);
#pragma unroll
      for (int h = 0; h < E; h += EH) {
        double rv[EH];
        float dv[EH];
#pragma unroll
        for (int j = 0; j < EH; ++j) {
          const int g = bg + ofs(h + j) * NP;
          rv[j] = r[g];
          dv[j] = dhf[g];
        }
#pragma unroll
        for (int j = 0; j < EH; ++j) {
          const int e = h + j;
          const bool ok = node_ok(e);
          const double rg = rv[j] - alpha * qa[e];
          if (ok) r[bg + ofs(e) * NP] = rg;
          rr += ok ? rg * rg : 0.0;
          const float ri = ok ? (float)((double)dv[j] * rg) : 0.0f;
          rin[e] = ri;
          rr_s += (double)ri * (double)ri;
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      block_sum2<BLOCK>(rr, rr_s, red0);
      ++it;
      if (rr <= stop) {
        conv = true;
        break;
      }
      dst_apply_big<MP>(rin, pow2_scale(rr_s), z, sf, xa, xb, slam, shift);
      double rz2 = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) rz2 += (double)rin[e] * (double)z[e];  // r . M^-1 r (padding: rin = 0)
      rz2 = block_sum<BLOCK>(rz2, red1);
      const double beta = rz2 / rz;
      rz = rz2;
      bases(bl, bg);
#pragma unroll
      for (int h = 0; h < E; h += EH) {
        double xv[EH];
        float pv[EH], dv[EH];
#pragma unroll
        for (int j = 0; j < EH; ++j) {
          const int o = ofs(h + j), g = bg + o * NP;
          pv[j] = p[bl + o * PP];
          xv[j] = x[g];
          dv[j] = dhf[g];
        }
#pragma unroll
        for (int j = 0; j < EH; ++j) {
          const int e = h + j, o = ofs(e);
          if (node_ok(e)) {
            x[bg + o * NP] = xv[j] + alpha * (double)pv[j];
            p[bl + o * PP] = (float)((double)dv[j] * (double)z[e] + beta * (double)pv[j]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      alpha = 0.0;
    }
    // the last step (or none: alpha = 0 when the loop ended on maxit after a
    // full iteration, or never ran), each lane on its own nodes
    bases(bl, bg);
    int bo = 4 * qq * m + c;  // output node index base (row m + col)
    asm volatile("" : "+v"(bo));
#pragma unroll
    for (int h = 0; h < E; h += EH) {
      double xv[EH];
#pragma unroll
      for (int j = 0; j < EH; ++j) {
        const int o = ofs(h + j);
        xv[j] = x[bg + o * NP] + alpha * (double)p[bl + o * PP];
      }
#pragma unroll
      for (int j = 0; j < EH; ++j) {
        const int e = h + j;
        if (node_ok(e)) store_sample(out, out_fp32, (int64_t)(bo + ofs(e) * m) * ld + col0 + s, xv[j]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (threadIdx.x == 0 && iters) iters[s] = conv ? it : -1;
  }
}

// ------------------------------------------ even meshes 129 < mesh_n <= 256
// Beyond n = 129 the fast-Poisson preconditioner no longer fits a CU, so it
// moves to the mesh of width 2h: an additive two-level preconditioner on the
// scaled system, M^-1 = I / 4 + P (L_c + 4 c I)^-1 P^T, with P the bilinear
// interpolation from the coarse mesh (n / 2, at most 127 inner points per
// side) and L_c the unit 5-point Laplacian there, applied in LDS and registers
// by the same fp16 matrix-core DST transform as above (MP = 128).  P^T L P is
// close to L_c for smooth functions (the weights of P^T sum to 4 = (2h / h)^2),
// and 4 c carries the mean potential shift of the scaled operator to the
// coarse mesh.  The conjugate-gradient inner product splits as
// r.z = r.r / 4 + (P^T r).z_c, so both parts come from values a pass already
// holds.  Fine-mesh state streams from a per-workgroup workspace: seven slots
// of gp doubles, halo grids of kTlRows x kTlPitch with vertex (i, j) at
// j kTlPitch + i (x, r, A p, eh, ev in float64; the direction and the scaled
// residual, then D^-1/2, in float).  The grids are sized for the largest
// lane layout, so every pass loads without bounds branches; stores are
// guarded.  The coarse correction goes to LDS as a float vertex grid
// ((n / 2 + 1)^2, zero border) over the exchange tiles.
constexpr int kTlRows = 258, kTlPitch = 272;

int64_t tl_stream_pitch() { return ((int64_t)kTlRows * kTlPitch + 127) / 128 * 128; }

// the per-workgroup slots, then eight ticket counters
int64_t tl_stream_workspace_doubles(int blocks) { return tl_stream_pitch() * 7 * (int64_t)blocks + 8; }

bool tl_stream_ok(int n) { return n - 1 > kDstStreamMP && n <= 2 * kDstStreamMP && n % 2 == 0; }

__global__ __launch_bounds__(4 * kDstStreamMP) void pcgtl_stream_kernel(
    PdeDev P, const double* __restrict__ Y, int64_t ns, double rtol, int maxit, void* __restrict__ out, int out_fp32,
    int64_t ld, int64_t col0, int* __restrict__ iters, double* __restrict__ ws, int64_t gp,
    const half8* __restrict__ sfrag, const float* __restrict__ lamtab, unsigned long long* __restrict__ tick) {
  constexpr int MP = kDstStreamMP, NT = MP / 16, KB = MP / 32, E = 4 * NT, BLOCK = 4 * MP, LDX = MP + 4;
  constexpr int PF = kTlPitch;
  extern __shared__ double lds[];
  __shared__ double coef[kMaxD];
  __shared__ double red0[2 * (BLOCK / kWave)];
  __shared__ double red1[2 * (BLOCK / kWave)];
  __shared__ __attribute__((aligned(16))) float slam[MP];
  half8* sfl = reinterpret_cast<half8*>(lds);
  _Float16* xa = reinterpret_cast<_Float16*>(sfl + KB * NT * 64);
  _Float16* xb = xa + MP * LDX;
  float* zc = reinterpret_cast<float*>(xa);  // coarse correction, vertex (A, B) at B PC + A
  const int n = P.n, m = n - 1, nc = n / 2, mc = nc - 1, PC = nc + 1;
  double* x = ws + (size_t)blockIdx.x * 7 * gp;
  double* r = x + gp;
  double* q = r + gp;  // A p (before the first iteration: D^-1/2 in float64)
  double* eh = q + gp;
  double* ev = eh + gp;
  float* p = reinterpret_cast<float*>(ev + gp);
  float* rt = p + gp;                                   // scaled residual D^-1/2 r
  float* dhf = reinterpret_cast<float*>(ev + 2 * gp);  // D^-1/2 rounded to float
  const int lane = threadIdx.x & 63, qq = lane >> 4, c = 16 * (threadIdx.x >> 6) + (lane & 15);
  const int wv = threadIdx.x >> 6;
  for (int f = threadIdx.x; f < KB * NT * 64; f += BLOCK) sfl[f] = sfrag[f];
  for (int i = threadIdx.x; i < MP; i += BLOCK) slam[i] = lamtab[i];
  const FragLds sf{sfl, lane};
  auto ofs = [](int e) { return 16 * (e >> 2) + (e & 3); };
  // fine passes: wave wv takes rows wv, wv + 8, ..., a lane the columns
  // lane + 64 k (the passes of the iteration two rows per step); rows and
  // columns up to 255 stay inside the halo grids
  const int kc = (m + 63) / 64, tr = (m + 7) / 8;
  // the halo grids' borders (and entries of no mesh node) are never written
  // afterwards: cleared once per launch
  for (int e = threadIdx.x; e < kTlRows * PF; e += BLOCK) {
    p[e] = 0.0f;
    rt[e] = 0.0f;
  }
  // P^T rt for the lane's coarse nodes (column c, rows 4 qq + o(e)): the
  // 3 x 3 fine neighbourhood of fine vertex (2 (c + 1), 2 (row + 1)) with
  // weights 1, 1/2, 1/4; the sum of squares returned
  auto restrict_rt = [&](float (&rin)[E]) {
    constexpr int RH = 8;  // coarse nodes per load chunk
    double ss = 0.0;
    int bR = (8 * qq + 2) * PF + 2 * (c + 1);
    asm volatile("" : "+v"(bR));
#pragma unroll
    for (int h = 0; h < E; h += RH) {
      float v[RH][9];
#pragma unroll
      for (int j = 0; j < RH; ++j) {
        const int ci = bR + 2 * ofs(h + j) * PF;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
          for (int di = 0; di < 3; ++di) v[j][3 * dj + di] = rt[ci + (dj - 1) * PF + di - 1];
      }
#pragma unroll
      for (int j = 0; j < RH; ++j) {
        const int e = h + j;
        const bool ok = c < mc && 4 * qq + ofs(e) < mc;
        const float val = v[j][4] + 0.5f * (v[j][1] + v[j][3] + v[j][5] + v[j][7]) +
                          0.25f * (v[j][0] + v[j][2] + v[j][6] + v[j][8]);
        rin[e] = ok ? val : 0.0f;
        ss += (double)rin[e] * (double)rin[e];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    return ss;
  };
  // the coarse correction into the LDS vertex grid (after the transform is
  // done with the tiles), zero on the border
  auto coarse_grid = [&](const float (&z)[E]) {
    __syncthreads();
    for (int e = threadIdx.x; e < PC; e += BLOCK) {
      zc[e] = 0.0f;
      zc[e * PC] = 0.0f;
    }
    int bz = (4 * qq + 1) * PC + c + 1;
    asm volatile("" : "+v"(bz));
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int J = 4 * qq + ofs(e);
      if (c <= mc && J <= mc) zc[bz + ofs(e) * PC] = (c < mc && J < mc) ? z[e] : 0.0f;
    }
    __syncthreads();
  };
  // p = D^-1/2 (rt / 4 + P z_c) + beta p on the fine mesh
  auto direction = [&](double beta) {
#pragma unroll 1
    for (int t = 0; t < tr; t += 2) {
      float pv[8], rv[8], dv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int hf = (wv + 8 * (t + (u >> 2)) + 1) * PF + lane + 64 * (u & 3) + 1;
        pv[u] = p[hf];
        rv[u] = rt[hf];
        dv[u] = dhf[hf];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int i = lane + 64 * (k & 3), j = wv + 8 * (t + (k >> 2));
        if ((k & 3) < kc && i < m && j < m) {
          // bilinear weights 1 (on a coarse line) or 1/2, 1/2 (between two):
          // all four corners read (a + 1, b + 1 <= n / 2), weight 0 where unused
          const int iv = i + 1, jv = j + 1, a = iv >> 1, b = jv >> 1;
          const float wa1 = (iv & 1) ? 0.5f : 0.0f, wa0 = 1.0f - wa1;
          const float wb1 = (jv & 1) ? 0.5f : 0.0f, wb0 = 1.0f - wb1;
          const float* zr = zc + b * PC + a;
          const float pz = wb0 * (wa0 * zr[0] + wa1 * zr[1]) + wb1 * (wa0 * zr[PC] + wa1 * zr[PC + 1]);
          const float zt = 0.25f * rv[k] + pz;
          const double old = beta != 0.0 ? beta * (double)pv[k] : 0.0;  // the first direction ignores p
          p[(j + 1) * PF + iv] = (float)((double)dv[k] * (double)zt + old);
        }
      }
    }
  };
  const Tickets tk(tick, ns);
  __shared__ int64_t s_next;
  for (;;) {
    const int64_t s = tk.next(&s_next);  // the previous sample is done with coef and the workspace
    if (s >= tk.hi) break;
    load_coef(P, Y, s, coef);
    __syncthreads();
    // triangle values T_q[cj PF + ci] of eq. (1.2) (T_0 in the x slot, T_1 in
    // the r slot), as in pcgdst_stream_kernel, the row factors read from the
    // padded tables in global memory (a table of n + 16 rows per term would
    // not fit LDS beside the fragments for every d)
    {
      constexpr int RC = 16;
      const int S = row_tab_pitch(n);
      const int rpg = (n + 3) / 4;
      const int cj0 = __builtin_amdgcn_readfirstlane((threadIdx.x >> 7) * rpg);
      const int rows = min(rpg, n - cj0);
      const bool logn = P.model == USFFT_MODEL_LOGNORMAL;
#pragma unroll 1
      for (int qt = 0; qt < 2; ++qt) {
        double* T = qt == 0 ? x : r;
#pragma unroll 1
        for (int cb = 0; cb < n; cb += 128) {
          const int ci = min(cb + (int)(threadIdx.x & 127), n - 1);
          const bool cok = cb + (int)(threadIdx.x & 127) < n;
          const double* tx = P.tab + (size_t)qt * P.d * n + ci;
#pragma unroll 1
          for (int u0 = 0; u0 < rows; u0 += RC) {
            const double* ty = P.tab + (size_t)4 * P.d * n + (size_t)qt * P.d * S + 1 + cj0 + u0;
            double acc[RC];
#pragma unroll
            for (int u = 0; u < RC; ++u) acc[u] = logn ? 0.0 : P.a0;
#pragma unroll 1
            for (int k0 = 0; k0 < P.d; k0 += 8) {
              double t8[8];
#pragma unroll
              for (int kk = 0; kk < 8; ++kk) t8[kk] = tx[(size_t)min(k0 + kk, P.d - 1) * n];
#pragma unroll
              for (int kk = 0; kk < 8; ++kk) {
                if (k0 + kk < P.d) {
                  const double w = coef[k0 + kk] * t8[kk];
                  const double* tyk = ty + (size_t)(k0 + kk) * S;
#pragma unroll
                  for (int u = 0; u < RC; ++u) acc[u] += w * tyk[u];
                }
              }
            }
#pragma unroll
            for (int u = 0; u < RC; ++u)
              if (u0 + u < rows && cok) T[(cj0 + u0 + u) * PF + ci] = logn ? P.a0 + exp(acc[u]) : acc[u];
          }
        }
      }
    }
    __syncthreads();
    // edge weights at vertex index j PF + i, as in pcgdst_stream_kernel
    {
      const int rpg = (n + 3) / 4;
      const int j0 = (threadIdx.x >> 7) * rpg, j1 = min(j0 + rpg, n);
#pragma unroll 1
      for (int cb = 0; cb < n; cb += 128) {
        const int i = min(cb + (int)(threadIdx.x & 127), n - 1);
        const bool cok = cb + (int)(threadIdx.x & 127) < n;
        double t1b = j0 > 0 ? r[(j0 - 1) * PF + i] : 0.0;
#pragma unroll 1
        for (int jb = j0; jb < j1; jb += 8) {
          double a0[8], a1[8], aw[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = min(jb + u, n - 1);
            a0[u] = x[j * PF + i];
            a1[u] = r[j * PF + i];
            aw[u] = x[j * PF + max(i - 1, 0)];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = jb + u;
            if (j < j1 && cok) {
              if (j >= 1) eh[j * PF + i] = 0.5 * (a0[u] + t1b);
              if (i >= 1) ev[j * PF + i] = 0.5 * (a1[u] + aw[u]);
            }
            t1b = a1[u];
          }
        }
      }
    }
    __syncthreads();
    // D^-1/2 (float64 into the A p slot for the shift, float copy), x = 0,
    // r = b, the scaled residual
    double bb = 0.0, rtt = 0.0;
#pragma unroll 1
    for (int t = 0; t < tr; ++t) {
      const int j = wv + 8 * t;
      double w4[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int hf = (j + 1) * PF + lane + 64 * k + 1;
        w4[k][0] = eh[hf];
        w4[k][1] = eh[hf - 1];
        w4[k][2] = ev[hf];
        w4[k][3] = ev[hf - PF];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = lane + 64 * k;
        if (k < kc && i < m && j < m) {
          const int hf = (j + 1) * PF + i + 1;
          const double dg = 2.0 / sqrt(w4[k][0] + w4[k][1] + w4[k][2] + w4[k][3]);
          const float df = (float)dg;
          q[hf] = dg;
          dhf[hf] = df;
          x[hf] = 0.0;
          r[hf] = P.h2;
          const float rv = (float)((double)df * P.h2);
          rt[hf] = rv;
          bb += P.h2 * P.h2;
          rtt += (double)rv * (double)rv;
        }
      }
    }
    __syncthreads();  // D^-1/2 of the neighbours
    // row sums of the scaled operator away from the boundary: the potential
    // shift (as in the single-level solvers)
    double rs = 0.0;
#pragma unroll 1
    for (int t = 0; t < tr; ++t) {
      const int j = wv + 8 * t;
      double v9[4][9];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int hf = (j + 1) * PF + lane + 64 * k + 1;
        v9[k][0] = q[hf];
        v9[k][1] = eh[hf];
        v9[k][2] = q[hf + 1];
        v9[k][3] = eh[hf - 1];
        v9[k][4] = q[hf - 1];
        v9[k][5] = ev[hf];
        v9[k][6] = q[hf + PF];
        v9[k][7] = ev[hf - PF];
        v9[k][8] = q[hf - PF];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = lane + 64 * k;
        const double tv = 4.0 - v9[k][0] * (v9[k][1] * v9[k][2] + v9[k][3] * v9[k][4] + v9[k][5] * v9[k][6] +
                                            v9[k][7] * v9[k][8]);
        rs += k < kc && i >= 1 && i <= m - 2 && j >= 1 && j <= m - 2 ? tv : 0.0;
      }
    }
    block_sum2<BLOCK>(bb, rs, red0);
    rtt = block_sum<BLOCK>(rtt, red1);
    const float shift = 4.0f * potential_shift(rs, m);
    const double stop = rtol * rtol * bb;
    float rin[E], z[E];
    double rr_s = restrict_rt(rin);
    rr_s = block_sum<BLOCK>(rr_s, red0);
    dst_apply_big<MP>(rin, pow2_scale(rr_s), z, sf, xa, xb, slam, shift);
    double rzc = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) rzc += (double)rin[e] * (double)z[e];
    rzc = block_sum<BLOCK>(rzc, red1);
    double rz = 0.25 * rtt + rzc;
    coarse_grid(z);
    direction(0.0);
    int it = 0;
    bool conv = !(bb > 0.0);
    while (!conv && it < maxit) {
      __syncthreads();  // every direction value is written
      double pq = 0.0;
#pragma unroll 1
      for (int t = 0; t < tr; t += 2) {
        float pc[8], pe[8], pw[8], pn[8], ps[8];
        double eo[8], ew[8], eu[8], es[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int hf = (wv + 8 * (t + (k >> 2)) + 1) * PF + lane + 64 * (k & 3) + 1;
          pc[k] = p[hf];
          pe[k] = p[hf + 1];
          pw[k] = p[hf - 1];
          pn[k] = p[hf + PF];
          ps[k] = p[hf - PF];
          eo[k] = eh[hf];
          ew[k] = eh[hf - 1];
          eu[k] = ev[hf];
          es[k] = ev[hf - PF];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = lane + 64 * (k & 3), j = wv + 8 * (t + (k >> 2));
          const double c0 = pc[k];
          const double qv = eo[k] * (c0 - (double)pe[k]) + ew[k] * (c0 - (double)pw[k]) +
                            eu[k] * (c0 - (double)pn[k]) + es[k] * (c0 - (double)ps[k]);
          if ((k & 3) < kc && i < m && j < m) {
            q[(j + 1) * PF + i + 1] = qv;
            pq += c0 * qv;
          }
        }
      }
      pq = block_sum<BLOCK>(pq, red0);
      const double alpha = rz / pq;
      double rr = 0.0;
      rtt = 0.0;
#pragma unroll 1
      for (int t = 0; t < tr; t += 2) {
        double rv[8], qv[8], xv[8];
        float pv[8], dv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int hf = (wv + 8 * (t + (k >> 2)) + 1) * PF + lane + 64 * (k & 3) + 1;
          rv[k] = r[hf];
          qv[k] = q[hf];
          xv[k] = x[hf];
          pv[k] = p[hf];
          dv[k] = dhf[hf];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = lane + 64 * (k & 3), j = wv + 8 * (t + (k >> 2));
          if ((k & 3) < kc && i < m && j < m) {
            const int hf = (j + 1) * PF + i + 1;
            const double rg = rv[k] - alpha * qv[k];
            r[hf] = rg;
            x[hf] = xv[k] + alpha * (double)pv[k];
            const float rs1 = (float)((double)dv[k] * rg);
            rt[hf] = rs1;
            rr += rg * rg;
            rtt += (double)rs1 * (double)rs1;
          }
        }
      }
      block_sum2<BLOCK>(rr, rtt, red1);
      ++it;
      if (rr <= stop) {
        conv = true;
        break;
      }
      rr_s = restrict_rt(rin);  // the barrier of block_sum2 ordered the rt writes
      rr_s = block_sum<BLOCK>(rr_s, red0);
      dst_apply_big<MP>(rin, pow2_scale(rr_s), z, sf, xa, xb, slam, shift);
      rzc = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) rzc += (double)rin[e] * (double)z[e];
      rzc = block_sum<BLOCK>(rzc, red1);
      const double rz2 = 0.25 * rtt + rzc;
      const double beta = rz2 / rz;
      rz = rz2;
      coarse_grid(z);
      direction(beta);
    }
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < tr; ++t) {
      const int j = wv + 8 * t;
      double xv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) xv[k] = x[(j + 1) * PF + lane + 64 * k + 1];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = lane + 64 * k;
        if (k < kc && i < m && j < m) store_sample(out, out_fp32, (int64_t)(j * m + i) * ld + col0 + s, xv[k]);
      }
    }
    if (threadIdx.x == 0 && iters) iters[s] = conv ? it : -1;
  }
}

int tl_stream_blocks() {
  int cus = 0, dev = 0, per_cu = 0;
  USFFT_HIP(hipGetDevice(&dev));
  USFFT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  USFFT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(pcgtl_stream_kernel),
                                                         4 * kDstStreamMP, (size_t)dst_stream_lds_bytes()));
  return std::max(1, per_cu) * std::max(1, cus);
}

void launch_pde_solve_tl_stream(const PdeDev& P, const double* Y, int64_t ns, double rtol, int maxit, void* out,
                                int out_fp32, int64_t ld, int64_t col0, int* iters, double* ws, int blocks,
                                const void* frag, const float* lam, hipStream_t st) {
  if (ns <= 0) return;
  USFFT_REQUIRE(tl_stream_ok(P.n), USFFT_EINVAL, "mesh outside the two-level streaming solver's range");
  const unsigned grid = (unsigned)std::min<int64_t>(ns, blocks);
  unsigned long long* tick = reinterpret_cast<unsigned long long*>(ws + tl_stream_workspace_doubles(blocks) - 8);
  hipLaunchKernelGGL(zero_u64x8_kernel, dim3(1), dim3(8), 0, st, tick);
  hipLaunchKernelGGL(pcgtl_stream_kernel, dim3(grid), dim3(4 * kDstStreamMP), (size_t)dst_stream_lds_bytes(), st,
                     P, Y, ns, rtol, maxit, out, out_fp32, ld, col0, iters, ws, tl_stream_pitch(),
                     static_cast<const half8*>(frag), lam, tick);
  USFFT_HIP(hipGetLastError());
}

bool dst_stream_ok(int n) { return n - 1 > 64 && n - 1 <= kDstStreamMP; }

int dst_stream_blocks() {
  int cus = 0, dev = 0, per_cu = 0;
  USFFT_HIP(hipGetDevice(&dev));
  USFFT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  USFFT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(pcgdst_stream_kernel),
                                                         4 * kDstStreamMP, (size_t)dst_stream_lds_bytes()));
  return std::max(1, per_cu) * std::max(1, cus);
}

void dst_stream_tables_build(int n, void* frag, float* lam, hipStream_t st) {
  const int mp = kDstStreamMP;
  const int cnt = (mp / 32) * (mp / 16) * 64;
  hipLaunchKernelGGL(dst_tables_kernel, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, n, mp,
                     static_cast<half8*>(frag), lam);
  USFFT_HIP(hipGetLastError());
}

void launch_pde_solve_dst_stream(const PdeDev& P, const double* Y, int64_t ns, double rtol, int maxit, void* out,
                                 int out_fp32, int64_t ld, int64_t col0, int* iters, double* ws, int blocks,
                                 const void* frag, const float* lam, hipStream_t st) {
  if (ns <= 0) return;
  USFFT_REQUIRE(dst_stream_ok(P.n), USFFT_EINVAL, "mesh outside the streaming DST solver's range");
  const unsigned grid = (unsigned)std::min<int64_t>(ns, blocks);
  unsigned long long* tick =
      reinterpret_cast<unsigned long long*>(ws + dst_stream_workspace_doubles(P.n, blocks) - 8);
  hipLaunchKernelGGL(zero_u64x8_kernel, dim3(1), dim3(8), 0, st, tick);
  hipLaunchKernelGGL(pcgdst_stream_kernel, dim3(grid), dim3(4 * kDstStreamMP), (size_t)dst_stream_lds_bytes(), st,
                     P, Y, ns, rtol, maxit, out, out_fp32, ld, col0, iters, ws, dst_stream_pitch(P.n),
                     static_cast<const half8*>(frag), lam, tick);
  USFFT_HIP(hipGetLastError());
}

static int dst_occupancy_of(const void* kernel, int mp, int64_t lds) {
  int per_cu = 0;
  USFFT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 4 * mp, (size_t)lds));
  return std::max(1, per_cu);
}

template <typename T, int MP, bool LR>
static int dst_occupancy(int n) {
  return dst_occupancy_of(reinterpret_cast<const void*>(pcgdst_kernel<T, MP, LR>), MP,
                          dst_lds_bytes(n, std::is_same<T, float>::value ? USFFT_FP32_REFINE : USFFT_FP64, LR ? 1 : 0));
}

int dst_persistent_blocks(int n, int precision, int variant) {
  static int cache[2][2][3] = {};  // [float32?][mp == 64?][variant]
  const int mp = dst_padded(n);
  const int a = precision == USFFT_FP64 ? 0 : 1, b = mp == 64 ? 1 : 0, c = variant;
  USFFT_REQUIRE(c >= 0 && c <= 2 && !(c == 2 && a == 0), USFFT_EINVAL, "bad DST solver variant");
  if (cache[a][b][c] == 0) {
    int cus = 0, dev = 0;
    USFFT_HIP(hipGetDevice(&dev));
    USFFT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 1;
#define USFFT_OCC(TT, MM, LL) per_cu = dst_occupancy<TT, MM, LL>(n)
    if (c == 2) {
      const int64_t lds = dst_lds_bytes(n, precision, 2);
      per_cu = b ? dst_occupancy_of(reinterpret_cast<const void*>(pcgdst32c_kernel<64>), 64, lds)
                 : dst_occupancy_of(reinterpret_cast<const void*>(pcgdst32c_kernel<32>), 32, lds);
    } else if (a == 0) {
      if (b) { if (c) USFFT_OCC(double, 64, true); else USFFT_OCC(double, 64, false); }
      else { if (c) USFFT_OCC(double, 32, true); else USFFT_OCC(double, 32, false); }
    } else {
      if (b) { if (c) USFFT_OCC(float, 64, true); else USFFT_OCC(float, 64, false); }
      else { if (c) USFFT_OCC(float, 32, true); else USFFT_OCC(float, 32, false); }
    }
#undef USFFT_OCC
    cache[a][b][c] = per_cu * std::max(1, cus);
  }
  return cache[a][b][c];
}

int64_t dst_scratch_doubles(int n, int variant, int blocks) {
  // the edge slots (none in variant 1), then eight ticket counters
  return (variant == 1 ? 0 : (variant == 2 ? 2 : 3) * dst_edge_stride(dst_padded(n)) * (int64_t)blocks) + 8;
}

void launch_pde_solve_dst(const SolveSeg* segs, int nseg, int n, int precision, int variant, int64_t ns,
                          double rtol, int maxit, double inner_rtol, int refine_every, int out_fp32, double* wscr,
                          int wblocks, const void* frag, const float* lam, hipStream_t st) {
  if (ns <= 0) return;
  const int mp = dst_padded(n);
  USFFT_REQUIRE(mp > 0, USFFT_EINVAL, "mesh too large for the DST-preconditioned solver");
  USFFT_REQUIRE(nseg >= 1, USFFT_EINVAL, "no solver segment");
  USFFT_REQUIRE(variant == 0 || variant == 1 || (variant == 2 && precision != USFFT_FP64), USFFT_EINVAL,
                "bad DST solver variant");
  const int64_t ws = dst_edge_stride(mp);
  const unsigned grid = (unsigned)std::min<int64_t>(ns, wblocks);
  const size_t lds = (size_t)dst_lds_bytes(n, precision, variant);
  const half8* sf = static_cast<const half8*>(frag);
#define USFFT_DST(TT, MM, LL)                                                                                  \
  hipLaunchKernelGGL((pcgdst_kernel<TT, MM, LL>), dim3(grid), dim3(4 * MM), lds, st, segs, nseg, ns, rtol, maxit, \
                     inner_rtol, refine_every, out_fp32, wscr, ws, sf, lam, tick)
  unsigned long long* tick = reinterpret_cast<unsigned long long*>(
      wscr + (variant == 1 ? 0 : (variant == 2 ? 2 : 3) * ws * (int64_t)wblocks));
  hipLaunchKernelGGL(zero_u64x8_kernel, dim3(1), dim3(8), 0, st, tick);
  if (variant == 2) {
    if (mp == 64)
      hipLaunchKernelGGL(pcgdst32c_kernel<64>, dim3(grid), dim3(256), lds, st, segs, nseg, ns, rtol, maxit,
                         inner_rtol, refine_every, out_fp32, wscr, ws, sf, lam, tick);
    else
      hipLaunchKernelGGL(pcgdst32c_kernel<32>, dim3(grid), dim3(128), lds, st, segs, nseg, ns, rtol, maxit,
                         inner_rtol, refine_every, out_fp32, wscr, ws, sf, lam, tick);
  } else if (precision == USFFT_FP64) {
    if (mp == 64) { if (variant) USFFT_DST(double, 64, true); else USFFT_DST(double, 64, false); }
    else { if (variant) USFFT_DST(double, 32, true); else USFFT_DST(double, 32, false); }
  } else {
    if (mp == 64) { if (variant) USFFT_DST(float, 64, true); else USFFT_DST(float, 64, false); }
    else { if (variant) USFFT_DST(float, 32, true); else USFFT_DST(float, 32, false); }
  }
#undef USFFT_DST
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
