// Lattice DFTs of the usFFT on gfx950 (Alg. 1 step 1&2a and Algorithm A, App. A).
//
// Lattice DFT.  Sampling along a rank-1 lattice of prime size M turns the
// coefficient of candidate k into bin k.z mod M of a length-M DFT.  Every
// node needs that DFT, at the bins of the candidates assigned to the
// lattice.  For prime M, Rader's algorithm (C. M. Rader, Proc. IEEE 1968)
// writes X[g^-p] - x[0] as the cyclic convolution of a_q = x[g^q] with
// b_j = exp(-2 pi i g^-j / M), q, j < L = M-1, g a generator mod M.  Lattice
// sizes are restricted to primes with 7-smooth L, so the convolution is two
// mixed-radix FFTs of length L plus one pointwise product with the
// precomputed spectrum of b.  One workgroup handles two nodes (two real
// columns packed as one complex column), keeps the whole length-L transform in
// LDS (L <= 9600 complex doubles = 150 KB), reads its two sample rows once,
// coalesced, and writes only the requested bins: HBM traffic is the
// algorithmic minimum, M reads and n_bins writes per node.
//
// FFT in LDS: in-place mixed-radix decimation-in-frequency stages forward and
// decimation-in-time stages back, with the convolution's pointwise product in
// the digit-reversed order in between (no reordering pass, one LDS buffer,
// R registers per butterfly).
//
// Line DFT: the length-K_t DFT of the 1-D detection, evaluated directly.
#include "kernels.h"

#include <cmath>
#include <vector>

namespace usfft {

constexpr int kLMax = kMaxLattice - 1;  // 19200 (float32; float64 stops at 9600)
constexpr int kFftBlock = 512;

// correctly rounded cos / sin of 2 pi m / R
template <int R>
struct RootTab;
template <>
struct RootTab<3> {
  static constexpr double c[3] = {1.0, -0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.8660254037844386, -0.8660254037844386};
};
template <>
struct RootTab<5> {
  static constexpr double c[5] = {1.0, 0.30901699437494745, -0.8090169943749475, -0.8090169943749475,
                                  0.30901699437494745};
  static constexpr double s[5] = {0.0, 0.9510565162951535, 0.5877852522924731, -0.5877852522924731,
                                  -0.9510565162951535};
};
template <>
struct RootTab<7> {
  static constexpr double c[7] = {1.0, 0.6234898018587335, -0.2225209339563144, -0.9009688679024191,
                                  -0.9009688679024191, -0.2225209339563144, 0.6234898018587335};
  static constexpr double s[7] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.4338837391175581,
                                  -0.4338837391175581, -0.9749279121818236, -0.7818314824680298};
};

template <>
struct RootTab<9> {
  static constexpr double c[9] = {1.0, 0.766044443118978, 0.17364817766693036, -0.5, -0.9396926207859084, -0.9396926207859084, -0.5, 0.17364817766693036, 0.766044443118978};
  static constexpr double s[9] = {0.0, 0.6427876096865394, 0.984807753012208, 0.8660254037844386, 0.3420201433256687, -0.3420201433256687, -0.8660254037844386, -0.984807753012208, -0.6427876096865394};
};
template <>
struct RootTab<16> {
  static constexpr double c[16] = {1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898, 0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867};
  static constexpr double s[16] = {0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867, 1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898};
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) { return {a.y, -a.x}; }  // * (-i)
template <typename T>
__device__ __forceinline__ cplx<T> conjc(cplx<T> a) { return {a.x, -a.y}; }

template <typename T>
__device__ __forceinline__ void dft4(cplx<T>& a0, cplx<T>& a1, cplx<T>& a2, cplx<T>& a3) {
  const cplx<T> s02 = cadd(a0, a2), d02 = csub(a0, a2), s13 = cadd(a1, a3), d13 = mul_mi(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T>* v);

// forward DFT of length R = R1 R2 in registers (two register-level stages):
// with n = n1 + R1 n2 and k = k2 + R2 k1,
//   X_k = sum_n1 w_R1^(n1 k1) w_R^(n1 k2) sum_n2 v_(n1 + R1 n2) w_R2^(n2 k2)
template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_comp(cplx<T>* v) {
  constexpr int R = R1 * R2;
  cplx<T> y[R1][R2];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    cplx<T> t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = v[n1 + R1 * n2];
    dft_small<T, R2>(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1][k2] = t[k2];
  }
#pragma unroll
  for (int n1 = 1; n1 < R1; ++n1)
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) {
      const int m = (n1 * k2) % R;
      const cplx<T> a = y[n1][k2];
      if (R % 4 == 0 && m == R / 4) {
        y[n1][k2] = mul_mi(a);
      } else if (R % 2 == 0 && m == R / 2) {
        y[n1][k2] = {-a.x, -a.y};
      } else if (R % 4 == 0 && m == 3 * R / 4) {
        y[n1][k2] = {-a.y, a.x};
      } else {
        const T c = (T)RootTab<R>::c[m], sn = (T)RootTab<R>::s[m];
        y[n1][k2] = {a.x * c + a.y * sn, a.y * c - a.x * sn};  // a exp(-2 pi i m / R)
      }
    }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    cplx<T> t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = y[n1][k2];
    dft_small<T, R1>(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = t[k1];
  }
}

// forward DFT of length R on v[0..R), in place
template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T>* v) {
  if constexpr (R == 2) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 9) {
    dft_comp<T, 3, 3>(v);
  } else if constexpr (R == 16) {
    dft_comp<T, 4, 4>(v);
  } else if constexpr (R == 8) {
    constexpr T h = (T)0.7071067811865476;
    cplx<T> b[4], c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      b[j] = cadd(v[j], v[j + 4]);
      c[j] = csub(v[j], v[j + 4]);
    }
    c[1] = {h * (c[1].x + c[1].y), h * (c[1].y - c[1].x)};   // * exp(-i pi/4)
    c[2] = mul_mi(c[2]);                                       // * exp(-i pi/2)
    c[3] = {h * (c[3].y - c[3].x), -h * (c[3].x + c[3].y)};  // * exp(-3 i pi/4)
    dft4(b[0], b[1], b[2], b[3]);
    dft4(c[0], c[1], c[2], c[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = b[k];
      v[2 * k + 1] = c[k];
    }
  } else {
    // odd R in symmetric pairs: with s_q = v_q + v_{R-q}, d_q = v_q - v_{R-q}
    // and t = 2 pi p q / R,  X_p = a_p - i b_p,  X_{R-p} = a_p + i b_p,
    // a_p = v_0 + sum_q s_q cos t,  b_p = sum_q d_q sin t  (q, p <= (R-1)/2)
    constexpr int H = (R - 1) / 2;
    cplx<T> sp[H], dm[H];
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      sp[q - 1] = cadd(v[q], v[R - q]);
      dm[q - 1] = csub(v[q], v[R - q]);
    }
    cplx<T> o[R];
    o[0] = v[0];
#pragma unroll
    for (int q = 0; q < H; ++q) o[0] = cadd(o[0], sp[q]);
#pragma unroll
    for (int p = 1; p <= H; ++p) {
      cplx<T> a = v[0], b = {(T)0, (T)0};
#pragma unroll
      for (int q = 1; q <= H; ++q) {
        const int m = (p * q) % R;
        const T c = (T)RootTab<R>::c[m], sn = (T)RootTab<R>::s[m];
        a.x += sp[q - 1].x * c;
        a.y += sp[q - 1].y * c;
        b.x += dm[q - 1].x * sn;
        b.y += dm[q - 1].y * sn;
      }
      o[p] = {a.x + b.y, a.y - b.x};
      o[R - p] = {a.x - b.y, a.y + b.x};
    }
#pragma unroll
    for (int p = 0; p < R; ++p) v[p] = o[p];
  }
}


// In-place mixed-radix FFT stages on buf[0..L) (no extra buffer, R registers
// per butterfly).  Stage s has block size N_s = L / (R_0 ... R_{s-1}) and
// M_s = N_s / R_s; butterfly (blk, j) touches base + m M_s, base = blk N_s + j.
//  DIF stage: butterfly over m, then twiddle w_{N_s}^{j q}; running all
//    stages forward turns natural order into digit-reversed order, A = Pi F x.
//  DIT stage: twiddle first, then butterfly (the transpose of a DIF stage);
//    running the stages backwards on Pi y gives F y, because F is symmetric
//    and so F = S_0^T ... S_{S-1}^T Pi.
// A convolution therefore never needs natural order in between: forward DIF,
// pointwise product with a spectrum produced by the same DIF, DIT back.
// COLS transforms of length L side by side (column c at buf + c L): a
// butterfly loads its twiddles and spectrum values once for all columns.
// tw[0] = 1 exactly, so butterflies with j = 0 read their unit twiddles from
// the table like the others (no branch around the loads).
// b / M for 0 <= b < 2^15: the float quotient with the hardware reciprocal is
// within 0.01 of b / M, so its truncation is off by at most one, which the
// remainder corrects
__device__ __forceinline__ int div_small(int b, int M, float rM) {
  const int q = (int)((float)b * rM);
  const int r = b - q * M;
  return r < 0 ? q - 1 : (r >= M ? q + 1 : q);
}

template <typename T, int R, int BLOCK, int COLS, bool MB>
__device__ void dif_stage(cplx<T>* buf, int L, int N, int M, const cplx<T>* __restrict__ tw,
                          const cplx<T>* __restrict__ mulB) {
  const int nb = L / R;
  const float rM = __builtin_amdgcn_rcpf((float)M);
  for (int b = threadIdx.x; b < nb; b += BLOCK) {
    const int blk = div_small(b, M, rM), j = b - blk * M, base = blk * N + j;
    // this butterfly's R - 1 twiddles, contiguous in the stage's table
    const cplx<T>* twj = tw + j * (R - 1);
    // twiddles held for all columns, except the float64 radices above 8
    // (their registers would not fit), which read each one where it is used
    constexpr bool WREG = sizeof(T) == 4 || R <= 8;
    cplx<T> w[R], bq[R];
    if constexpr (WREG) {
#pragma unroll
      for (int q = 1; q < R; ++q) w[q] = twj[q - 1];
    }
    if constexpr (MB) {
#pragma unroll
      for (int q = 0; q < R; ++q) bq[q] = mulB[base + q * M];
    }
    // one column at a time: a radix-16 butterfly holds 16 values and 15
    // twiddles, and unrolled columns would multiply the former
#pragma unroll 1
    for (int c = 0; c < COLS; ++c) {
      cplx<T>* bc = buf + c * L;
      cplx<T> v[R];
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = bc[base + m * M];
      dft_small<T, R>(v);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        cplx<T> o = v[q];
        if (q > 0) o = cmul(o, WREG ? w[q] : twj[q - 1]);
        if constexpr (MB) o = conjc(cmul(o, bq[q]));
        bc[base + q * M] = o;
      }
    }
  }
  __syncthreads();
}

template <typename T, int R, int BLOCK, int COLS>
__device__ void dit_stage(cplx<T>* buf, int L, int N, int M, const cplx<T>* __restrict__ tw) {
  const int nb = L / R;
  const float rM = __builtin_amdgcn_rcpf((float)M);
  for (int b = threadIdx.x; b < nb; b += BLOCK) {
    const int blk = div_small(b, M, rM), j = b - blk * M, base = blk * N + j;
    const cplx<T>* twj = tw + j * (R - 1);       // as in dif_stage
    constexpr bool WREG = sizeof(T) == 4 || R <= 8;  // as in dif_stage
    cplx<T> w[R];
    if constexpr (WREG) {
#pragma unroll
      for (int q = 1; q < R; ++q) w[q] = twj[q - 1];
    }
#pragma unroll 1
    for (int c = 0; c < COLS; ++c) {
      cplx<T>* bc = buf + c * L;
      cplx<T> v[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        cplx<T> a = bc[base + q * M];
        if (q > 0) a = cmul(a, WREG ? w[q] : twj[q - 1]);
        v[q] = a;
      }
      dft_small<T, R>(v);
#pragma unroll
      for (int m = 0; m < R; ++m) bc[base + m * M] = v[m];
    }
  }
  __syncthreads();
}

// WIDE instantiations include the radix-9 and radix-16 stages of the float32
// plans (the float64 transforms, whose plans have none, leave their registers
// out).
// Forward DIF over all stages; with mulB, the last stage multiplies by mulB
// and conjugates (the forward half of a convolution, set up for the inverse
// transform by conjugation).
template <typename T, int BLOCK, int COLS, bool WIDE = sizeof(T) == 4>
__device__ void fft_dif(cplx<T>* buf, const FftPlanDev& F, const cplx<T>* tw, const cplx<T>* mulB) {
  int N = F.L;
  for (int s = 0; s < F.nrad; ++s) {
    const int R = F.radix[s], M = N / R;
    // the spectrum product is compiled only into the last stage
    if (s == F.nrad - 1 && mulB) {
      switch (R) {
        case 2: dif_stage<T, 2, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
        case 3: dif_stage<T, 3, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
        case 4: dif_stage<T, 4, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
        case 5: dif_stage<T, 5, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
        case 7: dif_stage<T, 7, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
        case 9: if constexpr (WIDE) dif_stage<T, 9, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
        case 16: if constexpr (WIDE) dif_stage<T, 16, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
        default: dif_stage<T, 8, BLOCK, COLS, true>(buf, F.L, N, M, tw + F.twoff[s], mulB); break;
      }
    } else {
      switch (R) {
        case 2: dif_stage<T, 2, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
        case 3: dif_stage<T, 3, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
        case 4: dif_stage<T, 4, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
        case 5: dif_stage<T, 5, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
        case 7: dif_stage<T, 7, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
        case 9: if constexpr (WIDE) dif_stage<T, 9, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
        case 16: if constexpr (WIDE) dif_stage<T, 16, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
        default: dif_stage<T, 8, BLOCK, COLS, false>(buf, F.L, N, M, tw + F.twoff[s], nullptr); break;
      }
    }
    N = M;
  }
}

// Forward DIT over all stages in reverse order (digit-reversed in, natural out).
template <typename T, int BLOCK, int COLS, bool WIDE = sizeof(T) == 4>
__device__ void fft_dit(cplx<T>* buf, const FftPlanDev& F, const cplx<T>* tw) {
  int Ns[24];
  int N = F.L;
  for (int s = 0; s < F.nrad; ++s) {
    Ns[s] = N;
    N /= F.radix[s];
  }
  for (int s = F.nrad - 1; s >= 0; --s) {
    const int R = F.radix[s], Nn = Ns[s], M = Nn / R;
    switch (R) {
      case 2: dit_stage<T, 2, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
      case 3: dit_stage<T, 3, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
      case 4: dit_stage<T, 4, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
      case 5: dit_stage<T, 5, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
      case 7: dit_stage<T, 7, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
      case 9: if constexpr (WIDE) dit_stage<T, 9, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
      case 16: if constexpr (WIDE) dit_stage<T, 16, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
      default: dit_stage<T, 8, BLOCK, COLS>(buf, F.L, Nn, M, tw + F.twoff[s]); break;
    }
  }
}

// ---------------------------------------------------------------- setup
// B = DFT_L(b) / L for b_j = exp(-2 pi i gen^-j / M), gen^-j = perm[(L - j) % L],
// stored in the digit-reversed order the forward DIF produces.
// The transform runs in LDS when its L float64 values fit, else in place in
// B64 (global memory; setup only).
__global__ __launch_bounds__(kFftBlock) void rader_setup_kernel(FftPlanDev F, int M, const int32_t* __restrict__ perm,
                                                               const cplx<double>* __restrict__ tw,
                                                               cplx<double>* __restrict__ B64,
                                                               cplx<float>* __restrict__ B32, int in_lds) {
  extern __shared__ char smem[];
  cplx<double>* buf = in_lds ? reinterpret_cast<cplx<double>*>(smem) : B64;
  const int L = F.L;
  for (int j = threadIdx.x; j < L; j += kFftBlock) {
    const int e = perm[(L - j) % L];
    double s, c;
    sincospi(-2.0 * (double)e / (double)M, &s, &c);
    buf[j] = {c, s};
  }
  __syncthreads();
  fft_dif<double, kFftBlock, 1, true>(buf, F, tw, nullptr);  // spectrum in the DIF (digit-reversed) order
  const double invL = 1.0 / (double)L;
  for (int k = threadIdx.x; k < L; k += kFftBlock) {
    const cplx<double> v = {buf[k].x * invL, buf[k].y * invL};
    B64[k] = v;
    B32[k] = {(float)v.x, (float)v.y};
  }
}

bool lattice_size_ok(int M) {
  if (M < 3 || M > kMaxLattice) return false;
  for (int f = 2; (int64_t)f * f <= M; ++f)
    if (M % f == 0) return false;
  int r = M - 1;
  for (int p : {2, 3, 5, 7})
    while (r % p == 0) r /= p;
  return r == 1;
}

static int64_t powmod(int64_t a, int64_t e, int64_t m) {
  int64_t r = 1 % m;
  a %= m;
  while (e > 0) {
    if (e & 1) r = r * a % m;
    a = a * a % m;
    e >>= 1;
  }
  return r;
}

// Byte offsets of the tables of one size inside its memory block.
namespace {
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
struct RaderLayout {
  size_t perm, outidx, dlog, tw64, tw32, B64, B32, total;
  explicit RaderLayout(int M) {
    const size_t L = (size_t)(M - 1);
    size_t o = 0;
    perm = o;
    o += align256(sizeof(int32_t) * L);
    outidx = o;
    o += align256(sizeof(int32_t) * M);
    dlog = o;
    o += align256(sizeof(int32_t) * M);
    tw64 = o;  // stage twiddles: fewer than 2 L per precision
    o += align256(sizeof(cplx<double>) * 2 * L);
    tw32 = o;
    o += align256(sizeof(cplx<float>) * 2 * L);
    B64 = o;
    o += align256(sizeof(cplx<double>) * L);
    B32 = o;
    o += align256(sizeof(cplx<float>) * L);
    total = o;
  }
};
}  // namespace

size_t rader_table_bytes(int M) { return RaderLayout(M).total; }

void rader_free(RaderTables& T) {
  if (T.owned && T.base) (void)hipFree(T.base);
  T = RaderTables{};
}

void rader_build(RaderTables& T, int M, bool wide, hipStream_t st) {
  USFFT_REQUIRE(lattice_size_ok(M), USFFT_EINVAL,
                "lattice size " + std::to_string(M) + " is not a prime <= 19201 with 7-smooth M-1");
  void* mem = nullptr;
  USFFT_HIP(hipMalloc(&mem, rader_table_bytes(M)));
  try {
    rader_build_at(T, M, wide, mem, st);
  } catch (...) {
    (void)hipFree(mem);
    throw;
  }
  T.owned = true;
}

void rader_build_at(RaderTables& T, int M, bool wide, void* mem, hipStream_t st) {
  USFFT_REQUIRE(lattice_size_ok(M), USFFT_EINVAL,
                "lattice size " + std::to_string(M) + " is not a prime <= 19201 with 7-smooth M-1");
  const RaderLayout Lay(M);
  char* base = static_cast<char*>(mem);
  T = RaderTables{};
  T.base = mem;
  T.owned = false;
  T.M = M;
  T.L = M - 1;
  const int L = T.L;
  // generator: g^(L/p) != 1 for every prime p | L
  int gen = 2;
  for (;; ++gen) {
    bool ok = true;
    for (int p : {2, 3, 5, 7})
      if (L % p == 0 && powmod(gen, L / p, M) == 1) ok = false;
    if (ok) break;
  }
  T.gen = gen;
  // radix plan, fewest stages: the 2^c2 factor in ceil(c2 / e) stages of
  // radix 2^e or less (the exponent spread evenly), e = 4 for wide plans and
  // 3 otherwise, then (wide) 9s and a 3, or 3s, then 5s and 7s (radices 9
  // and 16 run two levels in registers)
  int r = L, c2 = 0;
  while (r % 2 == 0) {
    r /= 2;
    ++c2;
  }
  T.nrad = 0;
  const int e2 = wide ? 4 : 3;
  for (int ns2 = (c2 + e2 - 1) / e2, left = c2; ns2 > 0; --ns2) {
    const int e = (left + ns2 - 1) / ns2;
    T.radix[T.nrad++] = 1 << e;
    left -= e;
  }
  {
    int c = 0;
    while (r % 3 == 0) {
      r /= 3;
      ++c;
    }
    if (wide)
      for (; c >= 2; c -= 2) T.radix[T.nrad++] = 9;
    for (; c >= 1; --c) T.radix[T.nrad++] = 3;
  }
  while (r % 5 == 0) {
    T.radix[T.nrad++] = 5;
    r /= 5;
  }
  while (r % 7 == 0) {
    T.radix[T.nrad++] = 7;
    r /= 7;
  }
  std::vector<int32_t> perm(L), dlog(M, -1), outidx(M, 0);
  int64_t v = 1;
  for (int q = 0; q < L; ++q) {
    perm[q] = (int32_t)v;
    dlog[v] = q;
    v = v * gen % M;
  }
  for (int b = 1; b < M; ++b) outidx[b] = (L - dlog[b]) % L;
  dlog[0] = 0;  // unused: x[0] enters only the sums
  std::vector<cplx<double>> tw(L);
  for (int k = 0; k < L; ++k) {
    const double a = -2.0 * M_PI * (double)k / (double)L;
    tw[k] = {std::cos(a), std::sin(a)};
  }
  // stage twiddles of the radix plan (the forward DIF stages and, in
  // reverse, the DIT stages use the same factors)
  std::vector<cplx<double>> st64;
  {
    int N = L;
    for (int s = 0; s < T.nrad; ++s) {
      const int R = T.radix[s], Ms = N / R, ts = L / N;
      T.twoff[s] = (int)st64.size();
      for (int j = 0; j < Ms; ++j)
        for (int q = 1; q < R; ++q) st64.push_back(tw[(size_t)j * q * ts]);
      N = Ms;
    }
  }
  USFFT_REQUIRE(st64.size() <= 2 * (size_t)L, USFFT_EINVAL, "stage twiddle table overflow");
  std::vector<cplx<float>> st32(st64.size());
  for (size_t k = 0; k < st64.size(); ++k) st32[k] = {(float)st64[k].x, (float)st64[k].y};
  T.perm = reinterpret_cast<int32_t*>(base + Lay.perm);
  T.outidx = reinterpret_cast<int32_t*>(base + Lay.outidx);
  T.dlog = reinterpret_cast<int32_t*>(base + Lay.dlog);
  T.tw64 = base + Lay.tw64;
  T.tw32 = base + Lay.tw32;
  T.B64 = base + Lay.B64;
  T.B32 = base + Lay.B32;
  USFFT_HIP(hipMemcpyAsync(T.perm, perm.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, st));
  USFFT_HIP(hipMemcpyAsync(T.outidx, outidx.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, st));
  USFFT_HIP(hipMemcpyAsync(T.dlog, dlog.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, st));
  USFFT_HIP(hipMemcpyAsync(T.tw64, st64.data(), sizeof(cplx<double>) * st64.size(), hipMemcpyHostToDevice, st));
  USFFT_HIP(hipMemcpyAsync(T.tw32, st32.data(), sizeof(cplx<float>) * st32.size(), hipMemcpyHostToDevice, st));
  FftPlanDev F;
  F.L = L;
  F.nrad = T.nrad;
  for (int i = 0; i < 24; ++i) {
    F.radix[i] = T.radix[i];
    F.twoff[i] = T.twoff[i];
  }
  const bool in_lds = sizeof(cplx<double>) * (size_t)L <= (150u << 10);
  hipLaunchKernelGGL(rader_setup_kernel, dim3(1), dim3(kFftBlock), in_lds ? sizeof(cplx<double>) * L : 0, st, F, M,
                     T.perm, (const cplx<double>*)T.tw64, (cplx<double>*)T.B64, (cplx<float>*)T.B32,
                     in_lds ? 1 : 0);
  USFFT_HIP(hipGetLastError());
  USFFT_HIP(hipStreamSynchronize(st));  // host vectors above go out of scope
}

// ---------------------------------------------------------------- lattice DFT
// Block-wide sums of N values in a fixed order (wave sums, then waves in
// order); every thread returns the same sums.
template <int BLOCK, int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double* red) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[w * N + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = red[i];
    for (int k = 1; k < NW; ++k) t += red[k * N + i];
    v[i] = t;
  }
}

// One lattice DFT for COLS node pairs (workgroup grp of the lattice), each
// pair packed as one complex column.
template <typename T, int BLOCK, int COLS>
__device__ __forceinline__ void rader_body(const FftPlanDev& F, int M, const int32_t* __restrict__ dlog,
                                           const int32_t* __restrict__ outidx, const cplx<T>* __restrict__ tw,
                                           const cplx<T>* __restrict__ B, const T* __restrict__ u, int64_t G,
                                           int64_t ld, int64_t col0, const int32_t* __restrict__ bins,
                                           const int32_t* __restrict__ pos, int pos_base, int nb, int out_kind,
                                           void* __restrict__ out, int64_t ldo, int64_t grp, cplx<T>* buf,
                                           double* red) {
  const int L = F.L;
  const T* r1[COLS];
  const T* r2[COLS];
  bool has1[COLS], has2[COLS];
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    const int64_t g1 = 2 * (grp * COLS + c), g2 = g1 + 1;
    has1[c] = g1 < G;
    has2[c] = g2 < G;
    r1[c] = u + (has1[c] ? g1 : 0) * ld + col0;  // rows past G are never read
    r2[c] = u + (has2[c] ? g2 : 0) * ld + col0;
  }
  // Rader input a_q = x[g^q]: each row segment is read in natural order
  // (coalesced) and scattered into LDS at q = dlog m; plus the sums for X[0].
  // A thread's next UI elements are loaded before any is stored (a
  // scheduling fence keeps the loads together), so their latencies overlap;
  // indices past M are clamped into the row and their values dropped.
  constexpr int UI = 4;
  double sums[2 * COLS];
#pragma unroll
  for (int i = 0; i < 2 * COLS; ++i) sums[i] = 0.0;
  for (int m0 = 1 + threadIdx.x; m0 < M; m0 += UI * BLOCK) {
    int qv[UI];
    T av[UI][COLS], bv[UI][COLS];
#pragma unroll
    for (int i = 0; i < UI; ++i) {
      const int mm = m0 + i * BLOCK, mc = mm < M ? mm : 0;
      qv[i] = dlog[mc];
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        av[i][c] = r1[c][mc];
        bv[i][c] = r2[c][mc];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < UI; ++i) {
      if (m0 + i * BLOCK >= M) break;
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        const T a = has1[c] ? av[i][c] : (T)0;
        const T b = has2[c] ? bv[i][c] : (T)0;
        buf[c * L + qv[i]] = {a, b};
        sums[2 * c] += (double)a;
        sums[2 * c + 1] += (double)b;
      }
    }
  }
  block_sum_n<BLOCK, 2 * COLS>(sums, red);  // also orders the LDS writes before the first stage
  // c = a (*) b: forward DIF, times B (same order), conjugate, forward DIT;
  // buf then holds conj(c) in natural order.
  fft_dif<T, BLOCK, COLS>(buf, F, tw, B);
  fft_dit<T, BLOCK, COLS>(buf, F, tw);
  const double invM = 1.0 / (double)M;
  double x01[COLS], x02[COLS], s1[COLS], s2[COLS];
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    x01[c] = (double)r1[c][0];
    x02[c] = has2[c] ? (double)r2[c][0] : 0.0;
    s1[c] = sums[2 * c] + x01[c];
    s2[c] = sums[2 * c + 1] + x02[c];
  }
  // bins in chunks of UO per thread: their table loads (bin, LDS positions,
  // output column) are issued together and serve every column
  constexpr int UO = 4;
  for (int a0 = threadIdx.x; a0 < nb; a0 += UO * BLOCK) {
    int ip[UO], im[UO];
    bool flip[UO], zero[UO];
    int64_t cc[UO];
#pragma unroll
    for (int i = 0; i < UO; ++i) {
      const int a = a0 + i * BLOCK, ac = a < nb ? a : a0;
      const int b = bins[ac];
      const int bcn = min(b, M - b);
      flip[i] = b > M - b;
      zero[i] = bcn == 0;
      const int bk = zero[i] ? 1 : bcn;  // X[0] reads no transform value
      ip[i] = outidx[bk];
      im[i] = outidx[M - bk];
      cc[i] = pos ? pos[ac] : pos_base + ac;  // contiguous when pos is null
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < UO; ++i) {
      if (a0 + i * BLOCK >= nb) break;
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        if (!has1[c]) continue;
        const int64_t g1 = 2 * (grp * COLS + c), g2 = g1 + 1;
        const cplx<T>* bc = buf + c * L;
        double X1r, X1i, X2r, X2i;
        if (zero[i]) {
          X1r = s1[c] * invM;
          X1i = 0.0;
          X2r = s2[c] * invM;
          X2i = 0.0;
        } else {
          const cplx<T> cp = bc[ip[i]];
          const cplx<T> cm = bc[im[i]];
          // X[bc] = x0 + c, X[M-bc] = x0 + c', with c = conj(buf)
          const double Xpr = x01[c] + (double)cp.x, Xpi = x02[c] - (double)cp.y;
          const double Xmr = x01[c] + (double)cm.x, Xmi = x02[c] - (double)cm.y;
          X1r = 0.5 * (Xpr + Xmr) * invM;
          X1i = 0.5 * (Xpi - Xmi) * invM;
          X2r = 0.5 * (Xpi + Xmi) * invM;
          X2i = -0.5 * (Xpr - Xmr) * invM;
        }
        if (flip[i]) {
          X1i = -X1i;
          X2i = -X2i;
        }
        double* o = static_cast<double*>(out);
        if (out_kind == USFFT_OUT_MAG2) {
          o[g1 * ldo + cc[i]] = X1r * X1r + X1i * X1i;
          if (has2[c]) o[g2 * ldo + cc[i]] = X2r * X2r + X2i * X2i;
        } else {
          o[(cc[i] * G + g1) * 2] = X1r;
          o[(cc[i] * G + g1) * 2 + 1] = X1i;
          if (has2[c]) {
            o[(cc[i] * G + g2) * 2] = X2r;
            o[(cc[i] * G + g2) * 2 + 1] = X2i;
          }
        }
      }
    }
  }
}

// One lattice (the stage entry point usfft_lattice_dft).
template <typename T, int BLOCK, int COLS>
__global__ __launch_bounds__(BLOCK) void rader_kernel(FftPlanDev F, int M, const int32_t* __restrict__ dlog,
                                                      const int32_t* __restrict__ outidx,
                                                      const cplx<T>* __restrict__ tw,
                                                      const cplx<T>* __restrict__ B, const T* __restrict__ u,
                                                      int64_t G, int64_t ld, int64_t col0,
                                                      const int32_t* __restrict__ bins,
                                                      const int32_t* __restrict__ pos, int pos_base, int nb,
                                                      int out_kind, void* __restrict__ out, int64_t ldo) {
  extern __shared__ char smem[];
  __shared__ double red[2 * COLS * (BLOCK / kWave)];
  rader_body<T, BLOCK, COLS>(F, M, dlog, outidx, tw, B, u, G, ld, col0, bins, pos, pos_base, nb, out_kind, out, ldo,
                             xcd_remap(blockIdx.x, gridDim.x), reinterpret_cast<cplx<T>*>(smem), red);
}

// Every lattice of a stage, and every iteration of a sampler batch, in one
// launch: workgroup w serves item w / wpi (wpi workgroups per item, all of
// the same G), node-pair group w % wpi.  Items of one XCD are contiguous, so
// an item's tables stay in one L2.
template <typename T, int BLOCK, int COLS>
__global__ __launch_bounds__(BLOCK) void rader_batch_kernel(const LatItem* __restrict__ items, int64_t wpi,
                                                            const T* __restrict__ u, int64_t G, int64_t ld,
                                                            int out_kind, void* __restrict__ out, int64_t ldo) {
  extern __shared__ char smem[];
  __shared__ double red[2 * COLS * (BLOCK / kWave)];
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  // the item stays in global memory: its radix plan is indexed by stage at
  // run time (scalar loads), which a private copy would send to scratch
  const LatItem& it = items[w / wpi];
  rader_body<T, BLOCK, COLS>(it.F, it.M, it.dlog, it.outidx, static_cast<const cplx<T>*>(it.tw),
                             static_cast<const cplx<T>*>(it.B), u, G, ld, it.col0, it.bins, it.pos, it.pos_base,
                             it.nb, out_kind, static_cast<double*>(out) + it.out_off, ldo, w % wpi,
                             reinterpret_cast<cplx<T>*>(smem), red);
}

void launch_lattice_dft(const RaderTables& T, const void* u, int u_fp32, int64_t G, int64_t ld, int64_t col0,
                        const int32_t* bins, const int32_t* pos, int pos_base, int nb, int out_kind, void* out,
                        int64_t ldo, hipStream_t st) {
  if (G <= 0 || nb <= 0) return;
  FftPlanDev F;
  F.L = T.L;
  F.nrad = T.nrad;
  for (int i = 0; i < 24; ++i) {
    F.radix[i] = T.radix[i];
    F.twoff[i] = T.twoff[i];
  }
  // workgroup sized to the transform (about L / 8 butterflies per radix-8
  // stage); several node pairs per workgroup while their transforms fit in
  // 64 KB of LDS, so twiddle and spectrum loads serve several columns
  const int block = T.L <= 1024 ? 128 : (T.L <= 3072 ? 256 : 512);
  const size_t colbytes = (size_t)T.L * (u_fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>));
  const int cols = 4 * colbytes <= (64u << 10) ? 4 : (2 * colbytes <= (64u << 10) ? 2 : 1);
  const unsigned grid = (unsigned)ceil_div(G, 2 * cols);
  const size_t lds = colbytes * cols;
#define USFFT_RADER(TT, BB, CC, TW, BS)                                                                     \
  hipLaunchKernelGGL((rader_kernel<TT, BB, CC>), dim3(grid), dim3(BB), lds, st, F, T.M, T.dlog, T.outidx,   \
                     (const cplx<TT>*)TW, (const cplx<TT>*)BS, (const TT*)u, G, ld, col0, bins, pos, pos_base, \
                     nb, out_kind, out, ldo)
#define USFFT_RADER_B(TT, CC, TW, BS)        \
  if (block == 128)                          \
    USFFT_RADER(TT, 128, CC, TW, BS);        \
  else if (block == 256)                     \
    USFFT_RADER(TT, 256, CC, TW, BS);        \
  else                                       \
    USFFT_RADER(TT, 512, CC, TW, BS)
#define USFFT_RADER_C(TT, TW, BS)            \
  if (cols == 4) {                           \
    USFFT_RADER_B(TT, 4, TW, BS);            \
  } else if (cols == 2) {                    \
    USFFT_RADER_B(TT, 2, TW, BS);            \
  } else {                                   \
    USFFT_RADER_B(TT, 1, TW, BS);            \
  }
  if (u_fp32) {
    USFFT_RADER_C(float, T.tw32, T.B32)
  } else {
    USFFT_RADER_C(double, T.tw64, T.B64)
  }
#undef USFFT_RADER_C
#undef USFFT_RADER_B
#undef USFFT_RADER
  USFFT_HIP(hipGetLastError());
}

// Workgroup shape of a batch whose largest transform has length Lmax (the
// same rule as one lattice).
static void rader_shape(int Lmax, int u_fp32, int* block, int* cols, size_t* lds) {
  *block = Lmax <= 1024 ? 128 : (Lmax <= 3072 ? 256 : 512);
  const size_t colbytes = (size_t)Lmax * (u_fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>));
  *cols = 4 * colbytes <= (64u << 10) ? 4 : (2 * colbytes <= (64u << 10) ? 2 : 1);
  *lds = colbytes * (size_t)*cols;
}

void fill_lat_item(LatItem& it, const RaderTables& T, int u_fp32) {
  it.F.L = T.L;
  it.F.nrad = T.nrad;
  for (int i = 0; i < 24; ++i) {
    it.F.radix[i] = T.radix[i];
    it.F.twoff[i] = T.twoff[i];
  }
  it.M = T.M;
  it.dlog = T.dlog;
  it.outidx = T.outidx;
  it.tw = u_fp32 ? T.tw32 : T.tw64;
  it.B = u_fp32 ? T.B32 : T.B64;
}

bool rader_shape_ok(int Lmax, int u_fp32, int block, int cols) {
  if (!(block == 128 || block == 256 || block == 512) || !(cols == 1 || cols == 2 || cols == 4)) return false;
  const size_t colbytes = (size_t)Lmax * (u_fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>));
  return colbytes * (size_t)cols <= (150u << 10);
}

void launch_lattice_dft_batch(const LatItem* items, int nitems, int Lmax, const void* u, int u_fp32, int64_t G,
                              int64_t ld, int out_kind, void* out, int64_t ldo, hipStream_t st, int shape_block,
                              int shape_cols) {
  if (G <= 0 || nitems <= 0) return;
  USFFT_REQUIRE(Lmax >= 2 && Lmax < lattice_mmax_for(u_fp32), USFFT_EINVAL, "lattice transform length out of range");
  int block = 0, cols = 0;
  size_t lds = 0;
  rader_shape(Lmax, u_fp32, &block, &cols, &lds);
  if (shape_block > 0 && rader_shape_ok(Lmax, u_fp32, shape_block, shape_cols)) {
    block = shape_block;
    cols = shape_cols;
    lds = (size_t)Lmax * (u_fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>)) * (size_t)cols;
  }
  const int64_t wpi = ceil_div(G, 2 * cols);
  const unsigned grid = (unsigned)(wpi * nitems);
#define USFFT_RB(TT, BB, CC) \
  hipLaunchKernelGGL((rader_batch_kernel<TT, BB, CC>), dim3(grid), dim3(BB), lds, st, items, wpi, (const TT*)u, G, ld, \
                     out_kind, out, ldo)
#define USFFT_RB_B(TT, CC)  \
  if (block == 128)         \
    USFFT_RB(TT, 128, CC);  \
  else if (block == 256)    \
    USFFT_RB(TT, 256, CC);  \
  else                      \
    USFFT_RB(TT, 512, CC)
#define USFFT_RB_C(TT)   \
  if (cols == 4) {       \
    USFFT_RB_B(TT, 4);   \
  } else if (cols == 2) { \
    USFFT_RB_B(TT, 2);   \
  } else {               \
    USFFT_RB_B(TT, 1);   \
  }
  if (u_fp32) {
    USFFT_RB_C(float)
  } else {
    USFFT_RB_C(double)
  }
#undef USFFT_RB_C
#undef USFFT_RB_B
#undef USFFT_RB
  USFFT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- line DFT
constexpr int kLineMax = 1024;
constexpr int kLineBlock = 256;
// The DFTs of the line samples u[g ld + col0 + l], l < K, of the npb nodes
// g0 .. g0 + npb - 1 (those below G), at the bins given (the canonical half
// spectrum: bins b and K - b are exact conjugates).  The nodes share one
// workgroup, so the phase table is computed once for all of them; each
// (node, bin) pair is one thread's direct sum over l.
template <typename T>
__device__ __forceinline__ void line_dft_nodes(const T* __restrict__ u, int64_t g0, int npb, int64_t G, int64_t ld,
                                               int64_t col0, int K, const int32_t* __restrict__ bins, int nb,
                                               int out_kind, void* __restrict__ out, int64_t ldo, double* x,
                                               double* cs, double* sn) {
  const int nn = (int)(G - g0 < npb ? G - g0 : (int64_t)npb);
  for (int l = threadIdx.x; l < K; l += kLineBlock) {
    double s, c;
    sincospi(2.0 * (double)l / (double)K, &s, &c);
    cs[l] = c;
    sn[l] = s;
  }
  for (int e = threadIdx.x; e < nn * K; e += kLineBlock) {
    const int j = e / K, l = e - j * K;
    x[e] = (double)u[(g0 + j) * ld + col0 + l];
  }
  __syncthreads();
  const double invK = 1.0 / (double)K;
  for (int e = threadIdx.x; e < nn * nb; e += kLineBlock) {
    const int j = e / nb, a = e - j * nb;
    const int64_t g = g0 + j;
    const double* xj = x + j * K;
    const int b = ((bins[a] % K) + K) % K;
    const int bc = min(b, K - b) % K;
    double re = 0.0, im = 0.0;
    int ph = 0;
    for (int l = 0; l < K; ++l) {
      re += xj[l] * cs[ph];
      im -= xj[l] * sn[ph];
      ph += bc;
      if (ph >= K) ph -= K;
    }
    re *= invK;
    im *= invK;
    if (b > K - b) im = -im;
    double* o = static_cast<double*>(out);
    if (out_kind == USFFT_OUT_MAG2) {
      o[g * ldo + a] = re * re + im * im;
    } else {
      o[((int64_t)a * G + g) * 2] = re;
      o[((int64_t)a * G + g) * 2 + 1] = im;
    }
  }
}

// Nodes per workgroup for lines of up to K samples: their samples (npb K
// doubles) and the phase table stay within 48 KB of LDS.
static int line_npb(int K) { return std::max(1, std::min(32, 4096 / std::max(K, 1))); }
static size_t line_lds(int K) { return sizeof(double) * (size_t)(line_npb(K) + 2) * (size_t)K; }

template <typename T>
__global__ __launch_bounds__(kLineBlock) void line_dft_kernel(const T* __restrict__ u, int64_t G, int64_t ld,
                                                              int64_t col0, int K, int npb,
                                                              const int32_t* __restrict__ bins, int nb, int out_kind,
                                                              void* __restrict__ out, int64_t ldo) {
  extern __shared__ double lsh[];
  line_dft_nodes(u, xcd_remap(blockIdx.x, gridDim.x) * npb, npb, G, ld, col0, K, bins, nb, out_kind, out, ldo, lsh,
                 lsh + (size_t)npb * K, lsh + (size_t)(npb + 1) * K);
}

// All step-1 lines in one launch: blockIdx.y = line y of coordinate
// t = y / line_r, samples from column loff[y], its K_t = lineK[t] candidates
// cands[sum_{j<t} K_j ..] at every bin, |.|^2 to columns y * line_stride ..
// of out (leading dimension ldo).  The LDS carve-up follows Kmax.
template <typename T>
__global__ __launch_bounds__(kLineBlock) void line_dft_lines_kernel(const T* __restrict__ u, int64_t G, int64_t ld,
                                                                    const int64_t* __restrict__ loff,
                                                                    const int32_t* __restrict__ lineK,
                                                                    const int32_t* __restrict__ cands, int line_r,
                                                                    int64_t line_stride, double* __restrict__ out,
                                                                    int64_t ldo, int Kmax, int npb) {
  extern __shared__ double lsh[];
  const int y = blockIdx.y, t = y / line_r;
  int64_t coff = 0;
  for (int j = 0; j < t; ++j) coff += lineK[j];
  const int K = lineK[t];
  line_dft_nodes(u, xcd_remap(blockIdx.x, gridDim.x) * npb, npb, G, ld, loff[y], K, cands + coff, K,
                 USFFT_OUT_MAG2, out + (int64_t)y * line_stride, ldo, lsh, lsh + (size_t)npb * Kmax,
                 lsh + (size_t)(npb + 1) * Kmax);
}

void launch_line_dft_lines(const void* u, int u_fp32, int64_t G, int64_t ld, const int64_t* loff,
                           const int32_t* lineK, const int32_t* cands, int nlines, int line_r, int Kmax,
                           int64_t line_stride, double* out, int64_t ldo, hipStream_t st) {
  USFFT_REQUIRE(Kmax >= 1 && Kmax <= kLineMax && line_stride >= Kmax, USFFT_EINVAL, "line DFT length out of range");
  if (G <= 0 || nlines <= 0) return;
  const int npb = line_npb(Kmax);
  const dim3 grid((unsigned)ceil_div(G, npb), (unsigned)nlines);
  if (u_fp32)
    hipLaunchKernelGGL(line_dft_lines_kernel<float>, grid, dim3(kLineBlock), line_lds(Kmax), st, (const float*)u, G,
                       ld, loff, lineK, cands, line_r, line_stride, out, ldo, Kmax, npb);
  else
    hipLaunchKernelGGL(line_dft_lines_kernel<double>, grid, dim3(kLineBlock), line_lds(Kmax), st, (const double*)u,
                       G, ld, loff, lineK, cands, line_r, line_stride, out, ldo, Kmax, npb);
  USFFT_HIP(hipGetLastError());
}

void launch_line_dft(const void* u, int u_fp32, int64_t G, int64_t ld, int64_t col0, int K, const int32_t* bins,
                     int nb, int out_kind, void* out, int64_t ldo, hipStream_t st) {
  USFFT_REQUIRE(K >= 1 && K <= kLineMax, USFFT_EINVAL, "line DFT length out of range");
  if (G <= 0 || nb <= 0) return;
  const int npb = line_npb(K);
  const unsigned grid = (unsigned)ceil_div(G, npb);
  if (u_fp32)
    hipLaunchKernelGGL(line_dft_kernel<float>, dim3(grid), dim3(kLineBlock), line_lds(K), st, (const float*)u, G, ld,
                       col0, K, npb, bins, nb, out_kind, out, ldo);
  else
    hipLaunchKernelGGL(line_dft_kernel<double>, dim3(grid), dim3(kLineBlock), line_lds(K), st, (const double*)u, G,
                       ld, col0, K, npb, bins, nb, out_kind, out, ldo);
  USFFT_HIP(hipGetLastError());
}

}  // namespace usfft
