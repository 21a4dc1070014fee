// Mixed-precision Chebyshev products for gfx950.
//
// FQ_FP32: operands rounded to FP32, products on FP32 matrix cores
// (v_mfma_f32_16x16x4f32), FP32 accumulation.
// FQ_BF16X3: every operand element x is split into three BF16 pieces
// x ~ hi + mid + lo (each piece the rounded remainder of the previous ones,
// about 24 significant bits in total); a real product keeps the six piece
// products whose weight is at least 2^-16 of the leading one
// (hh, hm, mh, hl, mm, lh) on BF16 matrix cores (v_mfma_f32_16x16x32_bf16)
// with FP32 accumulation.
//
// In both, the propagated block X and the Chebyshev sum Y stay FP64: the first
// product of a step reads X and rounds / splits it while staging it into LDS,
// the epilogue adds the Bessel-weighted term to Y in FP64, and the last
// product applies the step phase in FP64. Only the chain P_1 .. P_L is held in
// the product format.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "formats.h"
#include "internal.h"

namespace fq {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  // lane l: A(l%16, l/16), B(l/16, l%16); holds D(4*(l/16)+r, l%16)
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  // lane l: A(l%16, 8*(l/16)+e), B(8*(l/16)+e, l%16), e = 0..7; holds D(4*(l/16)+r, l%16)
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int KIND>
struct EpiMix {
  ChebTermX t;
  long ld;
  __device__ __forceinline__ void operator()(int m, int n, float ar_, float ai_) const {
    const long idx = (long)m * ld + n;
    const double ar = ar_, ai = ai_;
    double pr, pi;
    load_c(t.p, t.p_fmt, t.plane, idx, pr, pi);
    if (KIND == CHEB_FIRST) {
      double o_r = ar, o_i = ai;
      store_c(t.o, t.o_fmt, t.plane, idx, o_r, o_i);
      t.y_re[idx] = t.c0r * pr - t.c0i * pi + t.cr * o_r - t.ci * o_i;
      t.y_im[idx] = t.c0r * pi + t.c0i * pr + t.cr * o_i + t.ci * o_r;
    } else if (KIND == CHEB_FIRST_LAST) {
      const double sr = t.c0r * pr - t.c0i * pi + t.cr * ar - t.ci * ai;
      const double si = t.c0r * pi + t.c0i * pr + t.cr * ai + t.ci * ar;
      double o_r = t.phr * sr - t.phi * si, o_i = t.phr * si + t.phi * sr;
      store_c(t.o, t.o_fmt, t.plane, idx, o_r, o_i);
    } else if (KIND == CHEB_MID) {
      double o_r = 2.0 * ar - pr, o_i = 2.0 * ai - pi;
      store_c(t.o, t.o_fmt, t.plane, idx, o_r, o_i);
      t.y_re[idx] += t.cr * o_r - t.ci * o_i;
      t.y_im[idx] += t.cr * o_i + t.ci * o_r;
    } else {
      const double qr = 2.0 * ar - pr, qi = 2.0 * ai - pi;
      const double sr = t.y_re[idx] + t.cr * qr - t.ci * qi;
      const double si = t.y_im[idx] + t.cr * qi + t.ci * qr;
      double o_r = t.phr * sr - t.phi * si, o_i = t.phr * si + t.phi * sr;
      store_c(t.o, t.o_fmt, t.plane, idx, o_r, o_i);
    }
  }
};

struct MixOperands {
  const void* a;  // A planes (format per kernel instance)
  const void* b;  // B planes
  long plane;
  int ld;
  int kdim;
  int tiles_m, tiles_n;
};

// ---------------------------------------------------------------------------------------------
// FP32 products. A = F32 planes, or F64 planes (X) rounded while staging.
// LDS row stride BK + 4 floats: the 16 rows read by one 16-lane group start on
// distinct 4-bank groups, so 16-byte reads are conflict-free.
// ---------------------------------------------------------------------------------------------
template <int BM, int BN, int BK, int WGM, int WGN, bool A_F64, class Epi>
__global__ __launch_bounds__(WGM* WGN * 64) void cheb_f32_kernel(MixOperands op, Epi epi) {
  constexpr int NT = WGM * WGN * 64;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int S = BK + 4;
  constexpr int AEL = A_F64 ? 2 : 4;  // elements per 16-byte global chunk of A
  constexpr int CPRA = BK / AEL, CPRB = BK / 4;
  constexpr int RA = BM * CPRA / NT, RB = BN * CPRB / NT;
  static_assert(BM * CPRA % NT == 0 && BN * CPRB % NT == 0, "load split");
  static_assert(BK % 16 == 0, "BK");

  __shared__ __attribute__((aligned(16))) float As[2][BM * S];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN * S];

  int tm, tn;
  tile_coords(blockIdx.x, op.tiles_m, op.tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WGN, wn = wid % WGN;
  const long ld = op.ld, plane = op.plane;

  f4 accR[FM][FN], accI[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accR[i][j] = f4{0, 0, 0, 0};
      accI[i][j] = f4{0, 0, 0, 0};
    }

  using AChunk = typename std::conditional<A_F64, d2, f4>::type;
  AChunk ga[2][RA];
  f4 gb[2][RB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int c = tid + r * NT, row = c / CPRA, col = AEL * (c % CPRA);
      const long off = (long)(m0 + row) * ld + k0 + col;
      if constexpr (A_F64) {
        const double* a = static_cast<const double*>(op.a);
        ga[0][r] = *reinterpret_cast<const d2*>(a + off);
        ga[1][r] = *reinterpret_cast<const d2*>(a + plane + off);
      } else {
        const float* a = static_cast<const float*>(op.a);
        ga[0][r] = *reinterpret_cast<const f4*>(a + off);
        ga[1][r] = *reinterpret_cast<const f4*>(a + plane + off);
      }
    }
    const float* b = static_cast<const float*>(op.b);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int c = tid + r * NT, row = c / CPRB, col = 4 * (c % CPRB);
      const long off = (long)(n0 + row) * ld + k0 + col;
      gb[0][r] = *reinterpret_cast<const f4*>(b + off);
      gb[1][r] = *reinterpret_cast<const f4*>(b + plane + off);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int c = tid + r * NT, row = c / CPRA, col = AEL * (c % CPRA);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if constexpr (A_F64) {
          *reinterpret_cast<f2*>(&As[p][row * S + col]) = f2{(float)ga[p][r][0], (float)ga[p][r][1]};
        } else {
          *reinterpret_cast<f4*>(&As[p][row * S + col]) = ga[p][r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int c = tid + r * NT, row = c / CPRB, col = 4 * (c % CPRB);
      *reinterpret_cast<f4*>(&Bs[0][row * S + col]) = gb[0][r];
      *reinterpret_cast<f4*>(&Bs[1][row * S + col]) = gb[1][r];
    }
  };

  gload(0);
  for (int k0 = 0; k0 < op.kdim; k0 += BK) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (k0 + BK < op.kdim) gload(k0 + BK);
    const int rr = lane & 15;
#pragma unroll
    for (int p = 0; p < BK / 16; ++p) {
      const int kk = 16 * p + 4 * (lane >> 4);
      f4 far_[FM], fai[FM], fbr[FN], fbi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int row = wm * WTM + i * 16 + rr;
        far_[i] = *reinterpret_cast<const f4*>(&As[0][row * S + kk]);
        fai[i] = *reinterpret_cast<const f4*>(&As[1][row * S + kk]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int row = wn * WTN + j * 16 + rr;
        fbr[j] = *reinterpret_cast<const f4*>(&Bs[0][row * S + kk]);
        fbi[j] = *reinterpret_cast<const f4*>(&Bs[1][row * S + kk]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) accR[i][j] = mfma_f32(far_[i][t], fbr[j][t], accR[i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) accI[i][j] = mfma_f32(far_[i][t], fbi[j][t], accI[i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) accR[i][j] = mfma_f32(-fai[i][t], fbi[j][t], accR[i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) accI[i][j] = mfma_f32(fai[i][t], fbr[j][t], accI[i][j]);
      }
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * WTN + j * 16 + (lane & 15);
        epi(m, n, accR[i][j][r], accI[i][j][r]);
      }
}

// ---------------------------------------------------------------------------------------------
// Split-BF16 products. A = BF16X3 planes, or F64 planes (X) split while staging.
// B = BF16X3 planes. One MFMA k-chunk (32) per LDS stage; LDS row stride 40
// halves (80 bytes) keeps the 16-byte fragment reads conflict-free.
// ---------------------------------------------------------------------------------------------
template <int BM, int BN, int WGM, int WGN, bool A_F64, class Epi>
__global__ __launch_bounds__(WGM* WGN * 64) void cheb_bf16x3_kernel(MixOperands op, Epi epi) {
  constexpr int BK = 32;
  constexpr int NT = WGM * WGN * 64;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int S = BK + 8;
  constexpr int CPR16 = BK / 8;                  // 16-byte chunks per row of a BF16 plane
  constexpr int CPR64 = BK / 2;                  // 16-byte chunks per row of an F64 plane
  constexpr int RA = A_F64 ? BM * CPR64 / NT : BM * CPR16 / NT;
  constexpr int RB = BN * CPR16 / NT;
  static_assert((A_F64 ? BM * CPR64 : BM * CPR16) % NT == 0 && BN * CPR16 % NT == 0, "split");

  __shared__ __attribute__((aligned(16))) u16 As[6][BM * S];
  __shared__ __attribute__((aligned(16))) u16 Bs[6][BN * S];

  int tm, tn;
  tile_coords(blockIdx.x, op.tiles_m, op.tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WGN, wn = wid % WGN;
  const long ld = op.ld, plane = op.plane;

  f4 accR[FM][FN], accI[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accR[i][j] = f4{0, 0, 0, 0};
      accI[i][j] = f4{0, 0, 0, 0};
    }

  using AChunk = typename std::conditional<A_F64, d2, u32x4>::type;
  constexpr int APL = A_F64 ? 2 : 6;
  AChunk ga[APL][RA];
  u32x4 gb[6][RB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      if constexpr (A_F64) {
        const int c = tid + r * NT, row = c / CPR64, col = 2 * (c % CPR64);
        const long off = (long)(m0 + row) * ld + k0 + col;
        const double* a = static_cast<const double*>(op.a);
        ga[0][r] = *reinterpret_cast<const d2*>(a + off);
        ga[1][r] = *reinterpret_cast<const d2*>(a + plane + off);
      } else {
        const int c = tid + r * NT, row = c / CPR16, col = 8 * (c % CPR16);
        const long off = (long)(m0 + row) * ld + k0 + col;
        const u16* a = static_cast<const u16*>(op.a);
#pragma unroll
        for (int p = 0; p < 6; ++p) ga[p][r] = *reinterpret_cast<const u32x4*>(a + p * plane + off);
      }
    }
    const u16* b = static_cast<const u16*>(op.b);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int c = tid + r * NT, row = c / CPR16, col = 8 * (c % CPR16);
      const long off = (long)(n0 + row) * ld + k0 + col;
#pragma unroll
      for (int p = 0; p < 6; ++p) gb[p][r] = *reinterpret_cast<const u32x4*>(b + p * plane + off);
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      if constexpr (A_F64) {
        const int c = tid + r * NT, row = c / CPR64, col = 2 * (c % CPR64);
#pragma unroll
        for (int q = 0; q < 2; ++q) {  // re, im
          u16 h0, m0_, l0, h1, m1, l1;
          split3((float)ga[q][r][0], h0, m0_, l0);
          split3((float)ga[q][r][1], h1, m1, l1);
          *reinterpret_cast<uint32_t*>(&As[3 * q + 0][row * S + col]) = h0 | ((uint32_t)h1 << 16);
          *reinterpret_cast<uint32_t*>(&As[3 * q + 1][row * S + col]) = m0_ | ((uint32_t)m1 << 16);
          *reinterpret_cast<uint32_t*>(&As[3 * q + 2][row * S + col]) = l0 | ((uint32_t)l1 << 16);
        }
      } else {
        const int c = tid + r * NT, row = c / CPR16, col = 8 * (c % CPR16);
#pragma unroll
        for (int p = 0; p < 6; ++p) *reinterpret_cast<u32x4*>(&As[p][row * S + col]) = ga[p][r];
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int c = tid + r * NT, row = c / CPR16, col = 8 * (c % CPR16);
#pragma unroll
      for (int p = 0; p < 6; ++p) *reinterpret_cast<u32x4*>(&Bs[p][row * S + col]) = gb[p][r];
    }
  };

  // (piece of A, piece of B) pairs kept below: weights 1, 2^-8 (x2), 2^-16 (x3)
  gload(0);
  for (int k0 = 0; k0 < op.kdim; k0 += BK) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (k0 + BK < op.kdim) gload(k0 + BK);
    const int rr = lane & 15, kk = 8 * (lane >> 4);
    bf8 fb[6][FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int row = wn * WTN + j * 16 + rr;
#pragma unroll
      for (int p = 0; p < 6; ++p) fb[p][j] = *reinterpret_cast<const bf8*>(&Bs[p][row * S + kk]);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int row = wm * WTM + i * 16 + rr;
      bf8 fa[6], fan[3];
#pragma unroll
      for (int p = 0; p < 6; ++p) fa[p] = *reinterpret_cast<const bf8*>(&As[p][row * S + kk]);
#pragma unroll
      for (int p = 0; p < 3; ++p) {  // -Ai pieces (sign flip of each half word)
        u32x4 u = __builtin_bit_cast(u32x4, fa[3 + p]);
        u.x ^= 0x80008000u;
        u.y ^= 0x80008000u;
        u.z ^= 0x80008000u;
        u.w ^= 0x80008000u;
        fan[p] = __builtin_bit_cast(bf8, u);
      }
#define FQ_PIECES(pa, pb)                                                                        \
  {                                                                                              \
    _Pragma("unroll") for (int j = 0; j < FN; ++j) accR[i][j] =                                  \
        mfma_bf16(fa[pa], fb[pb][j], accR[i][j]);                                                \
    _Pragma("unroll") for (int j = 0; j < FN; ++j) accI[i][j] =                                  \
        mfma_bf16(fa[pa], fb[3 + pb][j], accI[i][j]);                                            \
    _Pragma("unroll") for (int j = 0; j < FN; ++j) accR[i][j] =                                  \
        mfma_bf16(fan[pa], fb[3 + pb][j], accR[i][j]);                                           \
    _Pragma("unroll") for (int j = 0; j < FN; ++j) accI[i][j] =                                  \
        mfma_bf16(fa[3 + pa], fb[pb][j], accI[i][j]);                                            \
  }
      FQ_PIECES(0, 0)
      FQ_PIECES(0, 1)
      FQ_PIECES(1, 0)
      FQ_PIECES(0, 2)
      FQ_PIECES(1, 1)
      FQ_PIECES(2, 0)
#undef FQ_PIECES
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * WTN + j * 16 + (lane & 15);
        epi(m, n, accR[i][j][r], accI[i][j][r]);
      }
}

// ---- launchers ---------------------------------------------------------------------------------

template <bool A_F64, class Epi>
hipError_t launch_f32(MixOperands op, int mrows, int np, Epi epi, hipStream_t s) {
  if (mrows % 128 == 0 && np % 128 == 0 && (long)mrows * np >= 512L * 1024) {
    op.tiles_m = mrows / 128;
    op.tiles_n = np / 128;
    hipLaunchKernelGGL((cheb_f32_kernel<128, 128, 32, 2, 4, A_F64, Epi>),
                       dim3(op.tiles_m * op.tiles_n), dim3(512), 0, s, op, epi);
  } else if (mrows % 64 == 0 && np % 64 == 0) {
    op.tiles_m = mrows / 64;
    op.tiles_n = np / 64;
    hipLaunchKernelGGL((cheb_f32_kernel<64, 64, 32, 2, 2, A_F64, Epi>),
                       dim3(op.tiles_m * op.tiles_n), dim3(256), 0, s, op, epi);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool A_F64, class Epi>
hipError_t launch_bf16x3(MixOperands op, int mrows, int np, Epi epi, hipStream_t s) {
  if (mrows % 128 == 0 && np % 128 == 0 && (long)mrows * np >= 512L * 1024) {
    op.tiles_m = mrows / 128;
    op.tiles_n = np / 128;
    hipLaunchKernelGGL((cheb_bf16x3_kernel<128, 128, 2, 4, A_F64, Epi>),
                       dim3(op.tiles_m * op.tiles_n), dim3(512), 0, s, op, epi);
  } else if (mrows % 64 == 0 && np % 64 == 0) {
    op.tiles_m = mrows / 64;
    op.tiles_n = np / 64;
    hipLaunchKernelGGL((cheb_bf16x3_kernel<64, 64, 2, 2, A_F64, Epi>),
                       dim3(op.tiles_m * op.tiles_n), dim3(256), 0, s, op, epi);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class Epi>
hipError_t dispatch(const ChebTermX& t, int precision, int mrows, int np, Epi epi, hipStream_t s) {
  MixOperands op{t.a, t.b, t.plane, np, np, 0, 0};
  // The first product of a step (A = X in FP64) runs on FP64 matrix cores
  // (launch_cheb_first_mixed); these kernels take the P_l in the product format.
  if (t.a_fmt == FMT_F64) return hipErrorInvalidValue;
  if (precision == FQ_FP32) return launch_f32<false>(op, mrows, np, epi, s);
  if (precision == FQ_BF16X3) return launch_bf16x3<false>(op, mrows, np, epi, s);
  return hipErrorInvalidValue;
}

// The rescaled Hamiltonian in FP64 (for the first product of a step) and in
// the product format (for the others), from one pass over H0, Hmod and K.
__global__ void heff_mixed_kernel(const double* __restrict__ h0r, const double* __restrict__ h0i,
                                  const double* __restrict__ vr, const double* __restrict__ vi,
                                  const double* __restrict__ kr, const double* __restrict__ ki,
                                  double a, double b, double beta, double inv_dE, long n, long ld,
                                  double* __restrict__ hr, double* __restrict__ hi, void* out,
                                  int fmt) {
  const long total = n * ld, plane = ld * ld;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long i = e / ld, k = e % ld;
    if (k >= n) continue;
    double re = h0r[e] + a * vr[e] + b * kr[e];
    double im = h0i[e] + a * vi[e] + b * ki[e];
    if (i == k) re -= beta;
    re *= inv_dE;
    im *= inv_dE;
    hr[e] = re;
    hi[e] = im;
    store_c(out, fmt, plane, e, re, im);
  }
}

}  // namespace

hipError_t launch_cheb_mixed(const ChebTermX& t, int precision, int mrows, int np, hipStream_t s) {
  switch (t.kind) {
    case CHEB_FIRST:
      return dispatch(t, precision, mrows, np, EpiMix<CHEB_FIRST>{t, np}, s);
    case CHEB_FIRST_LAST:
      return dispatch(t, precision, mrows, np, EpiMix<CHEB_FIRST_LAST>{t, np}, s);
    case CHEB_MID:
      return dispatch(t, precision, mrows, np, EpiMix<CHEB_MID>{t, np}, s);
    case CHEB_LAST:
      return dispatch(t, precision, mrows, np, EpiMix<CHEB_LAST>{t, np}, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_heff_mixed(const double* h0r, const double* h0i, const double* vr,
                             const double* vi, const double* kr, const double* ki, double a,
                             double b, double beta, double dE, long n, long ld, double* hr,
                             double* hi, void* out, int precision, hipStream_t s) {
  const int fmt = precision == FQ_FP32 ? FMT_F32 : FMT_BF16X3;
  long g = (n * ld + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(heff_mixed_kernel, dim3((unsigned)g), dim3(256), 0, s, h0r, h0i, vr, vi, kr,
                     ki, a, b, beta, 1.0 / dE, n, ld, hr, hi, out, fmt);
  return hipGetLastError();
}

}  // namespace fq
