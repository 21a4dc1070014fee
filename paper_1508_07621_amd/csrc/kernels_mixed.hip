// Mixed-precision Chebyshev products for gfx950.
//
// FQ_FP32: operands rounded to FP32 (planar, row-major), products on FP32
// matrix cores (v_mfma_f32_16x16x4f32), FP32 accumulation.
// FQ_BF16X3: every operand element x is split into three BF16 pieces
// x ~ hi + mid + lo (each piece the rounded remainder of the previous ones,
// about 24 significant bits in total), stored k-blocked (bf3_offset); a real
// product keeps the six piece products whose weight is at least 2^-16 of the
// leading one (hh, hm, mh, hl, mm, lh) on BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation.
//
// In both, the propagated block X and the Chebyshev sum Y stay FP64: the first
// product of a step, P_1 = Ht X, runs on FP64 matrix cores (its term carries
// the largest weight |c_1| ~ R) and stores P_1 in the product format; the
// kernels here form P_2 .. P_L, add each Bessel-weighted term to Y in FP64,
// and the last one applies the step phase in FP64.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "epilogues.h"
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
    load_c(t.p, t.p_fmt, t.plane, m, n, ld, pr, pi);
    if (KIND == CHEB_FIRST) {
      double o_r = ar, o_i = ai;
      store_c(t.o, t.o_fmt, t.plane, m, n, ld, o_r, o_i);
      t.y_re[idx] = t.c0r * pr - t.c0i * pi + t.cr * o_r - t.ci * o_i;
      t.y_im[idx] = t.c0r * pi + t.c0i * pr + t.cr * o_i + t.ci * o_r;
    } else if (KIND == CHEB_FIRST_LAST) {
      const double sr = t.c0r * pr - t.c0i * pi + t.cr * ar - t.ci * ai;
      const double si = t.c0r * pi + t.c0i * pr + t.cr * ai + t.ci * ar;
      double o_r = t.phr * sr - t.phi * si, o_i = t.phr * si + t.phi * sr;
      store_c(t.o, t.o_fmt, t.plane, m, n, ld, o_r, o_i);
    } else if (KIND == CHEB_MID) {
      double o_r = 2.0 * ar - pr, o_i = 2.0 * ai - pi;
      store_c(t.o, t.o_fmt, t.plane, m, n, ld, o_r, o_i);
      t.y_re[idx] += t.cr * o_r - t.ci * o_i;
      t.y_im[idx] += t.cr * o_i + t.ci * o_r;
    } else {
      const double qr = 2.0 * ar - pr, qi = 2.0 * ai - pi;
      const double sr = t.y_re[idx] + t.cr * qr - t.ci * qi;
      const double si = t.y_im[idx] + t.cr * qi + t.ci * qr;
      double o_r = t.phr * sr - t.phi * si, o_i = t.phr * si + t.phi * sr;
      store_c(t.o, t.o_fmt, t.plane, m, n, ld, o_r, o_i);
    }
  }
  __device__ __forceinline__ void finish() const {}
};

struct MixOperands {
  const void* a;  // A planes (format per kernel instance): real plane, imaginary plane
  const void* b;  // B planes
  long plane_a;   // elements from A's real plane to its imaginary plane
  long plane_b;   // same for B
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

  __shared__ __attribute__((aligned(16))) float As[2][2][BM * S];  // [stage][re, im]
  __shared__ __attribute__((aligned(16))) float Bs[2][2][BN * S];

  int tm, tn;
  tile_coords(blockIdx.x, op.tiles_m, op.tiles_n, tm, tn);
  if (tm >= op.tiles_m) return;  // grid padding
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WGN, wn = wid % WGN;
  const long ld = op.ld, plane = op.plane_a, plane_b = op.plane_b;

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
      gb[1][r] = *reinterpret_cast<const f4*>(b + plane_b + off);
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int c = tid + r * NT, row = c / CPRA, col = AEL * (c % CPRA);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if constexpr (A_F64) {
          *reinterpret_cast<f2*>(&As[st][p][row * S + col]) =
              f2{(float)ga[p][r][0], (float)ga[p][r][1]};
        } else {
          *reinterpret_cast<f4*>(&As[st][p][row * S + col]) = ga[p][r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int c = tid + r * NT, row = c / CPRB, col = 4 * (c % CPRB);
      *reinterpret_cast<f4*>(&Bs[st][0][row * S + col]) = gb[0][r];
      *reinterpret_cast<f4*>(&Bs[st][1][row * S + col]) = gb[1][r];
    }
  };

  // Two LDS stages, one barrier per K-stage (as in the FP64 kernel).
  const int nk = op.kdim / BK;
  gload(0);
  lstore(0);
  if (nk > 1) gload(BK);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int cur = kb & 1;
    if (kb + 1 < nk) lstore(cur ^ 1);  // that stage was last read before the previous barrier
    if (kb + 2 < nk) gload((kb + 2) * BK);
    const int rr = lane & 15;
#pragma unroll
    for (int p = 0; p < BK / 16; ++p) {
      const int kk = 16 * p + 4 * (lane >> 4);
      f4 far_[FM], fai[FM], fbr[FN], fbi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int row = wm * WTM + i * 16 + rr;
        far_[i] = *reinterpret_cast<const f4*>(&As[cur][0][row * S + kk]);
        fai[i] = *reinterpret_cast<const f4*>(&As[cur][1][row * S + kk]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int row = wn * WTN + j * 16 + rr;
        fbr[j] = *reinterpret_cast<const f4*>(&Bs[cur][0][row * S + kk]);
        fbi[j] = *reinterpret_cast<const f4*>(&Bs[cur][1][row * S + kk]);
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
    __syncthreads();
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
  epi.finish();
}

// ---------------------------------------------------------------------------------------------
// Split-BF16 products P_{l+1} = 2 Ht P_l - P_{l-1} on 32x32x16 BF16 matrix cores.
//
// A = P_l and B = Ht are BF16X3 matrices in the k-blocked layout (bf3_offset)
// with six stored planes: the three pieces of the real part and of the
// imaginary part; the three pieces of their sum are formed while staging, so
// that LDS holds nine planes. A complex product takes three real ones (Gauss):
// T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi), Re = T1 - T2,
// Im = T3 - T1 - T2, each over the 6 kept piece pairs (hh, hm, mh, hl, mm, lh):
// 18 products of 32x32x16 per tile and k-block instead of 24.
//
// One k-block (16 columns) of a BM-row tile is 6 contiguous runs of BM x 32
// bytes in the stored planes. Each thread owns one 16-byte chunk (8 columns of
// one row) of A or of B: it loads that chunk from the six planes (coalesced
// across the threads), forms the pieces of re + im from the values the pieces
// hold (split3 of hi + mid + lo of re plus that of im, in FP32), and writes all
// nine planes to LDS in the stored row-swizzled layout, so the fragment reads
// (lane l: row l % 32, columns 8 (l / 32) .. + 7) are conflict-free. Two LDS
// stages: while the waves multiply out of one, the next k-block is written to
// the other from registers loaded one stage earlier; one barrier per k-block.
//
// Epilogue: Re and Im are written to LDS in the k-blocked order, then each
// thread takes 8 consecutive columns of one row (one 16-byte chunk of every
// BF16 plane): it reads P_{l-1}, forms P_{l+1} = 2 acc - P_{l-1} in FP64,
// stores its split pieces, and adds c_l P_{l+1} (the stored value) to the
// FP64 sum Y; the last product of a step instead writes
// X_k = exp(-i beta h) (Y + c_L P_L) as FP64 planes.
// ---------------------------------------------------------------------------------------------
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f16v mfma32_bf16(bf8 a, bf8 b, f16v c) {
  // lane l: A(l%32, 8*(l/32)+e), B(8*(l/32)+e, l%32); holds D(8*(r/4)+4*(l/32)+r%4, l%32)
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

struct Bf3Args {
  const u16* a;        // A, k-blocked BF16X3 (row capacity np): P_l, or X for the first product
  const u16* b;        // B = Ht, k-blocked BF16X3
  const void* p;       // P_{l-1}: k-blocked BF16X3, or FP64 planes (P_0 = X; X itself for the
                       // first product, whose sum starts with c_0 X)
  void* o;             // P_{l+1} (k-blocked BF16X3) or X_k (FP64 planes, last product)
  double* y_re;        // Chebyshev sum, FP64 planes
  double* y_im;
  long plane;          // np * np
  int np;
  int tiles_m, tiles_n;
  double c0r, c0i, cr, ci, phr, phi;
};

// The leading `npc` pieces of x (fp32): hi, or hi and mid, or all three.
template <int NPC>
__device__ __forceinline__ void split_n(float x, u16* out) {
  if constexpr (NPC == 3) {
    split3(x, out[0], out[1], out[2]);
  } else {
    const __bf16 bh = (__bf16)x;
    out[0] = bf16_bits(bh);
    if constexpr (NPC == 2) out[1] = bf16_bits((__bf16)(x - (float)bh));
  }
}

// Epilogue of a split-BF16 product tile from its Re and Im in LDS (FP32,
// k-blocked order, see the writers): each thread takes 8 consecutive columns
// of one row at a time (one 16-byte chunk of every BF16 plane), reads P_{l-1}
// (or X for the first product), forms the term in FP64 and stores it as BF16X3
// pieces with its stored value weighted into the sum Y, or, for the last
// product, writes X_k = exp(-i beta h) (Y + c_L P_L) as FP64 planes. The
// global loads of two chunks (P_{l-1} and Y) are issued before any of their
// stores: the stores may alias later loads of the same buffers in the
// compiler's view (P_{l+1} overwrites P_{l-1} in place), which would otherwise
// serialise one memory round trip per chunk and per buffer.
template <int BM, int BN, int NT, int KIND, bool P_F64, int BATCH = 2>
__device__ __forceinline__ void bf3_tile_epilogue(const Bf3Args& g, const float* cre,
                                                  const float* cim, int m0, int n0, int tid) {
  constexpr int NS = BF3_PLANES;
  constexpr bool FIRST = KIND == CHEB_FIRST || KIND == CHEB_FIRST_LAST;
  constexpr bool TO_X = KIND == CHEB_LAST || KIND == CHEB_FIRST_LAST;
  constexpr int NQ = BM * BN / 8 / NT;     // chunks per thread
  constexpr int B = NQ >= BATCH ? BATCH : 1;  // chunks whose loads are in flight together
  static_assert(NQ * NT * 8 == BM * BN && NQ % B == 0, "chunk split");
  const long np = g.np, plane = g.plane;
  const double cr_ = g.cr, ci_ = g.ci;
#pragma unroll
  for (int i0 = 0; i0 < NQ; i0 += B) {
    long mrow[B], ncol[B], chunk[B];
    float ar[B][8], ai[B][8];
    u32x4 pw[B][6];          // P_{l-1} as stored pieces (BF16X3)
    d2 pd[B][8];             // or as FP64 pairs: [0..3] re, [4..7] im
    d2 yv[B][8];             // Y pairs: [0..3] re, [4..7] im
    // ---- loads of B chunks ----
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int q = tid + (i0 + b) * NT;
      const int kbl = q / (2 * BM), rem = q % (2 * BM);
      const int row = rem >> 1, slot = rem & 1;
      mrow[b] = m0 + row;
      ncol[b] = n0 + kbl * 16 + 8 * (slot ^ ((row >> 3) & 1));  // first of 8 columns
      chunk[b] = ((long)(n0 / 16 + kbl) * np + mrow[b]) * 16 + 8 * slot;  // in a BF16X3 plane
      *reinterpret_cast<f4*>(ar[b]) = *reinterpret_cast<const f4*>(cre + q * 8);
      *reinterpret_cast<f4*>(ar[b] + 4) = *reinterpret_cast<const f4*>(cre + q * 8 + 4);
      *reinterpret_cast<f4*>(ai[b]) = *reinterpret_cast<const f4*>(cim + q * 8);
      *reinterpret_cast<f4*>(ai[b] + 4) = *reinterpret_cast<const f4*>(cim + q * 8 + 4);
      if constexpr (P_F64) {
        const double* p = static_cast<const double*>(g.p) + mrow[b] * np + ncol[b];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          pd[b][e] = *reinterpret_cast<const d2*>(p + 2 * e);
          pd[b][4 + e] = *reinterpret_cast<const d2*>(p + plane + 2 * e);
        }
      } else {
        const u16* p = static_cast<const u16*>(g.p) + chunk[b];
#pragma unroll
        for (int k = 0; k < 6; ++k) pw[b][k] = *reinterpret_cast<const u32x4*>(p + k * plane);
      }
      if constexpr (!FIRST) {
        const double* yr = g.y_re + mrow[b] * np + ncol[b];
        const double* yi = g.y_im + mrow[b] * np + ncol[b];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          yv[b][e] = *reinterpret_cast<const d2*>(yr + 2 * e);
          yv[b][4 + e] = *reinterpret_cast<const d2*>(yi + 2 * e);
        }
      }
    }
    // ---- arithmetic and stores ----
#pragma unroll
    for (int b = 0; b < B; ++b) {
      double pr[8], pi[8];  // P_{l-1} (X for the first product)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if constexpr (P_F64) {
          pr[e] = pd[b][e >> 1][e & 1];
          pi[e] = pd[b][4 + (e >> 1)][e & 1];
        } else {
          float s3[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            const uint32_t word = pw[b][k][e >> 1];
            s3[k] = bf16_val((u16)((e & 1) ? (word >> 16) : (word & 0xffffu)));
          }
          pr[e] = (double)(s3[0] + s3[1] + s3[2]);
          pi[e] = (double)(s3[3] + s3[4] + s3[5]);
        }
      }
      double* yr = g.y_re + mrow[b] * np + ncol[b];
      double* yi = g.y_im + mrow[b] * np + ncol[b];
      if constexpr (!TO_X) {
        // P_{l+1} = 2 acc - P_{l-1}, or P_1 = acc: stored as BF16X3, and its
        // stored value weighted into Y (Y = c_0 X + c_1 P_1 for the first)
        u32x4 w[NS];
        double vr8[8], vi8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double orr = FIRST ? (double)ar[b][e] : 2.0 * (double)ar[b][e] - pr[e];
          const double oii = FIRST ? (double)ai[b][e] : 2.0 * (double)ai[b][e] - pi[e];
          u16 hs[NS];
          split3((float)orr, hs[0], hs[1], hs[2]);
          split3((float)oii, hs[3], hs[4], hs[5]);
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            if (e & 1)
              w[k][e >> 1] |= (uint32_t)hs[k] << 16;
            else
              w[k][e >> 1] = hs[k];
          }
          vr8[e] = (double)(bf16_val(hs[0]) + bf16_val(hs[1]) + bf16_val(hs[2]));
          vi8[e] = (double)(bf16_val(hs[3]) + bf16_val(hs[4]) + bf16_val(hs[5]));
        }
        u16* o = static_cast<u16*>(g.o) + chunk[b];
#pragma unroll
        for (int k = 0; k < NS; ++k) *reinterpret_cast<u32x4*>(o + k * plane) = w[k];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          d2 vr, vi;
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const double tr = cr_ * vr8[e + u] - ci_ * vi8[e + u];
            const double ti = cr_ * vi8[e + u] + ci_ * vr8[e + u];
            if constexpr (FIRST) {
              vr[u] = g.c0r * pr[e + u] - g.c0i * pi[e + u] + tr;
              vi[u] = g.c0r * pi[e + u] + g.c0i * pr[e + u] + ti;
            } else {
              vr[u] = yv[b][e >> 1][u] + tr;
              vi[u] = yv[b][4 + (e >> 1)][u] + ti;
            }
          }
          *reinterpret_cast<d2*>(yr + e) = vr;
          *reinterpret_cast<d2*>(yi + e) = vi;
        }
      } else {  // X_k = ph (Y + c_L (2 acc - P_{L-1})), or ph (c_0 X + c_1 acc) when L = 1
        double* o = static_cast<double*>(g.o) + mrow[b] * np + ncol[b];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          d2 xr, xi;
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            double qr, qi, sr, si;
            if constexpr (FIRST) {
              qr = (double)ar[b][e + u];
              qi = (double)ai[b][e + u];
              sr = g.c0r * pr[e + u] - g.c0i * pi[e + u];
              si = g.c0r * pi[e + u] + g.c0i * pr[e + u];
            } else {
              qr = 2.0 * (double)ar[b][e + u] - pr[e + u];
              qi = 2.0 * (double)ai[b][e + u] - pi[e + u];
              sr = yv[b][e >> 1][u];
              si = yv[b][4 + (e >> 1)][u];
            }
            sr += cr_ * qr - ci_ * qi;
            si += cr_ * qi + ci_ * qr;
            xr[u] = g.phr * sr - g.phi * si;
            xi[u] = g.phr * si + g.phi * sr;
          }
          *reinterpret_cast<d2*>(o + e) = xr;
          *reinterpret_cast<d2*>(o + plane + e) = xi;
        }
      }
    }
  }
}

// Split-BF16 product on 32x32x16 matrix cores with NPC = 1, 2 or 3 pieces per
// operand: the piece pairs of weight at least 2^-8 (NPC - 1) of the leading one
// ((hh); (hh, hm, mh); (hh, hm, mh, hl, mm, lh)), so the product carries about
// 8, 16 or 24 significant bits. The stored matrices always hold three pieces;
// fewer pieces read fewer planes. KIND CHEB_FIRST / CHEB_FIRST_LAST take
// A = X (a BF16X3 copy) and p = X in FP64 for the c_0 X of the sum.
template <int BM, int BN, int WGM, int WGN, int KIND, bool P_F64, int NPC>
__global__ __launch_bounds__(WGM* WGN * 64) void cheb_bf3_kernel(Bf3Args g) {
  constexpr int NT = WGM * WGN * 64;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 32, FN = WTN / 32;
  constexpr int NL = 2 * NPC;                // stored planes read per operand (re, im pieces)
  constexpr int NP = 3 * NPC;                // planes in LDS (re, im, re + im pieces)
  constexpr int NS = BF3_PLANES;             // stored planes written by the epilogue
  constexpr int SA = BM * 32, SB = BN * 32;  // bytes per plane and k-block
  constexpr int STAGE = NP * (SA + SB);
  constexpr int NCA = 2 * BM;                // 16-byte chunks of A per plane and k-block
  constexpr int EPI = 2 * BM * BN * 4;       // FP32 Re, Im in k-blocked order
  constexpr int SMEM = (2 * STAGE > EPI) ? 2 * STAGE : EPI;
  constexpr bool FIRST = KIND == CHEB_FIRST || KIND == CHEB_FIRST_LAST;
  constexpr bool TO_X = KIND == CHEB_LAST || KIND == CHEB_FIRST_LAST;  // FP64 X_k out
  static_assert(2 * (BM + BN) == NT, "one 16-byte chunk column of A or B per thread");
  static_assert(FM >= 1 && FN >= 1 && WTM % 32 == 0 && WTN % 32 == 0, "wave tile");
  static_assert(NPC >= 1 && NPC <= 3, "pieces");
  static_assert(!FIRST || P_F64, "the first product reads X in FP64");

  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];

  int tm, tn;
  tile_coords(blockIdx.x, g.tiles_m, g.tiles_n, tm, tn);
  if (tm >= g.tiles_m) return;  // grid padding
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WGN, wn = wid % WGN;
  const long np = g.np, plane = g.plane;
  const int nk = g.np / 16;
  const long kstride = np * 16;  // words between consecutive k-blocks of a plane

  // This thread's chunk column: A (threads < NCA, whole waves) or B.
  const bool is_a = tid < NCA;
  const int cq = is_a ? tid : tid - NCA;
  const u16* src = is_a ? g.a + (long)m0 * 16 + cq * 8 : g.b + (long)n0 * 16 + cq * 8;
  const int ldst = is_a ? cq * 16 : NP * SA + cq * 16;
  const int pstep = is_a ? SA : SB;
  u32x4 st[NL];
  auto gload = [&](int kb) {
#pragma unroll
    for (int p = 0; p < NPC; ++p) {
      st[p] = *reinterpret_cast<const u32x4*>(src + p * plane + kb * kstride);
      st[NPC + p] = *reinterpret_cast<const u32x4*>(src + (3 + p) * plane + kb * kstride);
    }
  };
  auto lstore = [&](int buf) {
    unsigned char* d = smem + buf * STAGE + ldst;
#pragma unroll
    for (int p = 0; p < NL; ++p) *reinterpret_cast<u32x4*>(d + p * pstep) = st[p];
    u32x4 sum[NPC];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t o[NPC];
#pragma unroll
      for (int q = 0; q < NPC; ++q) o[q] = 0u;
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const int sh = 16 * hf;
        auto piece = [&](int p) { return bf16_val((u16)(st[p][w] >> sh)); };
        float re = piece(0), im = piece(NPC);
#pragma unroll
        for (int p = 1; p < NPC; ++p) {
          re += piece(p);
          im += piece(NPC + p);
        }
        u16 hs[NPC];
        split_n<NPC>(re + im, hs);
#pragma unroll
        for (int q = 0; q < NPC; ++q) o[q] |= (uint32_t)hs[q] << sh;
      }
#pragma unroll
      for (int q = 0; q < NPC; ++q) sum[q][w] = o[q];
    }
#pragma unroll
    for (int q = 0; q < NPC; ++q) *reinterpret_cast<u32x4*>(d + (NL + q) * pstep) = sum[q];
  };

  // Fragment offsets (bytes within a plane of a stage).
  int aoff[FM], boff[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int row = wm * WTM + i * 32 + (lane & 31);
    aoff[i] = row * 32 + 16 * ((lane >> 5) ^ ((row >> 3) & 1));
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int row = wn * WTN + j * 32 + (lane & 31);
    boff[j] = NP * SA + row * 32 + 16 * ((lane >> 5) ^ ((row >> 3) & 1));
  }

  f16v t1[FM][FN], t2[FM][FN], t3[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        t1[i][j][r] = 0.f;
        t2[i][j][r] = 0.f;
        t3[i][j][r] = 0.f;
      }

  gload(0);
  lstore(0);
  gload(nk > 1 ? 1 : 0);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int cur = kb & 1;
    const unsigned char* sb = smem + cur * STAGE;
    bf8 fb[NP][FN];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int p = 0; p < NP; ++p) fb[p][j] = *reinterpret_cast<const bf8*>(sb + p * SB + boff[j]);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      bf8 fa[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) fa[p] = *reinterpret_cast<const bf8*>(sb + p * SA + aoff[i]);
#define FQ_PAIR(pa, pb)                                                         \
  _Pragma("unroll") for (int j = 0; j < FN; ++j) {                              \
    t1[i][j] = mfma32_bf16(fa[pa], fb[pb][j], t1[i][j]);                        \
    t2[i][j] = mfma32_bf16(fa[NPC + pa], fb[NPC + pb][j], t2[i][j]);            \
    t3[i][j] = mfma32_bf16(fa[2 * NPC + pa], fb[2 * NPC + pb][j], t3[i][j]);    \
  }
      FQ_PAIR(0, 0)
      if constexpr (NPC >= 2) {
        FQ_PAIR(0, 1)
        FQ_PAIR(1, 0)
      }
      if constexpr (NPC >= 3) {
        FQ_PAIR(0, 2)
        FQ_PAIR(1, 1)
        FQ_PAIR(2, 0)
      }
#undef FQ_PAIR
    }
    // After this k-block's products: the next k-block (in registers since the
    // previous iteration) into the other buffer, last read before the previous
    // barrier, and the one after that into registers. Both unconditional, in
    // the block of the products, so that the staging arithmetic can run beside
    // them; the last iteration fills a buffer nobody reads.
    lstore(cur ^ 1);
    gload(kb + 2 < nk ? kb + 2 : nk - 1);
    __syncthreads();
  }

  // ---- epilogue ----
  // Re and Im to LDS, k-blocked order: element (row, col) of the tile at float
  // index ((col / 16) * BM + row) * 16 + 8 * slot + col % 8 with
  // slot = ((col / 8) & 1) ^ ((row / 8) & 1); real parts first, then imaginary.
  float* cre = reinterpret_cast<float*>(smem);
  float* cim = cre + BM * BN;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = wn * WTN + j * 32 + (lane & 31);
        const int slot = ((col >> 3) & 1) ^ ((row >> 3) & 1);
        const int f = ((col >> 4) * BM + row) * 16 + 8 * slot + (col & 7);
        cre[f] = t1[i][j][r] - t2[i][j][r];
        cim[f] = t3[i][j][r] - t1[i][j][r] - t2[i][j][r];
      }
  __syncthreads();

  bf3_tile_epilogue<BM, BN, NT, KIND, P_F64>(g, cre, cim, m0, n0, tid);
}

// ---------------------------------------------------------------------------------------------
// One- and two-piece products on 128 x 128 tiles with four waves of 64 x 64
// and the four real products of the complex one (Re = Ar Br - Ai Bi,
// Im = Ar Bi + Ai Br, -Ai by flipping sign bits in registers) instead of
// Gauss's three: per wave and k-block 4 NPC fragments of A and of B feed 16
// matrix-core operations per piece pair, a quarter of the LDS reads per
// operation of the 64 x 32 Gauss tiles, whose three operands also need the
// pieces of re + im staged. LDS holds only the 2 NPC stored planes of A and B,
// in two stages (32 or 64 KiB), so that two workgroups share a CU and cover
// each other's waits. The epilogue runs in two halves of 64 columns through
// 64 KiB of LDS.
// ---------------------------------------------------------------------------------------------
template <int KIND, bool P_F64, int NPC>
__global__ __launch_bounds__(256, 2) void cheb_x4_kernel(Bf3Args g) {
  constexpr int BM = 128, BN = 128, NT = 256, FM = 2, FN = 2;
  constexpr int NL = 2 * NPC;                // stored planes read per operand
  constexpr int SA = BM * 32, SB = BN * 32;  // bytes per plane and k-block
  constexpr int STAGE = NL * (SA + SB);
  constexpr int EPI = 2 * 128 * 64 * 4;      // FP32 Re, Im of one half, k-blocked order
  constexpr int SMEM = (2 * STAGE > EPI) ? 2 * STAGE : EPI;
  constexpr int NPAIR = NPC == 1 ? 1 : 3;
  constexpr bool FIRST = KIND == CHEB_FIRST || KIND == CHEB_FIRST_LAST;
  static_assert(NPC == 1 || NPC == 2, "pieces (three take the Gauss kernel)");
  static_assert(!FIRST || P_F64, "the first product reads X in FP64");
  static_assert(EPI == 2 * 2 * 4096 * 4, "two 128 x 32 groups of Re and of Im");
  static_assert(2 * BM == NT && 2 * BN == NT, "one 16-byte chunk of A and of B per thread");

  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];

  int tm, tn;
  tile_coords(blockIdx.x, g.tiles_m, g.tiles_n, tm, tn);
  if (tm >= g.tiles_m) return;  // grid padding
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const long np = g.np, plane = g.plane;
  const int nk = g.np / 16;
  const long kstride = np * 16;  // words between consecutive k-blocks of a plane

  // Staging: thread t copies 16-byte chunk t of A and of B in every plane.
  const u16* srca = g.a + (long)m0 * 16 + tid * 8;
  const u16* srcb = g.b + (long)n0 * 16 + tid * 8;
  u32x4 sta[NL], stb[NL];
  auto gload = [&](int kb) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const long po = (q < NPC ? q : 3 + q - NPC) * plane + kb * kstride;
      sta[q] = *reinterpret_cast<const u32x4*>(srca + po);
      stb[q] = *reinterpret_cast<const u32x4*>(srcb + po);
    }
  };
  auto lstore = [&](int buf) {
    unsigned char* d = smem + buf * STAGE + tid * 16;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      *reinterpret_cast<u32x4*>(d + q * SA) = sta[q];
      *reinterpret_cast<u32x4*>(d + NL * SA + q * SB) = stb[q];
    }
  };

  // Fragment offsets (bytes within a plane of a stage).
  int aoff[FM], boff[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int row = wm * 64 + i * 32 + (lane & 31);
    aoff[i] = row * 32 + 16 * ((lane >> 5) ^ ((row >> 3) & 1));
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int row = wn * 64 + j * 32 + (lane & 31);
    boff[j] = NL * SA + row * 32 + 16 * ((lane >> 5) ^ ((row >> 3) & 1));
  }
  // fragments [plane q][i]: q < NPC the real pieces, q >= NPC the imaginary ones
  bf8 fa[NL][FM], fb[NL][FN];
  auto fload = [&](int buf, bf8 (&xa)[NL][FM], bf8 (&xb)[NL][FN]) {
    const unsigned char* sb = smem + buf * STAGE;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
#pragma unroll
      for (int i = 0; i < FM; ++i) xa[q][i] = *reinterpret_cast<const bf8*>(sb + q * SA + aoff[i]);
#pragma unroll
      for (int j = 0; j < FN; ++j) xb[q][j] = *reinterpret_cast<const bf8*>(sb + q * SB + boff[j]);
    }
  };

  f16v cre[FM][FN], cim[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) cre[i][j][r] = cim[i][j][r] = 0.f;

  gload(0);
  lstore(0);
  gload(nk > 1 ? 1 : 0);
  lstore(1);
  gload(nk > 2 ? 2 : nk - 1);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    fload(kb & 1, fa, fb);
    bf8 ma[NPC][FM];  // -Ai pieces: flipped sign bits
#pragma unroll
    for (int q = 0; q < NPC; ++q)
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        u32x4 w = __builtin_bit_cast(u32x4, fa[NPC + q][i]);
        w ^= u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
        ma[q][i] = __builtin_bit_cast(bf8, w);
      }
    // piece pairs (pa, pb), the leading pair last
#pragma unroll
    for (int t = NPAIR - 1; t >= 0; --t) {
      constexpr int PA[3] = {0, 0, 1}, PB[3] = {0, 1, 0};
      const int pa = PA[t], pb = PB[t];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          cre[i][j] = mfma32_bf16(fa[pa][i], fb[pb][j], cre[i][j]);
          cim[i][j] = mfma32_bf16(fa[pa][i], fb[NPC + pb][j], cim[i][j]);
        }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          cre[i][j] = mfma32_bf16(ma[pa][i], fb[NPC + pb][j], cre[i][j]);
          cim[i][j] = mfma32_bf16(fa[NPC + pa][i], fb[pb][j], cim[i][j]);
        }
    }
    // k-block kb + 2 into the buffer kb came from, once every wave has read
    // its fragments there; the one after into registers
    __syncthreads();
    lstore(kb & 1);
    gload(kb + 3 < nk ? kb + 3 : nk - 1);
    __syncthreads();
  }

  // ---- epilogue in two halves: half h takes every wave's fragments j = h, the
  // 128 x 32 column groups n0 + 64 s + 32 h (s = wave column), so that each
  // wave keeps only the other half's accumulators while the first is written.
  // Re and Im to LDS, k-blocked order per group: element (row, col) of group s
  // at float index s * 4096 + ((col / 16) * 128 + row) * 16 + 8 * slot + col % 8
  // with slot = ((col / 8) & 1) ^ ((row / 8) & 1); real parts, then imaginary.
  float* ere = reinterpret_cast<float*>(smem);
  float* eim = ere + 2 * 128 * 32;  // two groups of 128 x 32 each
#pragma unroll
  for (int h = 0; h < FN; ++h) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = lane & 31;
        const int slot = ((col >> 3) & 1) ^ ((row >> 3) & 1);
        const int f = wn * 4096 + ((col >> 4) * 128 + row) * 16 + 8 * slot + (col & 7);
        ere[f] = cre[i][h][r];
        eim[f] = cim[i][h][r];
      }
    __syncthreads();
#pragma unroll
    for (int sgrp = 0; sgrp < 2; ++sgrp)
      bf3_tile_epilogue<128, 32, NT, KIND, P_F64, 1>(
          g, ere + sgrp * 4096, eim + sgrp * 4096, m0, n0 + 64 * sgrp + 32 * h, tid);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Split-BF16 product with FP64 accumulation, for the terms whose Bessel weight
// is too large for FP32 accumulators (P_1 of every step, and any term with a
// comparable weight). Each operand is split into three BF16 pieces; per FLUSH
// k-blocks of 16 columns the six kept piece pairs of the four real products
// (Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br) go into FP32 partial sums that
// start from zero, smallest pairs first within a k-block, and are then added
// into FP64 sums. The error of a product is then a few FP32 roundings of a
// partial sum over 16 FLUSH columns instead of one per accumulation over the
// whole contraction, so the product carries about 24 significant bits
// independently of N. Tile BM x 64
// (BM = 128 or 64), waves of 32 x 32; two LDS stages of the six stored planes. The
// epilogue works from the FP64 sums in registers: the Chebyshev sum Y takes
// the unrounded FP64 term, the stored P_{l+1} its BF16X3 rounding.
// ---------------------------------------------------------------------------------------------
template <int BM, int KIND, bool P_F64, int FLUSH>
__global__ __launch_bounds__(BM * 4) void cheb_acc_kernel(Bf3Args g) {
  constexpr int BN = 64, WGN = 2, NT = BM * 4;
  constexpr int NS = BF3_PLANES;             // 6 planes: re pieces, im pieces
  constexpr int SA = BM * 32, SB = BN * 32;  // bytes per plane and k-block
  constexpr int STAGE = NS * (SA + SB);
  constexpr int NCA = 2 * BM, NCB = 2 * BN;  // 16-byte chunk columns of A, B
  constexpr bool FIRST = KIND == CHEB_FIRST || KIND == CHEB_FIRST_LAST;
  constexpr bool TO_X = KIND == CHEB_LAST || KIND == CHEB_FIRST_LAST;
  static_assert(!FIRST || P_F64, "the first product reads X in FP64");

  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * STAGE];

  int tm, tn;
  tile_coords(blockIdx.x, g.tiles_m, g.tiles_n, tm, tn);
  if (tm >= g.tiles_m) return;  // grid padding
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WGN, wn = wid % WGN;
  const long np = g.np, plane = g.plane;
  const int nk = g.np / 16;
  const long kstride = np * 16;

  // Staging: threads [0, NCA) take a chunk column of A, [NCA, NCA + NCB) of B.
  const bool stager = tid < NCA + NCB;
  const bool is_a = tid < NCA;
  const int cq = is_a ? tid : tid - NCA;
  const u16* src = is_a ? g.a + (long)m0 * 16 + cq * 8 : g.b + (long)n0 * 16 + cq * 8;
  const int ldst = is_a ? cq * 16 : NS * SA + cq * 16;
  const int pstep = is_a ? SA : SB;
  u32x4 st[NS];
  auto gload = [&](int kb) {
    if (!stager) return;
#pragma unroll
    for (int p = 0; p < NS; ++p)
      st[p] = *reinterpret_cast<const u32x4*>(src + p * plane + kb * kstride);
  };
  auto lstore = [&](int buf) {
    if (!stager) return;
    unsigned char* d = smem + buf * STAGE + ldst;
#pragma unroll
    for (int p = 0; p < NS; ++p) *reinterpret_cast<u32x4*>(d + p * pstep) = st[p];
  };

  const int arow = wm * 32 + (lane & 31), brow = wn * 32 + (lane & 31);
  const int aoff = arow * 32 + 16 * ((lane >> 5) ^ ((arow >> 3) & 1));
  const int boff = NS * SA + brow * 32 + 16 * ((lane >> 5) ^ ((brow >> 3) & 1));

  double sre[16], sim[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) sre[r] = sim[r] = 0.0;
  f16v zero;
#pragma unroll
  for (int r = 0; r < 16; ++r) zero[r] = 0.f;

  gload(0);
  lstore(0);
  gload(nk > 1 ? 1 : 0);
  __syncthreads();
  f16v prr = zero, pii = zero, pim = zero;
  for (int kb0 = 0; kb0 < nk; kb0 += FLUSH) {
#pragma unroll
  for (int u = 0; u < FLUSH; ++u) {
    const int kb = kb0 + u;
    const unsigned char* sb = smem + (kb & 1) * STAGE;
    bf8 fa[NS], fb[NS];
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      fa[p] = *reinterpret_cast<const bf8*>(sb + p * SA + aoff);
      fb[p] = *reinterpret_cast<const bf8*>(sb + p * SB + boff);
    }
    // pairs (i, j) with i + j <= 2, the two hi x hi products last; Ar Br and
    // Ai Bi in separate partial sums (Re = their difference, taken in FP32 at
    // the flush), so no operand needs its sign flipped; the partial sums
    // start from zero every FLUSH k-blocks
    prr = mfma32_bf16(fa[2], fb[0], u == 0 ? zero : prr);
    pim = mfma32_bf16(fa[2], fb[3], u == 0 ? zero : pim);
    pii = mfma32_bf16(fa[5], fb[3], u == 0 ? zero : pii);
    pim = mfma32_bf16(fa[5], fb[0], pim);
#define FQ_ACC_PAIR(i, j)                          \
  prr = mfma32_bf16(fa[i], fb[j], prr);            \
  pim = mfma32_bf16(fa[i], fb[3 + (j)], pim);      \
  pii = mfma32_bf16(fa[3 + (i)], fb[3 + (j)], pii); \
  pim = mfma32_bf16(fa[3 + (i)], fb[j], pim);
    FQ_ACC_PAIR(1, 1)
    FQ_ACC_PAIR(0, 2)
    FQ_ACC_PAIR(1, 0)
    FQ_ACC_PAIR(0, 1)
    FQ_ACC_PAIR(0, 0)
#undef FQ_ACC_PAIR
    if (u == FLUSH - 1) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        sre[r] += (double)(prr[r] - pii[r]);
        sim[r] += (double)pim[r];
      }
    }
    lstore((kb & 1) ^ 1);
    gload(kb + 2 < nk ? kb + 2 : nk - 1);
    __syncthreads();
  }
  }

  // ---- epilogue, from the FP64 sums (lane: column n, rows of the 32 x 32 tile) ----
  const long n = n0 + wn * 32 + (lane & 31);
  const double cr_ = g.cr, ci_ = g.ci;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    // four rows at a time: keeps the scheduler from hoisting every row's loads
    // above the others' stores (that spills with the FP64 sums live)
    if (r % 4 == 0) __builtin_amdgcn_sched_barrier(0);
    const long m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const long idx = m * np + n;
    double pr, pi;
    load_c(g.p, P_F64 ? FMT_F64 : FMT_BF16X3, plane, m, n, np, pr, pi);
    double vr, vi;  // the term P_l (or the product for the first)
    if constexpr (FIRST) {
      vr = sre[r];
      vi = sim[r];
    } else {
      vr = 2.0 * sre[r] - pr;
      vi = 2.0 * sim[r] - pi;
    }
    double sr, si;
    if constexpr (FIRST) {
      sr = g.c0r * pr - g.c0i * pi + cr_ * vr - ci_ * vi;
      si = g.c0r * pi + g.c0i * pr + cr_ * vi + ci_ * vr;
    } else {
      sr = g.y_re[idx] + cr_ * vr - ci_ * vi;
      si = g.y_im[idx] + cr_ * vi + ci_ * vr;
    }
    if constexpr (TO_X) {
      double* o = static_cast<double*>(g.o);
      o[idx] = g.phr * sr - g.phi * si;
      o[plane + idx] = g.phr * si + g.phi * sr;
    } else {
      store_c(g.o, FMT_BF16X3, plane, m, n, np, vr, vi);
      g.y_re[idx] = sr;
      g.y_im[idx] = si;
    }
  }
}

// ---- launchers ---------------------------------------------------------------------------------

template <bool A_F64, class Epi>
hipError_t launch_f32(MixOperands op, int mrows, int np, Epi epi, hipStream_t s) {
  if (mrows % 128 == 0 && np % 128 == 0 && (long)mrows * np >= kBigTileElems) {
    op.tiles_m = mrows / 128;
    op.tiles_n = np / 128;
    hipLaunchKernelGGL((cheb_f32_kernel<128, 128, 32, 2, 4, A_F64, Epi>),
                       dim3(grid_rows(op.tiles_m) * op.tiles_n), dim3(512), 0, s, op, epi);
  } else if (mrows % 64 == 0 && np % 64 == 0) {
    op.tiles_m = mrows / 64;
    op.tiles_n = np / 64;
    hipLaunchKernelGGL((cheb_f32_kernel<64, 64, 32, 2, 2, A_F64, Epi>),
                       dim3(grid_rows(op.tiles_m) * op.tiles_n), dim3(256), 0, s, op, epi);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KIND, bool P_F64, int NPC>
hipError_t launch_bf3(const Bf3Args& g0, int mrows, hipStream_t s) {
  Bf3Args g = g0;
  const int np = g.np;
  if (mrows % 128 == 0 && np % 128 == 0 && (long)mrows * np >= kBigTileElems) {
    g.tiles_m = mrows / 128;
    g.tiles_n = np / 128;
    // one or two pieces: 64 x 64 wave tiles, four real products, two
    // workgroups per CU; three pieces: the Gauss form on 64 x 32 wave tiles
    // (measured faster there: the four-product form needs 96 KiB of LDS)
    if constexpr (NPC <= 2)
      hipLaunchKernelGGL((cheb_x4_kernel<KIND, P_F64, NPC>),
                         dim3(grid_rows(g.tiles_m) * g.tiles_n), dim3(256), 0, s, g);
    else
      hipLaunchKernelGGL((cheb_bf3_kernel<128, 128, 2, 4, KIND, P_F64, NPC>),
                         dim3(grid_rows(g.tiles_m) * g.tiles_n), dim3(512), 0, s, g);
  } else if (mrows % 64 == 0 && np % 64 == 0) {
    g.tiles_m = mrows / 64;
    g.tiles_n = np / 64;
    hipLaunchKernelGGL((cheb_bf3_kernel<64, 64, 2, 2, KIND, P_F64, NPC>),
                       dim3(grid_rows(g.tiles_m) * g.tiles_n), dim3(256), 0, s, g);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// k-blocks of 16 columns per FP32 partial sum of the FP64-sum product. Measured
// on the 4096-state model (whole build against the FP64 build; the product
// dominates the build's error), with Re in one partial sum: 1 -> e_col 3.7e-7,
// 3.59 ms per product; 2 -> 2.8e-7, 3.07 ms; 4 -> 2.7e-7, 2.94 ms; 8 -> 3.3e-7,
// 2.86 ms; 16 -> 4.5e-7, 2.85 ms. With Ar Br and Ai Bi in separate ones:
// 2 -> 1.9e-7, 2.84 ms; 4 -> 1.9e-7, 2.67 ms; 8 -> 2.4e-7, 2.60 ms.
constexpr int kAccFlush = 4;

template <int KIND, bool P_F64>
hipError_t launch_acc(const Bf3Args& g0, int mrows, hipStream_t s) {
  Bf3Args g = g0;
  if (mrows % 64 != 0 || g.np % 64 != 0) return hipErrorInvalidValue;
  g.tiles_n = g.np / 64;
  // 128-row tiles when they still give every CU a workgroup
  if (mrows % 128 == 0 && (long)(mrows / 128) * g.tiles_n >= 256) {
    g.tiles_m = mrows / 128;
    hipLaunchKernelGGL((cheb_acc_kernel<128, KIND, P_F64, kAccFlush>),
                       dim3(grid_rows(g.tiles_m) * g.tiles_n), dim3(512), 0, s, g);
  } else {
    g.tiles_m = mrows / 64;
    hipLaunchKernelGGL((cheb_acc_kernel<64, KIND, P_F64, kAccFlush>),
                       dim3(grid_rows(g.tiles_m) * g.tiles_n), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// One kind and P_{l-1} format of a split-BF16 product, in the given term format.
template <int KIND, bool P_F64>
hipError_t launch_term(const Bf3Args& g, int tf, int mrows, hipStream_t s) {
  switch (tf) {
    case TF_ACC: return launch_acc<KIND, P_F64>(g, mrows, s);
    case TF_X3: return launch_bf3<KIND, P_F64, 3>(g, mrows, s);
    case TF_X2: return launch_bf3<KIND, P_F64, 2>(g, mrows, s);
    case TF_X1: return launch_bf3<KIND, P_F64, 1>(g, mrows, s);
  }
  return hipErrorInvalidValue;
}

// Split-BF16 product of one Chebyshev term in term format tf (TF_ACC .. TF_X1):
// A = P_l (or the BF16X3 copy of X for the first product) in BF16X3; P_{l-1}
// in BF16X3 or FP64 (X, read for c_0 X by the first product); output P_{l+1}
// in BF16X3, or X_k in FP64 for the last product.
hipError_t dispatch_bf3(const ChebTermX& t, int tf, int mrows, int np, hipStream_t s) {
  if (t.a_fmt != FMT_BF16X3 || (t.p_fmt != FMT_BF16X3 && t.p_fmt != FMT_F64))
    return hipErrorInvalidValue;
  Bf3Args g{};
  g.a = static_cast<const u16*>(t.a);
  g.b = static_cast<const u16*>(t.b);
  g.p = t.p;
  g.o = t.o;
  g.y_re = t.y_re;
  g.y_im = t.y_im;
  g.plane = t.plane;
  g.np = np;
  g.c0r = t.c0r;
  g.c0i = t.c0i;
  g.cr = t.cr;
  g.ci = t.ci;
  g.phr = t.phr;
  g.phi = t.phi;
  const bool pf = t.p_fmt == FMT_F64;
  const bool to_x = t.kind == CHEB_LAST || t.kind == CHEB_FIRST_LAST;
  if (t.o_fmt != (to_x ? FMT_F64 : FMT_BF16X3)) return hipErrorInvalidValue;
  switch (t.kind) {
    case CHEB_FIRST:
      return pf ? launch_term<CHEB_FIRST, true>(g, tf, mrows, s) : hipErrorInvalidValue;
    case CHEB_FIRST_LAST:
      return pf ? launch_term<CHEB_FIRST_LAST, true>(g, tf, mrows, s) : hipErrorInvalidValue;
    case CHEB_MID:
      return pf ? launch_term<CHEB_MID, true>(g, tf, mrows, s)
                : launch_term<CHEB_MID, false>(g, tf, mrows, s);
    case CHEB_LAST:
      return pf ? launch_term<CHEB_LAST, true>(g, tf, mrows, s)
                : launch_term<CHEB_LAST, false>(g, tf, mrows, s);
  }
  return hipErrorInvalidValue;
}

template <class Epi>
hipError_t dispatch(const ChebTermX& t, int precision, int mrows, int np, Epi epi, hipStream_t s) {
  MixOperands op{t.a, t.b, t.plane, t.plane, np, np, 0, 0};
  // The first product of a step (A = X in FP64) runs on FP64 matrix cores and
  // reaches the product format through launch_to_product; these kernels take
  // the P_l in the product format.
  if (t.a_fmt == FMT_F64) return hipErrorInvalidValue;
  if (precision == FQ_FP32) return launch_f32<false>(op, mrows, np, epi, s);
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
    store_c(out, fmt, plane, i, k, ld, re, im);
  }
}

// BF16X3 variant: one thread per pair of columns (k, k + 1) of a row, in
// row-major order: a wave reads 1 KB contiguous from every FP64 plane and
// writes 4 bytes per lane into every BF16 plane (32-byte runs per k-block).
// Padding rows and columns stay zero.
__global__ void heff_bf3_kernel(const double* __restrict__ h0r, const double* __restrict__ h0i,
                                const double* __restrict__ vr, const double* __restrict__ vi,
                                const double* __restrict__ kr, const double* __restrict__ ki,
                                double a, double b, double beta, double inv_dE, long n, long np,
                                double* __restrict__ hr, double* __restrict__ hi,
                                u16* __restrict__ out) {
  const long pairs = np * np / 2, plane = np * np;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < pairs;
       q += (long)gridDim.x * blockDim.x) {
    const long i = q / (np / 2), k = 2 * (q % (np / 2)), idx = i * np + k;
    uint32_t wd[BF3_PLANES] = {};
    if (i < n && k < n) {
      const d2 h0r2 = *reinterpret_cast<const d2*>(h0r + idx);
      const d2 h0i2 = *reinterpret_cast<const d2*>(h0i + idx);
      const d2 vr2 = *reinterpret_cast<const d2*>(vr + idx);
      const d2 vi2 = *reinterpret_cast<const d2*>(vi + idx);
      const d2 kr2 = *reinterpret_cast<const d2*>(kr + idx);
      const d2 ki2 = *reinterpret_cast<const d2*>(ki + idx);
      d2 re2, im2;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        double re = 0.0, im = 0.0;
        if (k + e < n) {
          re = h0r2[e] + a * vr2[e] + b * kr2[e];
          im = h0i2[e] + a * vi2[e] + b * ki2[e];
          if (i == k + e) re -= beta;
          re *= inv_dE;
          im *= inv_dE;
        }
        re2[e] = re;
        im2[e] = im;
        u16 hs[BF3_PLANES];
        split3((float)re, hs[0], hs[1], hs[2]);
        split3((float)im, hs[3], hs[4], hs[5]);
#pragma unroll
        for (int p = 0; p < BF3_PLANES; ++p) wd[p] |= (uint32_t)hs[p] << (16 * e);
      }
      *reinterpret_cast<d2*>(hr + idx) = re2;
      *reinterpret_cast<d2*>(hi + idx) = im2;
    }
    u16* o = out + bf3_offset(i, k, np);  // columns k, k + 1: adjacent words
#pragma unroll
    for (int p = 0; p < BF3_PLANES; ++p) *reinterpret_cast<uint32_t*>(o + p * plane) = wd[p];
  }
}

// FP64 planes -> product format, one thread per pair of columns (k, k + 1) of a
// row in row-major order (16-byte reads per plane, 4-byte BF16 writes).
__global__ void to_product_kernel(const double* __restrict__ re, const double* __restrict__ im,
                                  void* __restrict__ out, int fmt, long mrows, long np) {
  const long pairs = mrows * np / 2, plane = np * np;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < pairs;
       q += (long)gridDim.x * blockDim.x) {
    const long i = q / (np / 2), k = 2 * (q % (np / 2)), idx = i * np + k;
    const d2 r2 = *reinterpret_cast<const d2*>(re + idx);
    const d2 i2 = *reinterpret_cast<const d2*>(im + idx);
    if (fmt == FMT_F32) {
      float* o = static_cast<float*>(out);
      *reinterpret_cast<f2*>(o + idx) = f2{(float)r2[0], (float)r2[1]};
      *reinterpret_cast<f2*>(o + plane + idx) = f2{(float)i2[0], (float)i2[1]};
    } else {
      uint32_t wd[BF3_PLANES] = {};
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        u16 hs[BF3_PLANES];
        split3((float)r2[e], hs[0], hs[1], hs[2]);
        split3((float)i2[e], hs[3], hs[4], hs[5]);
#pragma unroll
        for (int p = 0; p < BF3_PLANES; ++p) wd[p] |= (uint32_t)hs[p] << (16 * e);
      }
      u16* o = static_cast<u16*>(out) + bf3_offset(i, k, np);
#pragma unroll
      for (int p = 0; p < BF3_PLANES; ++p) *reinterpret_cast<uint32_t*>(o + p * plane) = wd[p];
    }
  }
}

}  // namespace

hipError_t launch_cheb_bf16(const ChebTermX& t, int term_fmt, int mrows, int np, hipStream_t s) {
  return dispatch_bf3(t, term_fmt, mrows, np, s);
}

hipError_t launch_cheb_mixed(const ChebTermX& t, int precision, int mrows, int np, hipStream_t s) {
  if (precision != FQ_FP32) return hipErrorInvalidValue;
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

hipError_t launch_adj_step_f32(const double* ar, int mrows, long plane_a, const float* ht,
                               double* sr, double* si, const double* lr, const double* li, double dr,
                               double di, double fac, int row_off, int np, hipStream_t s) {
  MixOperands op{ar, ht, plane_a, (long)np * np, np, np, 0, 0};
  EpiAdjStep e{sr, si, lr, li, dr, di, fac, np, row_off};
  return launch_f32<true>(op, mrows, np, e, s);
}

hipError_t launch_adj_dot_f32(const double* pr, long plane_a, const float* drive, long plane_b,
                              int ncols, const double* pbr, const double* pbi, double w,
                              double* out, int np, hipStream_t s) {
  MixOperands op{pr, drive, plane_a, plane_b, np, np, 0, 0};
  EpiAdjDot e{pbr, pbi, out, np, w};
  return launch_f32<true>(op, np, ncols, e, s);
}

__global__ void f64_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                  long count) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

hipError_t launch_f64_to_f32(const double* src, float* dst, long count, hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  long g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)g), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_heff_mixed(const double* h0r, const double* h0i, const double* vr,
                             const double* vi, const double* kr, const double* ki, double a,
                             double b, double beta, double dE, long n, long ld, double* hr,
                             double* hi, void* out, int precision, hipStream_t s) {
  if (precision == FQ_BF16X3) {
    long g = (ld * ld / 2 + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(heff_bf3_kernel, dim3((unsigned)g), dim3(256), 0, s, h0r, h0i, vr, vi, kr,
                       ki, a, b, beta, 1.0 / dE, n, ld, hr, hi, static_cast<u16*>(out));
    return hipGetLastError();
  }
  const int fmt = FMT_F32;
  long g = (n * ld + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(heff_mixed_kernel, dim3((unsigned)g), dim3(256), 0, s, h0r, h0i, vr, vi, kr,
                     ki, a, b, beta, 1.0 / dE, n, ld, hr, hi, out, fmt);
  return hipGetLastError();
}

hipError_t launch_to_product(const double* re, const double* im, void* out, int fmt, long mrows,
                             long np, hipStream_t s) {
  if (mrows < 1 || mrows > np || np % 2 || (fmt != FMT_F32 && fmt != FMT_BF16X3))
    return hipErrorInvalidValue;
  long g = (mrows * np / 2 + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(to_product_kernel, dim3((unsigned)g), dim3(256), 0, s, re, im, out, fmt,
                     mrows, np);
  return hipGetLastError();
}

}  // namespace fq
