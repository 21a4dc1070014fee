// Device-side storage formats of complex planes (see Fmt in internal.h):
// BF16 three-piece splitting and element load / store in any format.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace fq {

// Output tile of workgroup `bid` in a tiles_m x tiles_n grid. Workgroups are
// dispatched round-robin over the 8 XCDs (XCD = bid % 8), and each XCD has its
// own L2. XCD x owns the tile rows [x r, (x+1) r), r = grid_rows / 8, and walks
// them column by column with all r rows interleaved: the ~32 workgroups resident
// on one XCD then cover r rows and a few columns, so they stream r A panels and
// a few B panels, which its L2 can hold, instead of one distinct panel pair
// each. When tiles_m is not a multiple of 8 but large, the grid is padded to
// the next multiple (grid_rows) and the padding workgroups (tm >= tiles_m)
// return at once; small odd grids keep row-major order.
__host__ __device__ __forceinline__ int grid_rows(int tiles_m) {
  if (tiles_m % 8 == 0 || tiles_m < 64) return tiles_m;
  return (tiles_m + 7) / 8 * 8;
}
__device__ __forceinline__ void tile_coords(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int tp = grid_rows(tiles_m);
  if (tp % 8 == 0) {
    const int x = bid % 8, local = bid / 8, r = tp / 8;
    tm = x * r + local % r;
    tn = local / r;
  } else {
    tm = bid / tiles_n;
    tn = bid % tiles_n;
  }
}

// 128 x 128 output tiles only when they make at least 256 workgroups (one per
// CU); smaller products take 64 x 64 tiles so that every CU has work.
constexpr long kBigTileElems = 256L * 128 * 128;

typedef uint16_t u16;

__device__ __forceinline__ u16 bf16_bits(__bf16 v) { return __builtin_bit_cast(u16, v); }
__device__ __forceinline__ float bf16_val(u16 b) { return (float)__builtin_bit_cast(__bf16, b); }

// x ~ hi + mid + lo, each piece the BF16 rounding (to nearest even) of what the
// previous ones left; the three pieces carry about 24 significant bits.
__device__ __forceinline__ void split3(float x, u16& h, u16& m, u16& l) {
  const __bf16 bh = (__bf16)x;
  const float r1 = x - (float)bh;
  const __bf16 bm = (__bf16)r1;
  const float r2 = r1 - (float)bm;
  h = bf16_bits(bh);
  m = bf16_bits(bm);
  l = bf16_bits((__bf16)r2);
}

// BF16X3 matrices have six planes of 16-bit words: the hi, mid and lo pieces
// of the real part and of the imaginary part. They are stored k-blocked: each plane of an np x np
// matrix holds
// np/16 slices, one per block of 16 columns k; slice kb holds the np rows in
// order, 32 bytes per row (columns 16 kb .. 16 kb + 15), so the rows a
// workgroup stages for one k-block are one contiguous run. Within a row the
// two 8-column halves are swapped when bit 3 of the row index is set, which
// makes the 16-byte fragment reads of the 32x32 matrix-core tiles free of LDS
// bank conflicts. Offset of element (m, k) within plane 0, in 16-bit words:
__host__ __device__ __forceinline__ long bf3_offset(long m, long k, long np) {
  const long half = ((k >> 3) & 1) ^ ((m >> 3) & 1);
  return ((k >> 4) * np + m) * 16 + half * 8 + (k & 7);
}

// Element (m, n) of planar matrices with row stride ld (plane = ld * ld
// elements per plane) in the given format.
__device__ __forceinline__ void load_c(const void* base, int fmt, long plane, long m, long n,
                                       long ld, double& re, double& im) {
  if (fmt == FMT_F64) {
    const double* p = static_cast<const double*>(base);
    re = p[m * ld + n];
    im = p[plane + m * ld + n];
  } else if (fmt == FMT_F32) {
    const float* p = static_cast<const float*>(base);
    re = p[m * ld + n];
    im = p[plane + m * ld + n];
  } else {
    const u16* p = static_cast<const u16*>(base) + bf3_offset(m, n, ld);
    re = (double)(bf16_val(p[0]) + bf16_val(p[plane]) + bf16_val(p[2 * plane]));
    im = (double)(bf16_val(p[3 * plane]) + bf16_val(p[4 * plane]) + bf16_val(p[5 * plane]));
  }
}

// Store (re, im) in the given format and return in (re, im) the value the
// storage now holds.
__device__ __forceinline__ void store_c(void* base, int fmt, long plane, long m, long n, long ld,
                                        double& re, double& im) {
  if (fmt == FMT_F64) {
    double* p = static_cast<double*>(base);
    p[m * ld + n] = re;
    p[plane + m * ld + n] = im;
  } else if (fmt == FMT_F32) {
    float* p = static_cast<float*>(base);
    const float r = (float)re, i = (float)im;
    p[m * ld + n] = r;
    p[plane + m * ld + n] = i;
    re = r;
    im = i;
  } else {
    u16* p = static_cast<u16*>(base) + bf3_offset(m, n, ld);
    u16 h, md, l;
    split3((float)re, h, md, l);
    p[0] = h;
    p[plane] = md;
    p[2 * plane] = l;
    re = (double)(bf16_val(h) + bf16_val(md) + bf16_val(l));
    split3((float)im, h, md, l);
    p[3 * plane] = h;
    p[4 * plane] = md;
    p[5 * plane] = l;
    im = (double)(bf16_val(h) + bf16_val(md) + bf16_val(l));
  }
}

}  // namespace fq
