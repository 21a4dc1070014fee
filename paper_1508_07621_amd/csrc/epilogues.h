// Epilogues of the adjoint (reverse-sweep) products, shared by the FP64 and
// the FP32 product kernels: both call them with the tile element (m, n) and
// the accumulated complex value, and call finish() once per thread at the end.
#pragma once

#include <hip/hip_runtime.h>

namespace fq {

// One reverse term: with acc = Ht * (A rows), in place over the output stack
// (which holds P_{l+1} over Pbar_{l+2}):
//   rows < np:   P_{l-1} = 2 acc - P_{l+1}                    (backward recurrence)
//   rows >= np:  Pbar_l  = fac acc - Pbar_{l+2} + d * Lambda  (adjoint recurrence)
struct EpiAdjStep {
  double* sr;  // output stack planes (2np x np each)
  double* si;
  const double* lr;  // Lambda (np x np)
  const double* li;
  double dr, di;  // d = conj(phase c_l)
  double fac;     // 2, or 1 for l = 0
  long ld;        // np
  int row_off;    // 0, or np when only the adjoint half is launched
  __device__ __forceinline__ void operator()(int m, int n, double ar, double ai) const {
    const long mg = (long)m + row_off;
    const long idx = mg * ld + n;
    if (mg < ld) {
      sr[idx] = 2.0 * ar - sr[idx];
      si[idx] = 2.0 * ai - si[idx];
    } else {
      const long li_ = (mg - ld) * ld + n;
      const double xr = lr[li_], xi = li[li_];
      sr[idx] = fac * ar - sr[idx] + dr * xr - di * xi;
      si[idx] = fac * ai - si[idx] + dr * xi + di * xr;
    }
  }
  __device__ __forceinline__ void finish() const {}
};

// Gradient contraction of one term against the stacked drive block
// [B_0; B_1; ...] (each np rows): acc(j, i) = (B_q P_l)(i', j) for
// q = i / np, i' = i mod np; accumulates w Re <Pbar_{l+1}, B_q P_l> into out[q].
// np is a multiple of the tile width, so the columns of one wave's tile lie in
// one block and a wave adds a single partial sum.
struct EpiAdjDot {
  const double* pbr;  // Pbar_{l+1} (np x np)
  const double* pbi;
  double* out;
  long ld;
  double w;
  double acc = 0.0;
  long q = 0;
  __device__ __forceinline__ void operator()(int m, int n, double ar, double ai) {
    q = n / ld;
    const long idx = (long)m * ld + (n - q * ld);
    acc += pbr[idx] * ar + pbi[idx] * ai;  // Re(conj(pbar) * acc)
  }
  __device__ void finish() {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(out + q, w * acc);
  }
};

}  // namespace fq
