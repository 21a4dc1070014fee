// Tridiagonal operators (the Bose-Hubbard dimer of Sec. 4 in its Fock basis):
// the whole chain of single-step propagators for one state column runs inside
// one workgroup, with every term of every step held in registers.
//
// Step s uses Ht_s = D_s G_s D_s^+ with D_s = diag(w_s) unit gauge factors and
// G_s real symmetric tridiagonal (diagonal d_i, couplings g_i = |Ht_s[i][i+1]|),
// so the Chebyshev polynomial of Ht_s is D_s p(G_s) D_s^+. A real G_s acts on
// the real and imaginary parts of a state independently: one group of waves
// runs the recurrence P_{l+1} = 2 G P_l - P_{l-1} on the real part, another on
// the imaginary part, each lane holding R consecutive rows of P_{l-1}, P_l and
// of its share of the Chebyshev sum. Neighbour rows come from adjacent lanes by
// shuffles (and across waves through LDS when a part spans several waves).
// The two halves of the sum meet in LDS once per step, where the step phase
// and the change of gauge D_{s+1}^+ D_s are applied. The rows of G_s are
// formed in registers from H0, Hmod and the step scalars (a_s, b_s).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fq {
namespace {

constexpr int kMaxWaves = 8;  // waves per part

// Whole-wave DPP shifts by one lane; the lane without a source gets +0.0.
__device__ __forceinline__ double from_prev_lane(double v) {  // lane l <- lane l-1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_next_lane(double v) {  // lane l <- lane l+1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// coef, tape and snap come as separate restrict-qualified arguments so that the
// checkpoint and snapshot stores inside the step loop cannot be taken to alias
// the coefficient table, which then stays on scalar loads.
// Complex state elements of the user blocks: complex128, or complex64 when c64.
__device__ __forceinline__ void load_state(const void* base, long idx, int c64, double& re,
                                           double& im) {
  if (c64) {
    const float2 v = reinterpret_cast<const float2*>(base)[idx];
    re = v.x;
    im = v.y;
  } else {
    const double2 v = reinterpret_cast<const double2*>(base)[idx];
    re = v.x;
    im = v.y;
  }
}
// One part (0 = real, 1 = imaginary) of element idx.
__device__ __forceinline__ void store_part(void* base, long idx, int part, int c64, double v) {
  if (c64)
    reinterpret_cast<float*>(base)[2 * idx + part] = (float)v;
  else
    reinterpret_cast<double*>(base)[2 * idx + part] = v;
}

template <int R, int MAXT, bool MULTI>
__global__ __launch_bounds__(MAXT) void tridiag_gauge_kernel(TridiagJob job, int G,
                                                             const double2* __restrict__ coef,
                                                             double* __restrict__ tape,
                                                             double* __restrict__ snap) {
  extern __shared__ double ysh[];  // [part][lane in part][r][2]
  __shared__ double halo[2][2][2][kMaxWaves];  // [parity][part][0 first row, 1 last row][wave]

  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int part = wid / G, w = wid % G;
  const int pl = w * 64 + lane;  // lane index within its part
  const long col = blockIdx.x;
  const long n = job.n;
  const long base = (long)pl * R;
  const double sgn = part == 0 ? 1.0 : -1.0;
  const double2* gauge = reinterpret_cast<const double2*>(job.gauge);
  const double2* h0o = reinterpret_cast<const double2*>(job.h0_off);

  double pa[R], pb[R];  // the two most recent terms (roles alternate)
  double ys[R], yo[R];  // share of the sum: ys -> this part's component, yo -> the other one
  double d2[R], g2[R];  // 2 G: diagonal, coupling to the next row
  double gm2 = 0.0;     // 2 G coupling of row base-1 to row base

  // X~ = D_{k0}^+ X, this part's component
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    double v = 0.0;
    if (i < n) {
      double xr, xi;
      if (job.x0) {
        load_state(job.x0, i * job.ld_x0 + col, job.c64, xr, xi);
      } else {
        xr = (i == col) ? 1.0 : 0.0;
        xi = 0.0;
      }
      const double2 g = gauge[(long)job.k0 * n + i];
      v = part == 0 ? g.x * xr + g.y * xi : g.x * xi - g.y * xr;  // conj(w) x
      if (tape && job.k0 % job.ckpt == 0)  // checkpoint of X_{k0} (plain frame)
        tape[2 * (((long)(job.k0 / job.ckpt) * job.ncols + col) * n + i) + part] =
            part == 0 ? xr : xi;
    }
    pa[r] = v;
  }

  int parity = 0;
  auto neighbours = [&](const double* v, double& up, double& dn) {
    up = from_prev_lane(v[R - 1]);
    dn = from_next_lane(v[0]);
    if constexpr (MULTI) {  // wave ends exchange through LDS
      if (lane == 0) halo[parity][part][0][w] = v[0];
      if (lane == 63) halo[parity][part][1][w] = v[R - 1];
      __syncthreads();
      const double hu = (w > 0) ? halo[parity][part][1][w - 1] : 0.0;
      const double hd = (w + 1 < G) ? halo[parity][part][0][w + 1] : 0.0;
      up = (lane == 0) ? hu : up;
      dn = (lane == 63) ? hd : dn;
      parity ^= 1;
    }
  };
  // nw = 2 G v - nw (in place over the older term). The two edge rows, which
  // take the neighbour lanes' values, go first: their inputs (the previous
  // term's edge rows) are then the oldest results in flight, and the shifted
  // values of this term's edges are ready long before the next term needs them.
  auto advance = [&](const double* v, double* nw) {
    double up, dn;
    neighbours(v, up, dn);
    {
      double t = fma(d2[0], v[0], -nw[0]);
      t = fma(gm2, up, t);
      nw[0] = fma(g2[0], (R > 1) ? v[1] : dn, t);
    }
    if constexpr (R > 1) {
      double t = fma(d2[R - 1], v[R - 1], -nw[R - 1]);
      t = fma(g2[R - 2], v[R - 2], t);
      nw[R - 1] = fma(g2[R - 1], dn, t);
    }
#pragma unroll
    for (int r = 1; r < R - 1; ++r) {
      double t = fma(d2[r], v[r], -nw[r]);
      t = fma(g2[r - 1], v[r - 1], t);
      nw[r] = fma(g2[r], v[r + 1], t);
    }
  };
  // c_l P_l into the sum: even l has real c_l (this component), odd l imaginary
  auto acc_even = [&](const double* p, double c) {
#pragma unroll
    for (int r = 0; r < R; ++r) ys[r] = fma(c, p[r], ys[r]);
  };
  auto acc_odd = [&](const double* p, double c) {
#pragma unroll
    for (int r = 0; r < R; ++r) yo[r] = fma(c, p[r], yo[r]);
  };

  const int L = job.L;
  for (int s = job.k0; s < job.k1; ++s) {
    const double a = job.ab[2 * s], b = job.ab[2 * s + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      d2[r] = 0.0;
      g2[r] = 0.0;
      if (i < n) {
        const double vi = job.v_diag[i];
        d2[r] = 2.0 * (job.h0_diag[i] + a * vi - job.beta) * job.inv_dE;
        if (i + 1 < n) {
          const double2 h = h0o[i];
          const double q = b * (job.v_diag[i + 1] - vi);
          g2[r] = 2.0 * sqrt((h.x * h.x + h.y * h.y) * (1.0 + q * q)) * job.inv_dE;
        }
      }
    }
    gm2 = 0.0;
    if (base >= 1 && base < n) {
      const double2 h = h0o[base - 1];
      const double q = b * (job.v_diag[base] - job.v_diag[base - 1]);
      gm2 = 2.0 * sqrt((h.x * h.x + h.y * h.y) * (1.0 + q * q)) * job.inv_dE;
    }

    // l = 0, 1: P_0 = X~ (in pa), P_1 = G X~ (into pb)
    {
      const double c0 = coef[0].x, c1 = sgn * coef[1].y;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        pb[r] = 0.0;
        ys[r] = c0 * pa[r];
        yo[r] = 0.0;
      }
      advance(pa, pb);
#pragma unroll
      for (int r = 0; r < R; ++r) pb[r] *= 0.5;
      acc_odd(pb, c1);
    }
    // l = 2 .. L in pairs: P_{l} over P_{l-2}
    int l = 2;
    for (; l + 1 <= L; l += 2) {
      advance(pb, pa);  // P_l (even) into pa
      acc_even(pa, coef[l].x);
      advance(pa, pb);  // P_{l+1} (odd) into pb
      acc_odd(pb, sgn * coef[l + 1].y);
    }
    const bool last_in_a = (l <= L);
    if (last_in_a) {
      advance(pb, pa);
      acc_even(pa, coef[l].x);
    }

    // both halves of Y meet: X~_next = phase * w_s * conj(w_{s+1}) * Y (or
    // phase * w_s * Y after the last step); this part keeps its component.
    const bool final_step = (s + 1 == job.k1);
    const bool ckpt_step = tape && !final_step && (s + 1) % job.ckpt == 0;
    const bool snap_step = snap && (s + 1 - job.k0) % job.snap_every == 0;
    const long snap_j = snap_step ? (s + 1 - job.k0) / job.snap_every - 1 : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double* slot = ysh + (((long)part * G * 64 + pl) * R + r) * 2;
      slot[0] = ys[r];
      slot[1] = yo[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      const double* other = ysh + (((long)(1 - part) * G * 64 + pl) * R + r) * 2;
      // component sums: this part's own component and the other component
      const double own = ys[r] + other[1];
      const double oth = yo[r] + other[0];
      const double yr = part == 0 ? own : oth, yi = part == 0 ? oth : own;
      double v = 0.0;
      if (i < n) {
        const double2 ws = gauge[(long)s * n + i];
        // rot = phase * w_s [* conj(w_{s+1})]
        double rr = job.phr * ws.x - job.phi * ws.y, ri = job.phr * ws.y + job.phi * ws.x;
        const double plain = part == 0 ? rr * yr - ri * yi : rr * yi + ri * yr;  // X_{s+1}
        if (ckpt_step)
          tape[2 * (((long)((s + 1) / job.ckpt) * job.ncols + col) * n + i) + part] = plain;
        if (snap_step) store_part(snap, (snap_j * n + i) * job.ncols + col, part, job.c64, plain);
        if (!final_step) {
          const double2 wn = gauge[(long)(s + 1) * n + i];
          const double tr = rr * wn.x + ri * wn.y, ti = ri * wn.x - rr * wn.y;
          rr = tr;
          ri = ti;
        }
        v = part == 0 ? rr * yr - ri * yi : rr * yi + ri * yr;
      }
      pa[r] = v;
    }
    __syncthreads();
  }

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    if (i < n) store_part(job.x_out, i * job.ld_out + col, part, job.c64, pa[r]);
  }
}

template <int R, int MAXT, bool MULTI>
hipError_t launch_r(const TridiagJob& job, int G, hipStream_t s) {
  const size_t shmem = sizeof(double) * 2 * (size_t)G * 64 * R * 2;
  hipLaunchKernelGGL((tridiag_gauge_kernel<R, MAXT, MULTI>), dim3((unsigned)job.ncols),
                     dim3(2 * G * 64), shmem, s, job, G,
                     reinterpret_cast<const double2*>(job.coef), job.tape, job.snap);
  return hipGetLastError();
}

// ---- columns longer than one workgroup holds: k-term passes over HBM ----------------------------
//
// A column is cut into blocks of B owned rows; a workgroup loads its block with
// K ghost rows on each side (1024 G rows: 16 per lane, G waves per part), runs
// at most K terms of one step in registers exactly as above, and writes back
// only its owned rows: after t terms the rows within t of a cut are stale, the
// owned ones are not. One wave per part (G = 1) is what the library launches:
// its waves never wait for each other inside a pass, and the third of the rows
// that are ghosts costs less than a barrier per term does with G = 2 or 4. Between launches the state lives in HBM in the gauge frame of
// the current step, as 8 planes of ncols x n16 doubles: role 0 = latest even
// term, role 1 = latest odd term, role 2 = the part's own share of the sum,
// role 3 = its share of the other component; plane index (role * 2 + part).
// Within a column, row i sits at (i mod 16) nq + i / 16, so a lane's 16 rows
// are one element of 16 unit-stride wave-wide accesses (B and K are multiples
// of 16, so a row keeps its lane slot r = i mod 16 in every block that reads
// it). At a step start role 0 holds X~ = D_s^+ X.

// Per-step rows of 2 Ht, the phase-weighted gauge phi w_s and w_{s+1}, in the
// interleaved layout; rows n .. n16-1 are zero.
__global__ __launch_bounds__(256) void tridiag_stream_step_kernel(TridiagJob job, int s, int last,
                                                                  long n16, double* out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n16) return;
  const long n = job.n, nq = n16 >> 4;
  const long at = (i & 15) * nq + (i >> 4);
  double d2 = 0.0, g2 = 0.0, wr = 0.0, wi = 0.0, nr = 1.0, ni = 0.0;
  if (i < n) {
    const double a = job.ab[2 * s], b = job.ab[2 * s + 1];
    const double vi = job.v_diag[i];
    d2 = 2.0 * (job.h0_diag[i] + a * vi - job.beta) * job.inv_dE;
    if (i + 1 < n) {
      const double2 h = reinterpret_cast<const double2*>(job.h0_off)[i];
      const double q = b * (job.v_diag[i + 1] - vi);
      g2 = 2.0 * sqrt((h.x * h.x + h.y * h.y) * (1.0 + q * q)) * job.inv_dE;
    }
    const double2 g = reinterpret_cast<const double2*>(job.gauge)[(long)s * n + i];
    wr = job.phr * g.x - job.phi * g.y;
    wi = job.phr * g.y + job.phi * g.x;
    if (!last) {
      const double2 gn = reinterpret_cast<const double2*>(job.gauge)[(long)(s + 1) * n + i];
      nr = gn.x;
      ni = gn.y;
    }
  }
  out[at] = d2;
  out[n16 + at] = g2;
  out[2 * n16 + at] = wr;
  out[3 * n16 + at] = wi;
  out[4 * n16 + at] = nr;
  out[5 * n16 + at] = ni;
}

template <int R, int G>
__global__ __launch_bounds__(512) void tridiag_stream_kernel(TridiagJob job, TridiagStream st,
                                                             const double2* __restrict__ coef,
                                                             const double* __restrict__ stc) {
  static_assert(R == 16, "the interleaved state layout assumes 16 rows per lane");
  static_assert(G >= 1 && G <= 4 && G <= kMaxWaves, "waves per part (512 threads at most)");
  extern __shared__ double ysh[];  // [part][r][lane in part][2]
  __shared__ double halo[2][2][2][kMaxWaves];

  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int part = wid / G, w = wid % G;
  const int pl = w * 64 + lane;
  const long col = blockIdx.x / st.nblk, blk = blockIdx.x % st.nblk;
  const long n = job.n, n16 = st.n16, nq = n16 >> 4;
  const long a0 = blk * st.B;                       // first owned row
  const long own_end = (a0 + st.B < n) ? a0 + st.B : n;
  const long q = (a0 - st.K) / 16 + pl;             // row group of this lane (may be < 0)
  const long base = q * 16;                         // global row of this lane's first row
  const double sgn = part == 0 ? 1.0 : -1.0;
  const long cn = col * n16;                        // column offset in a state plane
  auto plane_in = [&](int role, int pt) { return st.in + (role * 2 + pt) * st.plane + cn; };
  auto plane_out = [&](int role, int pt) { return st.out + (role * 2 + pt) * st.plane + cn; };
  auto at = [&](int r) { return (long)r * nq + q; };

  double pe[R], po[R];  // latest even and odd terms
  double ys[R], yo[R];
  double d2[R], g2[R];
  double gm2 = 0.0;
  const int s = st.s;

  // rows of 2 Ht for step s; the coupling above the first row is row base - 1's
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    const bool in_col = i >= 0 && i < n;
    d2[r] = in_col ? stc[at(r)] : 0.0;
    g2[r] = in_col ? stc[n16 + at(r)] : 0.0;
  }
  if (base >= 1 && base < n) gm2 = stc[n16 + (long)(R - 1) * nq + q - 1];

  // load
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    const bool in_col = i >= 0 && i < n;
    const bool owned = i >= a0 && i < own_end;
    double e = 0.0, o = 0.0, y1 = 0.0, y2 = 0.0;
    if (in_col) {
      if (st.l0 == 0 && st.first_step) {
        double xr, xi;
        if (job.x0) {
          load_state(job.x0, i * job.ld_x0 + col, job.c64, xr, xi);
        } else {
          xr = (i == col) ? 1.0 : 0.0;
          xi = 0.0;
        }
        const double2 g = reinterpret_cast<const double2*>(job.gauge)[(long)s * n + i];
        e = part == 0 ? g.x * xr + g.y * xi : g.x * xi - g.y * xr;  // conj(w) x
      } else {
        e = plane_in(0, part)[at(r)];
        if (st.l0 > 0) {
          o = plane_in(1, part)[at(r)];
          if (owned) {
            y1 = plane_in(2, part)[at(r)];
            y2 = plane_in(3, part)[at(r)];
          }
        }
      }
    }
    pe[r] = e;
    po[r] = o;
    ys[r] = y1;
    yo[r] = y2;
  }

  // Neighbour values of the latest term: row base - 1 (up) and row base + R (dn).
  // post() starts their exchange as soon as the term's two edge rows are final
  // (lane shifts, and the wave ends through LDS); complete() waits for the other
  // waves and picks up the wave ends. advance() computes the edge rows first and
  // the interior rows between the two, so the exchange overlaps the interior.
  int parity = 0;
  double up = 0.0, dn = 0.0;
  auto post = [&](const double* v) {
    up = from_prev_lane(v[R - 1]);
    dn = from_next_lane(v[0]);
    if constexpr (G > 1) {
      if (lane == 0) halo[parity][part][0][w] = v[0];
      if (lane == 63) halo[parity][part][1][w] = v[R - 1];
    }
  };
  auto complete = [&]() {
    if constexpr (G > 1) {
      __syncthreads();
      const double hu = (w > 0) ? halo[parity][part][1][w - 1] : 0.0;
      const double hd = (w + 1 < G) ? halo[parity][part][0][w + 1] : 0.0;
      up = (lane == 0) ? hu : up;
      dn = (lane == 63) ? hd : dn;
    } else {
      up = (lane == 0) ? 0.0 : up;
      dn = (lane == 63) ? 0.0 : dn;
    }
    parity ^= 1;
  };
  auto advance = [&](const double* v, double* nw) {  // nw = 2 Ht v - nw
    {
      double t = fma(d2[0], v[0], -nw[0]);
      t = fma(gm2, up, t);
      nw[0] = fma(g2[0], v[1], t);
    }
    {
      double t = fma(d2[R - 1], v[R - 1], -nw[R - 1]);
      t = fma(g2[R - 2], v[R - 2], t);
      nw[R - 1] = fma(g2[R - 1], dn, t);
    }
    post(nw);
#pragma unroll
    for (int r = 1; r < R - 1; ++r) {
      double t = fma(d2[r], v[r], -nw[r]);
      t = fma(g2[r - 1], v[r - 1], t);
      nw[r] = fma(g2[r], v[r + 1], t);
    }
    complete();
  };

  int l = st.l0;
  // the latest term on entry: P_0 (l0 = 0) or P_{l0 - 1}, even in pe, odd in po
  if (l == 0 || (l & 1))
    post(pe);
  else
    post(po);
  complete();
  if (l == 0) {  // P_0 = X~ (in pe), P_1 = G X~ (into po)
    const double c0 = coef[0].x;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ys[r] = c0 * pe[r];
      yo[r] = 0.0;
      po[r] = 0.0;
    }
    l = 1;
    if (l < st.l1) {
      advance(pe, po);
      up *= 0.5;
      dn *= 0.5;
      const double c1 = sgn * coef[1].y;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        po[r] *= 0.5;
        yo[r] = fma(c1, po[r], yo[r]);
      }
      l = 2;
    }
  }
  if (l < st.l1 && (l & 1)) {  // odd start: P_l over P_{l-2} in po
    advance(pe, po);
    const double c = sgn * coef[l].y;
#pragma unroll
    for (int r = 0; r < R; ++r) yo[r] = fma(c, po[r], yo[r]);
    ++l;
  }
  for (; l + 1 < st.l1; l += 2) {  // even l into pe, odd l + 1 into po
    advance(po, pe);
    const double ce = coef[l].x;
#pragma unroll
    for (int r = 0; r < R; ++r) ys[r] = fma(ce, pe[r], ys[r]);
    advance(pe, po);
    const double co = sgn * coef[l + 1].y;
#pragma unroll
    for (int r = 0; r < R; ++r) yo[r] = fma(co, po[r], yo[r]);
  }
  if (l < st.l1) {
    advance(po, pe);
    const double ce = coef[l].x;
#pragma unroll
    for (int r = 0; r < R; ++r) ys[r] = fma(ce, pe[r], ys[r]);
  }

  if (st.l1 <= job.L) {  // mid-step: keep the two latest terms and the sum
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      if (i >= a0 && i < own_end) {
        plane_out(0, part)[at(r)] = pe[r];
        plane_out(1, part)[at(r)] = po[r];
        plane_out(2, part)[at(r)] = ys[r];
        plane_out(3, part)[at(r)] = yo[r];
      }
    }
    return;
  }

  // step end: both halves of Y meet; X~_{s+1} = phase w_s conj(w_{s+1}) Y, or
  // X = phase w_s Y after the last step (to x_out, row-major).
  const int np = G * 64;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double2* slot = reinterpret_cast<double2*>(ysh) + ((long)part * R + r) * np + pl;
    *slot = make_double2(ys[r], yo[r]);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    if (i < a0 || i >= own_end) continue;
    const double2 other = reinterpret_cast<const double2*>(ysh)[((long)(1 - part) * R + r) * np + pl];
    const double own = ys[r] + other.y;
    const double oth = yo[r] + other.x;
    const double yr = part == 0 ? own : oth, yi = part == 0 ? oth : own;
    double rr = stc[2 * n16 + at(r)], ri = stc[3 * n16 + at(r)];  // phase w_s
    if (job.snap && (s + 1 - job.k0) % job.snap_every == 0) {  // X_{s+1}, plain frame
      const long j = (s + 1 - job.k0) / job.snap_every - 1;
      store_part(job.snap, (j * n + i) * job.ncols + col, part, job.c64,
                 part == 0 ? rr * yr - ri * yi : rr * yi + ri * yr);
    }
    if (!st.last_step) {
      const double wr = stc[4 * n16 + at(r)], wi = stc[5 * n16 + at(r)];
      const double tr = rr * wr + ri * wi, ti = ri * wr - rr * wi;
      rr = tr;
      ri = ti;
    }
    const double v = part == 0 ? rr * yr - ri * yi : rr * yi + ri * yr;
    if (st.last_step)
      store_part(job.x_out, i * job.ld_out + col, part, job.c64, v);
    else
      plane_out(0, part)[at(r)] = v;
  }
}

template <int G>
hipError_t launch_stream_g(const TridiagJob& job, const TridiagStream& st, hipStream_t s) {
  constexpr int R = 16;
  // only a pass that ends its step exchanges the two halves of Y through LDS
  const size_t shmem = st.l1 > job.L ? sizeof(double) * 2 * (size_t)G * 64 * R * 2 : 0;
  const long grid = job.ncols * st.nblk;
  if (grid < 1 || grid > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((tridiag_stream_kernel<R, G>), dim3((unsigned)grid), dim3(2 * G * 64), shmem,
                     s, job, st, reinterpret_cast<const double2*>(job.coef), st.stepc);
  return hipGetLastError();
}

// ---- reverse sweep (gradient) ----------------------------------------------------------------
//
// One workgroup per state column, W waves, R consecutive rows per lane, complex
// values (real and imaginary parts side by side; no gauge: the operator is
// applied in its complex tridiagonal form). For every checkpoint segment, last
// first: the segment is recomputed forward from its tape entry, storing each
// step's input X_k and its last two terms P_{L-1}, P_L in the column's segment
// buffer; then the steps are reversed with the adjoint recurrence
//   Pbar_l = (2 - delta_l0) Ht Pbar_{l+1} - Pbar_{l+2} + conj(phase c_l) Lambda,
// the terms regenerated downwards by P_{l-1} = 2 Ht P_l - P_{l+1} (P_0 read
// back), and the contractions (2 - delta_l0) Re <Pbar_{l+1}, D P_l> for
// D = Hmod and D = K summed per wave and added to the step's accumulators.
// Lambda = Pbar_0 then enters the step before.
struct Cx {  // complex scalar helpers on (re, im) pairs
  __device__ static __forceinline__ void mul(double ar, double ai, double br, double bi,
                                             double& cr, double& ci) {
    cr = ar * br - ai * bi;
    ci = ar * bi + ai * br;
  }
};

template <int R, int W>
__global__ __launch_bounds__(W * 64) void tridiag_adjoint_kernel(TridiagAdjJob job) {
  __shared__ double halo[2][4][2][W];  // [parity][value][first row / last row][wave]

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long col = blockIdx.x;
  const long n = job.n;
  const long base = ((long)wid * 64 + lane) * R;
  const double2* h0o = reinterpret_cast<const double2*>(job.h0_off);
  const double2* coef = reinterpret_cast<const double2*>(job.coef);
  const double2* tape = reinterpret_cast<const double2*>(job.tape);
  double2* seg = reinterpret_cast<double2*>(job.seg);
  const long segcol = col * (long)job.ckpt * 3 * n;  // this column's segment buffer
  const int L = job.L;

  double lr[R], li[R];                 // Lambda
  double ar[R], ai[R], br[R], bi[R];   // two P terms
  double qr[R], qi[R], sr[R], si[R];   // two Pbar terms (Y in the forward recompute)
  double dd[R], er[R], ei[R], kr[R], ki[R], vv[R];
  double emr = 0.0, emi = 0.0, kmr = 0.0, kmi = 0.0;  // couplings from row base - 1

  // Lambda_M = Ubar column
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    lr[r] = li[r] = 0.0;
    vv[r] = 0.0;
    if (i < n) {
      load_state(job.u_bar, i * job.ncols + col, job.c64, lr[r], li[r]);
      vv[r] = job.v_diag[i];
    }
  }

  auto set_step = [&](int k) {
    const double a = job.ab[2 * k], b = job.ab[2 * k + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      dd[r] = er[r] = ei[r] = kr[r] = ki[r] = 0.0;
      if (i < n) {
        dd[r] = (job.h0_diag[i] + a * vv[r] - job.beta) * job.inv_dE;
        if (i + 1 < n) {
          const double2 h = h0o[i];
          const double dv = job.v_diag[i + 1] - vv[r], q = b * dv;
          er[r] = (h.x + h.y * q) * job.inv_dE;  // h (1 - i q) / dE
          ei[r] = (h.y - h.x * q) * job.inv_dE;
          kr[r] = h.y * dv;                      // K = -i h dv
          ki[r] = -h.x * dv;
        }
      }
    }
    emr = emi = kmr = kmi = 0.0;
    if (base >= 1 && base < n) {
      const double2 h = h0o[base - 1];
      const double dv = job.v_diag[base] - job.v_diag[base - 1], q = b * dv;
      emr = (h.x + h.y * q) * job.inv_dE;
      emi = (h.y - h.x * q) * job.inv_dE;
      kmr = h.y * dv;
      kmi = -h.x * dv;
    }
  };

  int parity = 0;
  // Neighbour values of up to two complex vectors: row base - 1 (u*) and base + R (d*).
  auto exchange = [&](const double* xr, const double* xi, const double* yr, const double* yi,
                      double nb[8]) {
    nb[0] = from_prev_lane(xr[R - 1]);
    nb[1] = from_prev_lane(xi[R - 1]);
    nb[2] = from_prev_lane(yr[R - 1]);
    nb[3] = from_prev_lane(yi[R - 1]);
    nb[4] = from_next_lane(xr[0]);
    nb[5] = from_next_lane(xi[0]);
    nb[6] = from_next_lane(yr[0]);
    nb[7] = from_next_lane(yi[0]);
    if constexpr (W > 1) {
      if (lane == 0) {
        halo[parity][0][0][wid] = xr[0];
        halo[parity][1][0][wid] = xi[0];
        halo[parity][2][0][wid] = yr[0];
        halo[parity][3][0][wid] = yi[0];
      }
      if (lane == 63) {
        halo[parity][0][1][wid] = xr[R - 1];
        halo[parity][1][1][wid] = xi[R - 1];
        halo[parity][2][1][wid] = yr[R - 1];
        halo[parity][3][1][wid] = yi[R - 1];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double hu = (wid > 0) ? halo[parity][q][1][wid - 1] : 0.0;
        const double hd = (wid + 1 < W) ? halo[parity][q][0][wid + 1] : 0.0;
        nb[q] = (lane == 0) ? hu : nb[q];
        nb[4 + q] = (lane == 63) ? hd : nb[4 + q];
      }
      parity ^= 1;
    }
  };
  // out = f Ht x - out + (cr + i ci) lam   (f = 1 or 2; cr = ci = 0 for no source)
  auto apply = [&](const double* xr, const double* xi, double ur, double ui, double dr_, double di_,
                   double f, double* or_, double* oi, double cr, double ci) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double lor = (r == 0) ? ur : xr[r - 1], loi = (r == 0) ? ui : xi[r - 1];
      const double hir = (r == R - 1) ? dr_ : xr[r + 1], hii = (r == R - 1) ? di_ : xi[r + 1];
      const double cer = (r == 0) ? emr : er[r - 1], cei = (r == 0) ? emi : ei[r - 1];
      // conj(e_{i-1}) x_{i-1} + e_i x_{i+1} + d_i x_i
      double hr = dd[r] * xr[r] + cer * lor + cei * loi + er[r] * hir - ei[r] * hii;
      double hi = dd[r] * xi[r] + cer * loi - cei * lor + er[r] * hii + ei[r] * hir;
      or_[r] = f * hr - or_[r] + (cr * lr[r] - ci * li[r]);
      oi[r] = f * hi - oi[r] + (cr * li[r] + ci * lr[r]);
    }
  };

  const int nseg = (job.M + job.ckpt - 1) / job.ckpt;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int k0 = sg * job.ckpt, k1 = (k0 + job.ckpt < job.M) ? k0 + job.ckpt : job.M;
    // ---- forward recompute of the segment from its checkpoint ----
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      ar[r] = ai[r] = 0.0;
      if (i < n) {
        const double2 x = tape[((long)sg * job.ncols + col) * n + i];
        ar[r] = x.x;
        ai[r] = x.y;
      }
    }
    for (int k = k0; k < k1; ++k) {
      set_step(k);
      double2* sx = seg + segcol + ((long)(k - k0) * 3) * n;  // X_k, P_{L-1}, P_L
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long i = base + r;
        if (i < n) sx[i] = make_double2(ar[r], ai[r]);
      }
      // P_0 in a, P_1 = Ht P_0 in b, Y (in q) = c0 P_0 + c1 P_1
      double nb[8];
      exchange(ar, ai, ar, ai, nb);
#pragma unroll
      for (int r = 0; r < R; ++r) br[r] = bi[r] = 0.0;
      apply(ar, ai, nb[0], nb[1], nb[4], nb[5], 1.0, br, bi, 0.0, 0.0);
      {
        const double2 c0 = coef[0], c1 = coef[1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          double t1r, t1i, t2r, t2i;
          Cx::mul(c0.x, c0.y, ar[r], ai[r], t1r, t1i);
          Cx::mul(c1.x, c1.y, br[r], bi[r], t2r, t2i);
          qr[r] = t1r + t2r;
          qi[r] = t1i + t2i;
        }
      }
      // P_{l+1} = 2 Ht P_l - P_{l-1}, alternating between a (even) and b (odd)
      for (int l = 1; l < L; ++l) {
        // P_l is in b for odd l (P_{l-1} in a is overwritten by P_{l+1}), in a for even l
        if (l & 1) {
          exchange(br, bi, br, bi, nb);
          apply(br, bi, nb[0], nb[1], nb[4], nb[5], 2.0, ar, ai, 0.0, 0.0);
        } else {
          exchange(ar, ai, ar, ai, nb);
          apply(ar, ai, nb[0], nb[1], nb[4], nb[5], 2.0, br, bi, 0.0, 0.0);
        }
        const double2 c = coef[l + 1];
        const bool in_a = (l & 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double pr = in_a ? ar[r] : br[r], pi = in_a ? ai[r] : bi[r];
          double tr, ti;
          Cx::mul(c.x, c.y, pr, pi, tr, ti);
          qr[r] += tr;
          qi[r] += ti;
        }
      }
      // P_L is in a if L even, else in b; P_{L-1} in the other
      const bool last_in_a = !(L & 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long i = base + r;
        if (i < n) {
          sx[n + i] = last_in_a ? make_double2(br[r], bi[r]) : make_double2(ar[r], ai[r]);
          sx[2 * n + i] = last_in_a ? make_double2(ar[r], ai[r]) : make_double2(br[r], bi[r]);
        }
      }
      // X_{k+1} = phase Y into a
#pragma unroll
      for (int r = 0; r < R; ++r) Cx::mul(job.phr, job.phi, qr[r], qi[r], ar[r], ai[r]);
    }
    // ---- reverse through the segment ----
    for (int k = k1 - 1; k >= k0; --k) {
      set_step(k);
      const double2* sx = seg + segcol + ((long)(k - k0) * 3) * n;
      // a = P_{L-1}, b = P_L; q = Pbar_L = d_L Lambda, s = Pbar_{L+1} = 0
      const double2 cL = coef[L];
      const double dLr = job.phr * cL.x - job.phi * cL.y, dLi = -(job.phr * cL.y + job.phi * cL.x);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long i = base + r;
        ar[r] = ai[r] = br[r] = bi[r] = 0.0;
        if (i < n) {
          const double2 pm = sx[n + i], pl = sx[2 * n + i];
          ar[r] = pm.x;
          ai[r] = pm.y;
          br[r] = pl.x;
          bi[r] = pl.y;
        }
        qr[r] = dLr * lr[r] - dLi * li[r];
        qi[r] = dLr * li[r] + dLi * lr[r];
        sr[r] = si[r] = 0.0;
      }
      double gv = 0.0, gk = 0.0;
      // one downward term: x = P_l, z = P_{l+1} (-> P_{l-1}); p = Pbar_{l+1}, o = Pbar_{l+2} (-> Pbar_l)
      auto down = [&](double* xr_, double* xi_, double* zr, double* zi, double* pr_, double* pi_,
                      double* or_, double* oi_, int l) {
        double nb[8];
        exchange(xr_, xi_, pr_, pi_, nb);
        const double w = (l >= 1) ? 2.0 : 1.0;
        // contractions with Hmod (diagonal) and K (tridiagonal, K_{i,i+1} = k_i)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          gv += w * vv[r] * (pr_[r] * xr_[r] + pi_[r] * xi_[r]);
          if (job.any_b) {
            const double lor = (r == 0) ? nb[0] : xr_[r - 1], loi = (r == 0) ? nb[1] : xi_[r - 1];
            const double hir = (r == R - 1) ? nb[4] : xr_[r + 1],
                         hii = (r == R - 1) ? nb[5] : xi_[r + 1];
            const double ckr = (r == 0) ? kmr : kr[r - 1], cki = (r == 0) ? kmi : ki[r - 1];
            // (K x)_i = conj(k_{i-1}) x_{i-1} + k_i x_{i+1}
            const double tr = ckr * lor + cki * loi + kr[r] * hir - ki[r] * hii;
            const double ti = ckr * loi - cki * lor + kr[r] * hii + ki[r] * hir;
            gk += w * (pr_[r] * tr + pi_[r] * ti);
          }
        }
        // Pbar_l = w Ht Pbar_{l+1} - Pbar_{l+2} + conj(phase c_l) Lambda
        const double2 cl = coef[l];
        const double dr = job.phr * cl.x - job.phi * cl.y, di = -(job.phr * cl.y + job.phi * cl.x);
        apply(pr_, pi_, nb[2], nb[3], nb[6], nb[7], w, or_, oi_, dr, di);
        // P_{l-1} = 2 Ht P_l - P_{l+1}; P_0 is read back
        if (l == 1) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const long i = base + r;
            zr[r] = zi[r] = 0.0;
            if (i < n) {
              const double2 x0 = sx[i];
              zr[r] = x0.x;
              zi[r] = x0.y;
            }
          }
        } else if (l >= 2) {
          apply(xr_, xi_, nb[0], nb[1], nb[4], nb[5], 2.0, zr, zi, 0.0, 0.0);
        }
      };
      int l = L - 1;
      for (; l >= 1; l -= 2) {
        down(ar, ai, br, bi, qr, qi, sr, si, l);      // P_l in a, P_{l-1} -> b; Pbar_l -> s
        down(br, bi, ar, ai, sr, si, qr, qi, l - 1);  // P_{l-1} in b; Pbar_{l-1} -> q
      }
      if (l == 0) {
        down(ar, ai, br, bi, qr, qi, sr, si, 0);      // Pbar_0 -> s
#pragma unroll
        for (int r = 0; r < R; ++r) {
          lr[r] = sr[r];
          li[r] = si[r];
        }
      } else {  // l == -1: Pbar_0 is in q
#pragma unroll
        for (int r = 0; r < R; ++r) {
          lr[r] = qr[r];
          li[r] = qi[r];
        }
      }
      // per-wave sums to the step's accumulators
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        gv += __shfl_xor(gv, o);
        gk += __shfl_xor(gk, o);
      }
      if (lane == 0) {
        atomicAdd(job.grad + 2 * k, gv);
        if (job.any_b) atomicAdd(job.grad + 2 * k + 1, gk);
      }
    }
  }
}

template <int R, int W>
hipError_t launch_adj_r(const TridiagAdjJob& job, hipStream_t s) {
  hipLaunchKernelGGL((tridiag_adjoint_kernel<R, W>), dim3((unsigned)job.ncols), dim3(W * 64), 0, s,
                     job);
  return hipGetLastError();
}

// ---- streamed reverse sweep ------------------------------------------------------------------
//
// For columns longer than one workgroup holds, the recurrences of
// tridiag_adjoint_kernel run one step at a time and at most K terms per
// launch. A workgroup holds a window of W*64*R consecutive rows of one column:
// the B rows it owns and K ghost rows on each side. Every term reads one
// neighbour row on each side, so after at most K terms the owned rows are still
// exact; they are written back and the next launch continues from them. Rows
// outside [0, n) are zero, as are their couplings, which is exact at the ends of
// the chain. Two kinds of pass:
//   forward (segment recompute): P_{lo+1} .. P_hi and the running sum Y of one
//     step, from P_0 = X_k when lo == 0; at hi == L it stores P_{L-1}, P_L and
//     X_{k+1} = phase Y for the reverse passes;
//   reverse: terms l = hi .. lo of the adjoint recurrence with P regenerated
//     downwards, the contractions over the owned rows added to the step's two
//     accumulators; at lo == 0 it stores Pbar_0, the Lambda of the step before.
// Both work in the gauge frame of the step, Ht = D G D^+ with D = diag(w) and
// G real symmetric tridiagonal (diagonal d_i, couplings g_i = |Ht[i][i+1]|), so
// every term applies real couplings: the terms are those of G on D^+ X, the
// step's output is phase D Y, Lambda enters as D^+ Lambda and leaves as
// D Pbar_0. Hmod is diagonal and unchanged by D; K becomes D^+ K D, whose
// couplings conj(w_i) k_i w_{i+1} stay complex.

// Per-window operator rows of one step and the neighbour exchange of the window.
template <int R, int W>
struct AdjWindow {
  double dd[R], gg[R], kr[R], ki[R], vv[R];  // G rows, D^+ K D couplings, Hmod
  double gm, kmr, kmi;                       // couplings from row base - 1
  double (*halo)[4][2][W];
  int parity, lane, wid;

  __device__ __forceinline__ void set(const TridiagAdjPass& p, long base) {
    const double2* h0o = reinterpret_cast<const double2*>(p.h0_off);
    const double2* w = reinterpret_cast<const double2*>(p.gauge);
    // coupling g_i = |h_i| sqrt(1 + q^2) / dE and, with b != 0, conj(w_i) k_i w_{i+1}
    // with k_i = -i h_i (v_{i+1} - v_i)
    auto coupling = [&](long i, double& g, double& tr, double& ti) {
      const double2 h = h0o[i];
      const double dv = p.v_diag[i + 1] - p.v_diag[i], q = p.b * dv;
      g = sqrt((h.x * h.x + h.y * h.y) * (1.0 + q * q)) * p.inv_dE;
      tr = ti = 0.0;
      if (p.any_b) {
        const double k_r = h.y * dv, k_i = -h.x * dv;
        const double2 w0 = w[i], w1 = w[i + 1];
        const double ur = k_r * w1.x - k_i * w1.y, ui = k_r * w1.y + k_i * w1.x;  // k w_{i+1}
        tr = w0.x * ur + w0.y * ui;                                               // conj(w_i) (.)
        ti = w0.x * ui - w0.y * ur;
      }
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      dd[r] = gg[r] = kr[r] = ki[r] = vv[r] = 0.0;
      if (i >= 0 && i < p.n) {
        vv[r] = p.v_diag[i];
        dd[r] = (p.h0_diag[i] + p.a * vv[r] - p.beta) * p.inv_dE;
        if (i + 1 < p.n) coupling(i, gg[r], kr[r], ki[r]);
      }
    }
    gm = kmr = kmi = 0.0;
    if (base >= 1 && base < p.n) coupling(base - 1, gm, kmr, kmi);
  }

  // Neighbour rows of two complex vectors: base - 1 (nb[0..3]) and base + R
  // (nb[4..7]); zero beyond the window.
  __device__ __forceinline__ void exchange(const double* xr, const double* xi, const double* yr,
                                           const double* yi,
                           double nb[8]) {
    nb[0] = from_prev_lane(xr[R - 1]);
    nb[1] = from_prev_lane(xi[R - 1]);
    nb[2] = from_prev_lane(yr[R - 1]);
    nb[3] = from_prev_lane(yi[R - 1]);
    nb[4] = from_next_lane(xr[0]);
    nb[5] = from_next_lane(xi[0]);
    nb[6] = from_next_lane(yr[0]);
    nb[7] = from_next_lane(yi[0]);
    if (lane == 0) {
      halo[parity][0][0][wid] = xr[0];
      halo[parity][1][0][wid] = xi[0];
      halo[parity][2][0][wid] = yr[0];
      halo[parity][3][0][wid] = yi[0];
    }
    if (lane == 63) {
      halo[parity][0][1][wid] = xr[R - 1];
      halo[parity][1][1][wid] = xi[R - 1];
      halo[parity][2][1][wid] = yr[R - 1];
      halo[parity][3][1][wid] = yi[R - 1];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double hu = (wid > 0) ? halo[parity][q][1][wid - 1] : 0.0;
      const double hd = (wid + 1 < W) ? halo[parity][q][0][wid + 1] : 0.0;
      nb[q] = (lane == 0) ? hu : nb[q];
      nb[4 + q] = (lane == 63) ? hd : nb[4 + q];
    }
    parity ^= 1;
  }

  // out = f G x - out (+ (cr + i ci) lam with SRC)
  template <bool SRC>
  __device__ __forceinline__ void apply(const double* xr, const double* xi, double ur, double ui,
                                        double dr_, double di_, double f, double* or_, double* oi,
                                        double cr, double ci, const double* lr,
                                        const double* li) const {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double lor = (r == 0) ? ur : xr[r - 1], loi = (r == 0) ? ui : xi[r - 1];
      const double hir = (r == R - 1) ? dr_ : xr[r + 1], hii = (r == R - 1) ? di_ : xi[r + 1];
      const double gl = (r == 0) ? gm : gg[r - 1];
      // g_{i-1} x_{i-1} + d_i x_i + g_i x_{i+1}
      const double hr = fma(dd[r], xr[r], fma(gl, lor, gg[r] * hir));
      const double hi = fma(dd[r], xi[r], fma(gl, loi, gg[r] * hii));
      if constexpr (SRC) {
        or_[r] = f * hr - or_[r] + (cr * lr[r] - ci * li[r]);
        oi[r] = f * hi - oi[r] + (cr * li[r] + ci * lr[r]);
      } else {
        or_[r] = f * hr - or_[r];
        oi[r] = f * hi - oi[r];
      }
    }
  }
};

// v times conj(w) (to the gauge frame) or w (back to the plain frame).
__device__ __forceinline__ void gauge_in(const double2 w, double& re, double& im) {
  const double r = w.x * re + w.y * im, i = w.x * im - w.y * re;
  re = r;
  im = i;
}
__device__ __forceinline__ void gauge_out(const double2 w, double& re, double& im) {
  const double r = w.x * re - w.y * im, i = w.x * im + w.y * re;
  re = r;
  im = i;
}

__device__ __forceinline__ void load_vec(const double* v, long idx, double& re, double& im) {
  const double2 x = reinterpret_cast<const double2*>(v)[idx];
  re = x.x;
  im = x.y;
}
__device__ __forceinline__ void store_vec(double* v, long idx, double re, double im) {
  reinterpret_cast<double2*>(v)[idx] = make_double2(re, im);
}

template <int R, int W>
__global__ __launch_bounds__(W * 64) void tridiag_adj_forward_kernel(TridiagAdjPass p) {
  __shared__ double halo[2][4][2][W];
  AdjWindow<R, W> win;
  win.halo = halo;
  win.parity = 0;
  win.lane = threadIdx.x & 63;
  win.wid = threadIdx.x >> 6;
  const long col = blockIdx.x / p.nblk, r0 = (long)(blockIdx.x % p.nblk) * p.B;
  const long n = p.n;
  const long base = r0 - p.K + ((long)win.wid * 64 + win.lane) * R;
  const long own_end = (r0 + p.B < n) ? r0 + p.B : n;
  const double2* coef = reinterpret_cast<const double2*>(p.coef);
  const double2* gw = reinterpret_cast<const double2*>(p.gauge);
  win.set(p, base);

  double ar[R], ai[R], br[R], bi[R], yr[R], yi[R];  // P in a and b, the running sum Y
  int l;
  if (p.lo == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      ar[r] = ai[r] = 0.0;
      if (i >= 0 && i < n) {
        if (p.x == nullptr)
          ar[r] = (i == col) ? 1.0 : 0.0;
        else
          load_state(p.x, p.x_rowmajor ? i * p.ncols + col : col * n + i, p.x_c64, ar[r], ai[r]);
        if (p.x_store && i >= r0 && i < own_end) store_vec(p.x_store, col * n + i, ar[r], ai[r]);
        gauge_in(gw[i], ar[r], ai[r]);  // P_0 = D^+ X
      }
      br[r] = bi[r] = 0.0;
    }
    double nb[8];
    win.exchange(ar, ai, ar, ai, nb);
    win.template apply<false>(ar, ai, nb[0], nb[1], nb[4], nb[5], 1.0, br, bi, 0.0, 0.0, ar, ai);
    const double2 c0 = coef[0], c1 = coef[1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      yr[r] = c0.x * ar[r] - c0.y * ai[r] + c1.x * br[r] - c1.y * bi[r];
      yi[r] = c0.x * ai[r] + c0.y * ar[r] + c1.x * bi[r] + c1.y * br[r];
    }
    l = 1;
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      ar[r] = ai[r] = br[r] = bi[r] = yr[r] = yi[r] = 0.0;
      if (i >= 0 && i < n) {
        load_vec(p.in[0], col * n + i, ar[r], ai[r]);
        load_vec(p.in[1], col * n + i, br[r], bi[r]);
        load_vec(p.in[2], col * n + i, yr[r], yi[r]);
      }
    }
    l = p.lo;
  }
  // P_l in b and P_{l-1} in a while `latest_b`, else the other way round
  bool latest_b = true;
  for (; l < p.hi; ++l) {
    double nb[8];
    const double2 c = coef[l + 1];
    if (latest_b) {
      win.exchange(br, bi, br, bi, nb);
      win.template apply<false>(br, bi, nb[0], nb[1], nb[4], nb[5], 2.0, ar, ai, 0.0, 0.0, br, bi);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        yr[r] += c.x * ar[r] - c.y * ai[r];
        yi[r] += c.x * ai[r] + c.y * ar[r];
      }
    } else {
      win.exchange(ar, ai, ar, ai, nb);
      win.template apply<false>(ar, ai, nb[0], nb[1], nb[4], nb[5], 2.0, br, bi, 0.0, 0.0, ar, ai);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        yr[r] += c.x * br[r] - c.y * bi[r];
        yi[r] += c.x * bi[r] + c.y * br[r];
      }
    }
    latest_b = !latest_b;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    if (i < r0 || i >= own_end) continue;
    const long at = col * n + i;
    const double pr = latest_b ? br[r] : ar[r], pi = latest_b ? bi[r] : ai[r];     // P_hi
    const double qr = latest_b ? ar[r] : br[r], qi = latest_b ? ai[r] : bi[r];     // P_{hi-1}
    if (p.hi == p.L) {
      store_vec(p.plm1, at, qr, qi);
      store_vec(p.pl, at, pr, pi);
      if (p.xnext) {  // X_{k+1} = phase D Y
        double xr = p.phr * yr[r] - p.phi * yi[r], xi = p.phr * yi[r] + p.phi * yr[r];
        gauge_out(gw[i], xr, xi);
        store_vec(p.xnext, at, xr, xi);
      }
    } else {
      store_vec(p.out[0], at, qr, qi);
      store_vec(p.out[1], at, pr, pi);
      store_vec(p.out[2], at, yr[r], yi[r]);
    }
  }
}

template <int R, int W>
__global__ __launch_bounds__(W * 64) void tridiag_adj_reverse_kernel(TridiagAdjPass p) {
  __shared__ double halo[2][4][2][W];
  AdjWindow<R, W> win;
  win.halo = halo;
  win.parity = 0;
  win.lane = threadIdx.x & 63;
  win.wid = threadIdx.x >> 6;
  const long col = blockIdx.x / p.nblk, r0 = (long)(blockIdx.x % p.nblk) * p.B;
  const long n = p.n;
  const long base = r0 - p.K + ((long)win.wid * 64 + win.lane) * R;
  const long own_end = (r0 + p.B < n) ? r0 + p.B : n;
  const double2* coef = reinterpret_cast<const double2*>(p.coef);
  const double2* gw = reinterpret_cast<const double2*>(p.gauge);
  win.set(p, base);

  double lr[R], li[R];                // Lambda
  double ar[R], ai[R], br[R], bi[R];  // two P terms
  double qr[R], qi[R], sr[R], si[R];  // two Pbar terms
  double own[R];                      // 1 on the rows this workgroup owns
  const bool first = (p.hi == p.L - 1);
  const double2 cL = coef[p.L];
  const double dLr = p.phr * cL.x - p.phi * cL.y, dLi = -(p.phr * cL.y + p.phi * cL.x);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const long i = base + r;
    own[r] = (i >= r0 && i < own_end) ? 1.0 : 0.0;
    lr[r] = li[r] = ar[r] = ai[r] = br[r] = bi[r] = qr[r] = qi[r] = sr[r] = si[r] = 0.0;
    if (i >= 0 && i < n) {
      load_state(p.lam, p.lam_rowmajor ? i * p.ncols + col : col * n + i, p.lam_c64, lr[r], li[r]);
      gauge_in(gw[i], lr[r], li[r]);  // D^+ Lambda
      if (first) {  // P_{L-1}, P_L; Pbar_L = d_L Lambda, Pbar_{L+1} = 0
        load_vec(p.seg_plm1, col * n + i, ar[r], ai[r]);
        load_vec(p.seg_pl, col * n + i, br[r], bi[r]);
        qr[r] = dLr * lr[r] - dLi * li[r];
        qi[r] = dLr * li[r] + dLi * lr[r];
      } else {
        load_vec(p.in[0], col * n + i, ar[r], ai[r]);
        load_vec(p.in[1], col * n + i, br[r], bi[r]);
        load_vec(p.in[2], col * n + i, qr[r], qi[r]);
        load_vec(p.in[3], col * n + i, sr[r], si[r]);
      }
    }
  }

  double gv = 0.0, gk = 0.0;
  // One downward term l with P_l in x, P_{l+1} in z (-> P_{l-1}), Pbar_{l+1} in
  // pb and Pbar_{l+2} in o (-> Pbar_l). AB: x = a, z = b, pb = q, o = s; else
  // the pairs swapped. Written out per assignment (no array pointers), so that
  // every array stays in registers.
#define FQ_DOWN(XR, XI, ZR, ZI, PR, PI, OR, OI, l_)                                           \
  {                                                                                          \
    const int lt = (l_);                                                                      \
    double nb[8];                                                                            \
    win.exchange(XR, XI, PR, PI, nb);                                                        \
    const double w = (lt >= 1) ? 2.0 : 1.0;                                                   \
    _Pragma("unroll") for (int r = 0; r < R; ++r) {                                          \
      gv += own[r] * w * win.vv[r] * (PR[r] * XR[r] + PI[r] * XI[r]);                        \
      if (p.any_b) {                                                                         \
        const double lor = (r == 0) ? nb[0] : XR[r - 1], loi = (r == 0) ? nb[1] : XI[r - 1]; \
        const double hir = (r == R - 1) ? nb[4] : XR[r + 1],                                 \
                     hii = (r == R - 1) ? nb[5] : XI[r + 1];                                 \
        const double ckr = (r == 0) ? win.kmr : win.kr[r - 1],                               \
                     cki = (r == 0) ? win.kmi : win.ki[r - 1];                               \
        const double tr = ckr * lor + cki * loi + win.kr[r] * hir - win.ki[r] * hii;         \
        const double ti = ckr * loi - cki * lor + win.kr[r] * hii + win.ki[r] * hir;         \
        gk += own[r] * w * (PR[r] * tr + PI[r] * ti);                                        \
      }                                                                                      \
    }                                                                                        \
    const double2 cl = coef[lt];                                                              \
    const double dr = p.phr * cl.x - p.phi * cl.y, di = -(p.phr * cl.y + p.phi * cl.x);      \
    win.template apply<true>(PR, PI, nb[2], nb[3], nb[6], nb[7], w, OR, OI, dr, di, lr, li); \
    if (lt == 1) {                                                                            \
      _Pragma("unroll") for (int r = 0; r < R; ++r) {                                        \
        const long i = base + r;                                                             \
        ZR[r] = ZI[r] = 0.0;                                                                 \
        if (i >= 0 && i < n) {                                                               \
          load_vec(p.p0, col * n + i, ZR[r], ZI[r]);                                         \
          gauge_in(gw[i], ZR[r], ZI[r]);                                                     \
        }                                                                                    \
      }                                                                                      \
    } else if (lt >= 2) {                                                                     \
      win.template apply<false>(XR, XI, nb[0], nb[1], nb[4], nb[5], 2.0, ZR, ZI, 0.0, 0.0,   \
                                lr, li);                                                     \
    }                                                                                        \
  }
  // Pbar_l = w Ht Pbar_{l+1} - Pbar_{l+2} + conj(phase c_l) Lambda, w = 2 (l >= 1) or 1;
  // P_{l-1} = 2 Ht P_l - P_{l+1}, P_0 read back; the contractions with Hmod
  // (diagonal) and K (K_{i,i+1} = k_i, (K x)_i = conj(k_{i-1}) x_{i-1} + k_i x_{i+1})
  int l = p.hi;
  for (; l - 1 >= p.lo; l -= 2) {
    FQ_DOWN(ar, ai, br, bi, qr, qi, sr, si, l)      // P_l in a, P_{l-1} -> b; Pbar_l -> s
    FQ_DOWN(br, bi, ar, ai, sr, si, qr, qi, l - 1)  // P_{l-1} in b; Pbar_{l-1} -> q
  }
  const bool odd = (l == p.lo);
  if (odd) FQ_DOWN(ar, ai, br, bi, qr, qi, sr, si, l)
#undef FQ_DOWN
  // even: P_{lo-1} a, P_lo b, Pbar_lo q, Pbar_{lo+1} s; odd: the pairs swapped.
  // (Separate branches rather than selects between arrays, which would take
  // their addresses and move them out of registers.)
#define FQ_STORE(P1R, P1I, P2R, P2I, Q1R, Q1I, Q2R, Q2I)                        \
  _Pragma("unroll") for (int r = 0; r < R; ++r) {                               \
    const long i = base + r;                                                    \
    if (i < r0 || i >= own_end) continue;                                       \
    const long at = col * n + i;                                                \
    if (p.lo == 0) {                                                            \
      double xr = Q1R[r], xi = Q1I[r];                                          \
      gauge_out(gw[i], xr, xi);                                                 \
      store_vec(p.lam_out, at, xr, xi);                                         \
    } else {                                                                    \
      store_vec(p.out[0], at, P1R[r], P1I[r]);                                  \
      store_vec(p.out[1], at, P2R[r], P2I[r]);                                  \
      store_vec(p.out[2], at, Q1R[r], Q1I[r]);                                  \
      store_vec(p.out[3], at, Q2R[r], Q2I[r]);                                  \
    }                                                                           \
  }
  if (odd) {
    FQ_STORE(br, bi, ar, ai, sr, si, qr, qi)
  } else {
    FQ_STORE(ar, ai, br, bi, qr, qi, sr, si)
  }
#undef FQ_STORE
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    gv += __shfl_xor(gv, o);
    gk += __shfl_xor(gk, o);
  }
  if (win.lane == 0) {
    atomicAdd(p.grad, gv);
    if (p.any_b) atomicAdd(p.grad + 1, gk);
  }
}

// 8 waves x 64 lanes x 4 rows: 2048-row windows.
constexpr int kAdjR = 4, kAdjW = 8;

}  // namespace

// 16 rows per lane and up to 4 waves per part (512 threads, <= 256 VGPRs).
long tridiag_resident_max_n() { return 4L * 64 * 16; }

hipError_t launch_tridiag_resident(const TridiagJob& job, hipStream_t s) {
  if (job.n < 1 || job.ncols < 1) return hipErrorInvalidValue;
  if (job.n <= 256) return launch_r<4, 128, false>(job, 1, s);
  if (job.n <= 1024) return launch_r<16, 512, false>(job, 1, s);
  if (job.n <= tridiag_resident_max_n()) {
    const int G = (int)((job.n + 1023) / 1024);
    return launch_r<16, 512, true>(job, G, s);
  }
  return hipErrorInvalidValue;
}

// ---- energy expectations of tridiagonal states -------------------------------------------------
//
// For states x (user layout, row i of column c at i * ncols + c) and
// H = H0 + f Hmod: num[c] += sum_i Re(conj(x_i) (H x)_i), den[c] += sum_i |x_i|^2
// over a chunk of rows per workgroup row (blockIdx.y), one thread per column;
// then energy_finish adds w num / den to avg and clears num, den.
namespace {
constexpr int kEnergyRows = 64;

__global__ __launch_bounds__(256) void tridiag_energy_kernel(const void* x, int c64, long n,
                                                            long ncols, const double* __restrict__ d,
                                                            const double2* __restrict__ off,
                                                            const double* __restrict__ v, double f,
                                                            double* __restrict__ num,
                                                            double* __restrict__ den) {
  const long c = (long)blockIdx.x * 256 + threadIdx.x;
  if (c >= ncols) return;
  const long i0 = (long)blockIdx.y * kEnergyRows;
  const long i1 = (i0 + kEnergyRows < n) ? i0 + kEnergyRows : n;
  double sn = 0.0, sd = 0.0;
  double pr = 0.0, pi = 0.0, xr, xi, nr = 0.0, ni = 0.0;
  if (i0 > 0) load_state(x, (i0 - 1) * ncols + c, c64, pr, pi);
  load_state(x, i0 * ncols + c, c64, xr, xi);
  for (long i = i0; i < i1; ++i) {
    nr = ni = 0.0;
    if (i + 1 < n) load_state(x, (i + 1) * ncols + c, c64, nr, ni);
    // (H x)_i = (d_i + f v_i) x_i + H[i][i+1] x_{i+1} + conj(H[i-1][i]) x_{i-1}
    const double dd = d[i] + f * v[i];
    double hr = dd * xr, hi = dd * xi;
    if (i + 1 < n) {
      const double2 e = off[i];
      hr += e.x * nr - e.y * ni;
      hi += e.x * ni + e.y * nr;
    }
    if (i > 0) {
      const double2 e = off[i - 1];
      hr += e.x * pr + e.y * pi;
      hi += e.x * pi - e.y * pr;
    }
    sn += xr * hr + xi * hi;
    sd += xr * xr + xi * xi;
    pr = xr;
    pi = xi;
    xr = nr;
    xi = ni;
  }
  atomicAdd(num + c, sn);
  atomicAdd(den + c, sd);
}

__global__ void energy_finish_kernel(double* __restrict__ num, double* __restrict__ den, long ncols,
                                     double w, double* __restrict__ avg) {
  const long c = (long)blockIdx.x * 256 + threadIdx.x;
  if (c >= ncols) return;
  avg[c] += w * num[c] / den[c];
  num[c] = 0.0;
  den[c] = 0.0;
}

}  // namespace

hipError_t launch_tridiag_energy(const void* x, bool c64, long n, long ncols, const double* d,
                                 const void* off, const double* v, double f, double* num,
                                 double* den, hipStream_t s) {
  if (n < 1 || ncols < 1 || (n > 1 && !off)) return hipErrorInvalidValue;
  const long gx = (ncols + 255) / 256, gy = (n + kEnergyRows - 1) / kEnergyRows;
  if (gx > 0x7fffffffL || gy > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tridiag_energy_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, x,
                     c64 ? 1 : 0, n, ncols, d, reinterpret_cast<const double2*>(off), v, f, num,
                     den);
  return hipGetLastError();
}

hipError_t launch_energy_finish(double* num, double* den, long ncols, double w, double* avg,
                                hipStream_t s) {
  if (ncols < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(energy_finish_kernel, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, s,
                     num, den, ncols, w, avg);
  return hipGetLastError();
}

long tridiag_stream_rows(int G) { return (long)G * 64 * 16; }

hipError_t launch_tridiag_stream(const TridiagJob& job, const TridiagStream& st, hipStream_t s) {
  if (job.n < 1 || job.ncols < 1 || st.K < 2 || st.l0 < 0 || st.l1 <= st.l0 ||
      st.l1 - st.l0 > st.K || st.l1 > job.L + 1 || st.B < 1 ||
      st.G != 1 || st.B + 2L * st.K != tridiag_stream_rows(st.G) ||
      st.nblk != (job.n + st.B - 1) / st.B ||
      (st.l0 == 1) || st.K % 16 || st.B % 16 || st.n16 != (job.n + 15) / 16 * 16 ||
      st.plane < st.n16 * job.ncols || st.stepc == nullptr)
    return hipErrorInvalidValue;
  return launch_stream_g<1>(job, st, s);
}

hipError_t launch_tridiag_stream_step(const TridiagJob& job, const TridiagStream& st,
                                      double* stepc, hipStream_t s) {
  if (job.n < 1 || st.n16 != (job.n + 15) / 16 * 16 || st.s < 0 || stepc == nullptr)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(tridiag_stream_step_kernel, dim3((unsigned)((st.n16 + 255) / 256)), dim3(256),
                     0, s, job, st.s, st.last_step, st.n16, stepc);
  return hipGetLastError();
}

long tridiag_adjoint_max_n() { return 8L * 64 * 4; }

hipError_t launch_tridiag_adjoint(const TridiagAdjJob& job, hipStream_t s) {
  if (job.n < 1 || job.ncols < 1 || job.L < 1 || job.M < 1 || job.ckpt < 1 ||
      job.ncols > 0x7fffffffL)
    return hipErrorInvalidValue;
  if (job.n <= 256) return launch_adj_r<4, 1>(job, s);
  if (job.n <= 1024) return launch_adj_r<4, 4>(job, s);
  if (job.n <= tridiag_adjoint_max_n()) return launch_adj_r<4, 8>(job, s);
  return hipErrorInvalidValue;
}

long tridiag_adj_window_rows() { return (long)kAdjW * 64 * kAdjR; }

static hipError_t check_adj_pass(const TridiagAdjPass& p) {
  const long win = tridiag_adj_window_rows();
  if (p.n < 1 || p.ncols < 1 || p.K < 1 || p.B < 1 || p.B + 2L * p.K != win) return hipErrorInvalidValue;
  if ((long)p.nblk * p.B < p.n || (long)(p.nblk - 1) * p.B >= p.n) return hipErrorInvalidValue;
  const long grid = p.ncols * p.nblk;
  if (grid > 0x7fffffffL) return hipErrorInvalidValue;
  return hipSuccess;
}

hipError_t launch_tridiag_adj_forward(const TridiagAdjPass& p, hipStream_t s) {
  if (hipError_t e = check_adj_pass(p); e != hipSuccess) return e;
  if (p.lo < 0 || p.hi <= p.lo || p.hi > p.L || p.hi - p.lo > p.K) return hipErrorInvalidValue;
  hipLaunchKernelGGL((tridiag_adj_forward_kernel<kAdjR, kAdjW>), dim3((unsigned)(p.ncols * p.nblk)),
                     dim3(kAdjW * 64), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_tridiag_adj_reverse(const TridiagAdjPass& p, hipStream_t s) {
  if (hipError_t e = check_adj_pass(p); e != hipSuccess) return e;
  if (p.lo < 0 || p.hi < p.lo || p.hi > p.L - 1 || p.hi - p.lo + 1 > p.K) return hipErrorInvalidValue;
  hipLaunchKernelGGL((tridiag_adj_reverse_kernel<kAdjR, kAdjW>), dim3((unsigned)(p.ncols * p.nblk)),
                     dim3(kAdjW * 64), 0, s, p);
  return hipGetLastError();
}

}  // namespace fq
