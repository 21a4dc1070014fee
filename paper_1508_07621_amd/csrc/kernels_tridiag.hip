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

// Whole-wave DPP shifts by one lane; the lane without a source gets +0.0
// (bound_ctrl: the shift itself writes the zero, with no separate zeroing of
// the destination).
__device__ __forceinline__ double from_prev_lane(double v) {  // lane l <- lane l-1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_next_lane(double v) {  // lane l <- lane l+1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, true);
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
          if (job.x0_colmajor)  // complex128, column col at col * n
            load_state(job.x0, col * n + i, 0, xr, xi);
          else
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
    }
    // (one wave per part: the shifts already read zero beyond the window)
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
  // even l into pe, odd l + 1 into po; each pair's coefficients are loaded one
  // pair ahead, so the scalar loads' latency hides behind a pair of terms
  {
    const int lc = job.L;  // coef holds c_0 .. c_L
    double ce_n = coef[l < lc ? l : lc].x, co_n = coef[l + 1 < lc ? l + 1 : lc].y;
    for (; l + 1 < st.l1; l += 2) {
      const double ce = ce_n, co = sgn * co_n;
      ce_n = coef[l + 2 < lc ? l + 2 : lc].x;
      co_n = coef[l + 3 < lc ? l + 3 : lc].y;
      advance(po, pe);
#pragma unroll
      for (int r = 0; r < R; ++r) ys[r] = fma(ce, pe[r], ys[r]);
      advance(pe, po);
#pragma unroll
      for (int r = 0; r < R; ++r) yo[r] = fma(co, po[r], yo[r]);
    }
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

  // step end: the last two terms P_{L-1}, P_L on request (planes [l & 1][part]);
  // both halves of Y meet; X~_{s+1} = phase w_s conj(w_{s+1}) Y, or X = phase
  // w_s Y after the last step (to x_out, row-major).
  if (st.save) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long i = base + r;
      if (i >= a0 && i < own_end) {
        st.save[part * st.plane + cn + at(r)] = pe[r];
        st.save[(2 + part) * st.plane + cn + at(r)] = po[r];
      }
    }
  }
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
// For columns longer than one workgroup holds, the reverse recurrences run one
// step at a time, at most K terms per launch, on the windows of the forward
// passes: B owned rows and K ghost rows on each side, 16 rows per lane, one
// wave for the real part and one for the imaginary part of every vector, the
// state between launches in planes of the interleaved row layout. The segment
// recompute is the forward pass itself (tridiag_stream_kernel), which leaves
// the last two terms P_{L-1}, P_L of every step in the segment buffer.
//
// Everything runs in the gauge frame of the step, Ht = D G D^+ with real G: a
// term applies G to the real and imaginary parts separately, so each wave only
// needs neighbour rows of its own part (lane shifts; the window edges read
// zero, which the ghost rows absorb). Per term l, going down from L - 1:
//   Pbar_l  = (2 - delta_l0) G Pbar_{l+1} - Pbar_{l+2} + d_l Lambda~,
//   P_{l-1} = 2 G P_l - P_{l+1}   (l >= 1; at l = 1 this regenerates P_0),
//   S_V    += Re Pbar_{l+1} P_l per row and part (Hmod is diagonal),
//   S_K    += Re conj(Pbar_{l+1}) (K~ P_l) per row and part,
// with d_l = conj(phase c_l), Lambda~ = D^+ Lambda and K~ = D^+ K D (complex
// couplings conj(w_i) k_i w_{i+1}). The source mixes the parts of Lambda~, so
// each wave holds both; K~ mixes the parts of P_l, so with the K contraction
// the two waves trade P_l through LDS once per term. The sums over the owned
// rows, (2 - delta_l0)-weighted, go to the step's two accumulators. At l = 0
// Pbar_0 leaves in the gauge frame of step k; the step before applies the
// factor conj(w_{k-1}) w_k as it reads it (the first reversed step reads
// U_bar with conj(w_{M-1})).

// Rows of the reverse pass tables of step k (interleaved layout, rows n .. n16-1
// zero): 2 d_i, 2 g_i, v_i, the factor that takes the Lambda planes into the
// gauge frame (conj(w_k) w_{k+1}, or conj(w_k) when Lambda is U_bar), and the
// K~ couplings conj(w_i) k_i w_{i+1} with k_i = -i h_i (v_{i+1} - v_i).
__global__ __launch_bounds__(256) void tridiag_adj_table_kernel(TridiagAdjStream p, int k,
                                                                int plain_lambda, double* tab) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const long n = p.n, n16 = p.n16;
  if (i >= n16) return;
  const long at = (i & 15) * (n16 >> 4) + (i >> 4);
  double d2 = 0, g2 = 0, vi = 0, fr = 0, fi = 0, kr = 0, ki = 0;
  if (i < n) {
    const double2* w = reinterpret_cast<const double2*>(p.gauge) + (long)k * n;
    vi = p.v_diag[i];
    d2 = 2.0 * (p.h0_diag[i] + p.a * vi - p.beta) * p.inv_dE;
    const double2 wk = w[i];
    double ur = 1.0, ui = 0.0;  // w_{k+1}
    if (!plain_lambda) {
      const double2 wn = w[n + i];
      ur = wn.x;
      ui = wn.y;
    }
    const double tr = wk.x * ur + wk.y * ui, ti = wk.x * ui - wk.y * ur;  // conj(w_k) u
    fr = p.phr * tr + p.phi * ti;  // conj(phase) conj(w_k) u
    fi = p.phr * ti - p.phi * tr;
    if (i + 1 < n) {
      const double2 h = reinterpret_cast<const double2*>(p.h0_off)[i];
      const double dv = p.v_diag[i + 1] - vi, q = p.b * dv;
      g2 = 2.0 * sqrt((h.x * h.x + h.y * h.y) * (1.0 + q * q)) * p.inv_dE;
      const double k_r = h.y * dv, k_i = -h.x * dv;  // -i h dv
      const double2 w1 = w[i + 1];
      const double tr = k_r * w1.x - k_i * w1.y, ti = k_r * w1.y + k_i * w1.x;
      kr = wk.x * tr + wk.y * ti;
      ki = wk.x * ti - wk.y * tr;
    }
  }
  tab[at] = d2;
  tab[n16 + at] = g2;
  tab[2 * n16 + at] = vi;
  tab[3 * n16 + at] = fr;
  tab[4 * n16 + at] = fi;
  tab[5 * n16 + at] = kr;
  tab[6 * n16 + at] = ki;
}

// U_bar (n x ncols row-major, the state type) into two planes (re, im) of the
// interleaved layout, rows n .. n16-1 zero.
__global__ __launch_bounds__(256) void tridiag_lam_pack_kernel(const void* ubar, int c64, long n,
                                                               long ncols, long n16,
                                                               double* out) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= n16 * ncols) return;
  const long i = t / ncols, col = t % ncols;
  double re = 0.0, im = 0.0;
  if (i < n) load_state(ubar, i * ncols + col, c64, re, im);
  const long at = col * n16 + (i & 15) * (n16 >> 4) + (i >> 4);
  out[at] = re;
  out[n16 * ncols + at] = im;
}

// Lane shifts for the reverse passes: the lane without a source reads +0.0
// (bound_ctrl), with no separate zeroing of the destination.
__device__ __forceinline__ double prev_lane_or_zero(double v) {  // lane l <- lane l-1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double next_lane_or_zero(double v) {  // lane l <- lane l+1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

template <int V>
struct Parity {
  static constexpr int value = V;
};

template <bool KC, bool HI_ODD>
__global__ __launch_bounds__(128) void tridiag_adj_stream_kernel(TridiagAdjStream p,
                                                                 const double* __restrict__ tab,
                                                                 const double2* __restrict__ coef) {
  constexpr int R = 16, XR = KC ? R : 1, XL = KC ? 64 : 1;
  // the pass's Chebyshev coefficients, P_l of both parts two terms deep (K
  // contraction), the waves' sums
  __shared__ double2 c_s[128];
  // Lambda' of the window for the K contraction (registers otherwise)
  __shared__ double lam_s[2][XR][XL];
  __shared__ double xs[2][2][XR][XL];
  __shared__ double d_s[XR][XL];  // K contraction: the diagonal of 2 G (registers otherwise)
  __shared__ double red[2][2];

  const int part = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long col = blockIdx.x / p.nblk, blk = blockIdx.x % p.nblk;
  const long n = p.n, n16 = p.n16, nq = n16 >> 4, plane = p.plane;
  const long a0 = blk * p.B;
  const long q = (a0 - p.K) / 16 + lane;  // row group of this lane (may be < 0)
  const long base = q * 16;
  // row base + r of this column sits at r nq + q of a plane: lane pointers
  // plus uniform offsets
  const long off = col * n16 + q;
  const double* tq = tab + q;
  auto in_col = [&](int r) { return base + r >= 0 && base + r < n; };
  // K and B are multiples of 16: a lane's 16 rows are all owned or all ghosts
  const bool own_lane = base >= a0 && base < a0 + p.B;

  double d2r[KC ? 1 : R], g2[R];   // rows of 2 G
  double x[R], z[R], pb[R], o[R];  // P_l, P_{l+1}, Pbar_{l+1}, Pbar_{l+2}
  double sv[R];                    // Re Pbar_{l+1} P_l summed over the terms
  double gk = 0.0;                 // Re <Pbar_{l+1}, K~ P_l> over the lane's rows, summed
  double kr[KC ? R : 1], ki[KC ? R : 1];  // K~ couplings k_i (re, im; im signed for this part)
  double gm2 = 0.0;                // coupling from row base - 1

  // Lambda' = f Lambda with f = conj(phase) conj(w_k) w_{k+1} from the table:
  // this part and the other (with the K contraction: in LDS, this wave
  // storing its own part)
  double lam_o[KC ? 1 : R], lam_x[KC ? 1 : R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double vr = 0.0, vi = 0.0;
    if (in_col(r)) {
      const double ar = p.lam[off + r * nq], ai = p.lam[plane + off + r * nq];
      const double fr = tq[3 * n16 + r * nq], fi = tq[4 * n16 + r * nq];
      vr = fr * ar - fi * ai;
      vi = fr * ai + fi * ar;
    }
    if constexpr (KC) {
      lam_s[part][r][lane] = part == 0 ? vr : vi;
    } else {
      lam_o[r] = part == 0 ? vr : vi;
      lam_x[r] = part == 0 ? vi : vr;
    }
  }
  auto lam = [&](bool other, int r) {
    if constexpr (KC)
      return lam_s[other ? 1 - part : part][r][lane];
    else
      return other ? lam_x[r] : lam_o[r];
  };
  for (int t = threadIdx.x; t <= p.hi - p.lo; t += 128) c_s[t] = coef[p.hi - t];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool ok = in_col(r);
    if constexpr (KC) {
      if (part == 0) d_s[r][lane] = ok ? tq[r * nq] : 0.0;
    } else {
      d2r[r] = ok ? tq[r * nq] : 0.0;
    }
    g2[r] = ok ? tq[n16 + r * nq] : 0.0;
    sv[r] = 0.0;
  }
  if (base >= 1 && base < n) gm2 = tq[n16 + (long)(R - 1) * nq - 1];  // row base - 1
  const double sgn = part == 0 ? 1.0 : -1.0;
  double kmr = 0.0, kmi = 0.0;  // K~ coupling from row base - 1
  if constexpr (KC) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      kr[r] = in_col(r) ? tq[5 * n16 + r * nq] : 0.0;
      ki[r] = in_col(r) ? sgn * tq[6 * n16 + r * nq] : 0.0;
    }
    if (base >= 1 && base < n) {
      kmr = tq[5 * n16 + (long)(R - 1) * nq - 1];
      kmi = sgn * tq[6 * n16 + (long)(R - 1) * nq - 1];
    }
  }
  __syncthreads();

  // d_l Lambda~ = conj(c_l) Lambda'. c_l is real for even l and imaginary for
  // odd l: a part takes its own part of Lambda' with Re c_l (even l), or the
  // other part with +/- Im c_l (odd l)

  const bool first = p.hi == p.L - 1;
  if (first) {  // P_{L-1}, P_L from the recompute; Pbar_L = d_L Lambda~, Pbar_{L+1} = 0
    const double2 cL = coef[p.L];
    const bool odd = p.L & 1;
    const double cs = odd ? sgn * cL.y : cL.x;
    const double* sx = p.seg + ((((p.L - 1) & 1) * 2 + part) * plane) + off;
    const double* sz = p.seg + (((p.L & 1) * 2 + part) * plane) + off;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = in_col(r);
      x[r] = ok ? sx[r * nq] : 0.0;
      z[r] = ok ? sz[r * nq] : 0.0;
      pb[r] = cs * lam(odd, r);
      o[r] = 0.0;
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = in_col(r);
      const double* v = p.in + part * plane + off + r * nq;
      x[r] = ok ? v[0] : 0.0;
      z[r] = ok ? v[2 * plane] : 0.0;
      pb[r] = ok ? v[4 * plane] : 0.0;
      o[r] = ok ? v[6 * plane] : 0.0;
    }
  }

  int parity = 0;
  // One term l >= 1 of parity P::value: Pbar_l = 2 G PB - O + d_l Lambda~ into
  // O, P_{l-1} = 2 G X - Z into Z, the sums. L0: the term l = 0 (G instead of
  // 2 G, no new P, the sums weighted by one half; every sum is doubled at the
  // end).
  auto term = [&](auto par, const double* X, double* Z, const double* PB, double* O, int l,
                  bool L0) {
    constexpr bool ODD = decltype(par)::value;
    // (LDS values are read in every term, not kept in registers)
    if constexpr (KC) asm volatile("" ::: "memory");
    const double2 cl = c_s[p.hi - l];
    const double cs = ODD ? sgn * cl.y : cl.x;
    auto d2 = [&](int r) {
      if constexpr (KC)
        return d_s[r][lane];
      else
        return d2r[r];
    };
    const double xu = prev_lane_or_zero(X[R - 1]), xd = next_lane_or_zero(X[0]);
    const double pu = prev_lane_or_zero(PB[R - 1]), pd = next_lane_or_zero(PB[0]);
    const double hw = L0 ? 0.5 : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) sv[r] = fma(hw * PB[r], X[r], sv[r]);
    if constexpr (KC) {
      // (K~ P)_r = conj(k_{r-1}) P_{r-1} + k_r P_{r+1}; this part of it takes
      // this part's P with Re k and the other part's with -/+ Im k
#pragma unroll
      for (int r = 0; r < R; ++r) xs[parity][part][r][lane] = X[r];
      __syncthreads();
      const auto ox = xs[parity][1 - part];
      // the other part's rows base - 1 and base + 16 (zero beyond the window)
      const double oe0 = ox[R - 1][(lane + 63) & 63], oe1 = ox[0][(lane + 1) & 63];
      const double om0 = lane > 0 ? oe0 : 0.0, op15 = lane < 63 ? oe1 : 0.0;
      double tk = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double om = r > 0 ? ox[r - 1][lane] : om0;
        const double op = r < R - 1 ? ox[r + 1][lane] : op15;
        const double xm = r > 0 ? X[r - 1] : xu, xp = r < R - 1 ? X[r + 1] : xd;
        const double cmr = r > 0 ? kr[r - 1] : kmr, cmi = r > 0 ? ki[r - 1] : kmi;
        double t = cmr * xm;
        t = fma(kr[r], xp, t);
        t = fma(cmi, om, t);
        t = fma(-ki[r], op, t);
        tk = fma(PB[r], t, tk);
      }
      gk = fma(hw, tk, gk);
      parity ^= 1;
    }
    if (!L0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double lo = r > 0 ? X[r - 1] : xu, hi = r < R - 1 ? X[r + 1] : xd;
        const double gl = r > 0 ? g2[r - 1] : gm2;
        double t = fma(d2(r), X[r], -Z[r]);
        t = fma(gl, lo, t);
        Z[r] = fma(g2[r], hi, t);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double lo = r > 0 ? PB[r - 1] : pu, hi = r < R - 1 ? PB[r + 1] : pd;
        const double gl = r > 0 ? g2[r - 1] : gm2;
        double t = fma(d2(r), PB[r], -O[r]);
        t = fma(gl, lo, t);
        t = fma(g2[r], hi, t);
        O[r] = fma(cs, lam(ODD, r), t);
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double lo = r > 0 ? PB[r - 1] : pu, hi = r < R - 1 ? PB[r + 1] : pd;
        const double gl = r > 0 ? g2[r - 1] : gm2;
        double h = d2(r) * PB[r];
        h = fma(gl, lo, h);
        h = fma(g2[r], hi, h);
        const double t = fma(0.5, h, -O[r]);
        O[r] = fma(cs, lam(ODD, r), t);
      }
    }
  };
  // After the terms down to lo (>= 1): P_{lo-1}, P_lo, Pbar_lo, Pbar_{lo+1} in
  // (X, Z, PB, O); with lo = 0 the l = 0 term, then Pbar_0 out.
  // (The lane offset is recomputed here rather than kept live through the terms.)
  auto finish = [&](double* X, double* Z, double* PB, double* O) {
    if (p.lo == 0) term(Parity<0>{}, X, Z, PB, O, 0, true);
    long off2 = off;
    asm volatile("" : "+v"(off2));
    if (!own_lane) return;
    if (p.lo == 0) {
      double* v = p.lam_out + part * plane + off2;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (base + r < n) v[r * nq] = O[r];
    } else {
      double* v = p.out + part * plane + off2;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (base + r < n) {
          v[r * nq] = X[r];
          v[2 * plane + r * nq] = Z[r];
          v[4 * plane + r * nq] = PB[r];
          v[6 * plane + r * nq] = O[r];
        }
      }
    }
  };
  // the terms l >= lmin from an even l down, in pairs (even, odd) so that the
  // parity of every term is known where it is compiled
  const int lmin = p.lo > 1 ? p.lo : 1;
  auto run = [&](double* X, double* Z, double* PB, double* O, int l) {
    for (; l - 1 >= lmin; l -= 2) {
      term(Parity<0>{}, X, Z, PB, O, l, false);      // P_{l-1} -> Z, Pbar_l -> O
      term(Parity<1>{}, Z, X, O, PB, l - 1, false);  // P_{l-2} -> X, Pbar_{l-1} -> PB
    }
    if (l >= lmin) {
      term(Parity<0>{}, X, Z, PB, O, l, false);
      finish(Z, X, O, PB);
    } else {
      finish(X, Z, PB, O);
    }
  };
  // (hi >= 1 when it is odd)
  if constexpr (HI_ODD) {
    term(Parity<1>{}, x, z, pb, o, p.hi, false);
    run(z, x, o, pb, p.hi - 1);
  } else {
    run(x, z, pb, o, p.hi);
  }

  // the owned rows' sums (rows beyond n hold zeros)
  double gv = 0.0;
  if (own_lane) {
    const double* vq = tab + 2 * n16 + q;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (base + r < n) gv = fma(vq[r * nq], sv[r], gv);
  } else {
    gk = 0.0;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    gv += __shfl_xor(gv, m);
    if constexpr (KC) gk += __shfl_xor(gk, m);
  }
  if (lane == 0) {
    red[part][0] = gv;
    red[part][1] = gk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // one add per workgroup, spread over the step's slots
    double* g = p.grad + 2 * (blockIdx.x % kAdjSlots);
    atomicAdd(g, 2.0 * (red[0][0] + red[1][0]));
    if constexpr (KC) atomicAdd(g + 1, 2.0 * (red[0][1] + red[1][1]));
  }
}

// Lambda' = f Lambda in place over both planes (n16 x ncols each), with f the
// Lambda factor of the step's table (zero on the padding rows n .. n16-1).
__global__ __launch_bounds__(256) void tridiag_lam_gauge_kernel(long n16, long plane,
                                                                const double* __restrict__ tab,
                                                                double* lam) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= plane) return;
  const long at = t % n16;
  const double fr = tab[3 * n16 + at], fi = tab[4 * n16 + at];
  const double ar = lam[t], ai = lam[plane + t];
  lam[t] = fr * ar - fi * ai;
  lam[plane + t] = fr * ai + fi * ar;
}

// The reverse pass without the K contraction (node-pair sums), persistent: a
// workgroup (one wave per part, as in tridiag_adj_stream_kernel) walks the
// items it, it + G, it + 2G, ... of the pass (item = window blk x column, blk =
// it / ncols), so consecutive items mostly share their window and the rows of
// 2 G stay in registers. While an item's terms run, the next item's state
// planes of the wave's part travel from HBM into LDS by direct global-to-LDS
// loads (no registers), one dword per lane and load; the coefficients come
// through the scalar cache, so nothing else in the term loop touches LDS or
// the vector memory pipeline. Lambda arrives already multiplied by its gauge
// factor (tridiag_lam_gauge_kernel), and each wave adds its V sums into the
// step's slot once, at the end.
template <bool HI_ODD>
__global__ __launch_bounds__(128) void tridiag_adj_persist_kernel(TridiagAdjStream p,
                                                                  const double* __restrict__ tab,
                                                                  const double2* __restrict__ coef) {
  constexpr int R = 16;
  // the next item's X, Z, PB, O of each part: [part][plane][row r][lane]
  __shared__ __attribute__((aligned(16))) double pf[2][4][R][64];

  const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const long n = p.n, n16 = p.n16, nq = n16 >> 4, plane = p.plane;
  const long items = p.ncols * p.nblk;
  const bool first = p.hi == p.L - 1;
  const int npf = first ? 2 : 4;  // planes that come from memory: X, Z (and PB, O)
  const double sgn = part == 0 ? 1.0 : -1.0;
  const int lmin = p.lo > 1 ? p.lo : 1;
  // plane a (0..3: X, Z, PB, O) of this part
  auto src_plane = [&](int a) -> const double* {
    if (first) return p.seg + ((((a == 0 ? p.L - 1 : p.L) & 1) * 2 + part) * plane);
    return p.in + (part + 2 * a) * plane;
  };
  // the direct loads of item it2 into pf: lane l takes dword l & 1 of the
  // lane-(32 h + l / 2) element of every row and plane (row groups outside the
  // column skipped; they are masked where pf is read)
  auto prefetch = [&](long it2) {
    const long blk2 = it2 / p.ncols, col2 = it2 % p.ncols;
    const long q2 = (blk2 * p.B - p.K) / 16;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long qe = q2 + 32 * h + (lane >> 1);
      if (qe >= 0 && qe < nq) {
        const long e = col2 * n16 + qe;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (a >= npf) break;
          const unsigned* s = reinterpret_cast<const unsigned*>(src_plane(a) + e) + (lane & 1);
#pragma unroll
          for (int r = 0; r < R; ++r)
            __builtin_amdgcn_global_load_lds(s + 2 * r * nq, &pf[part][a][r][32 * h], 4, 0, 0);
        }
      }
    }
  };

  double d2r[R], g2[R], gm2 = 0.0;
  long tblk = -1;
  double gsum = 0.0;  // this lane's share of the V sums over its items

  for (long it = blockIdx.x; it < items; it += gridDim.x) {
    const long blk = it / p.ncols, col = it % p.ncols;
    const long a0 = blk * p.B;
    const long q = (a0 - p.K) / 16 + lane;  // row group of this lane (may be < 0)
    const long base = q * 16;
    const long off = col * n16 + q;
    auto in_col = [&](int r) { return base + r >= 0 && base + r < n; };
    const bool own_lane = base >= a0 && base < a0 + p.B;
    if (blk != tblk) {  // rows of 2 G for this window
      const double* tq = tab + q;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool ok = in_col(r);
        d2r[r] = ok ? tq[r * nq] : 0.0;
        g2[r] = ok ? tq[n16 + r * nq] : 0.0;
      }
      gm2 = (base >= 1 && base < n) ? tq[n16 + (long)(R - 1) * nq - 1] : 0.0;
      tblk = blk;
    }
    // Lambda' of this part and of the other
    double lam_o[R], lam_x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = in_col(r);
      lam_o[r] = ok ? p.lam[part * plane + off + r * nq] : 0.0;
      lam_x[r] = ok ? p.lam[(1 - part) * plane + off + r * nq] : 0.0;
    }
    double x[R], z[R], pb[R], o[R], sv[R];
    if (it != (long)blockIdx.x) {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the direct loads have landed
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool ok = in_col(r);
        x[r] = ok ? pf[part][0][r][lane] : 0.0;
        z[r] = ok ? pf[part][1][r][lane] : 0.0;
        if (!first) {
          pb[r] = ok ? pf[part][2][r][lane] : 0.0;
          o[r] = ok ? pf[part][3][r][lane] : 0.0;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool ok = in_col(r);
        const double* v = src_plane(0) + off + r * nq;
        x[r] = ok ? v[0] : 0.0;
        z[r] = ok ? src_plane(1)[off + r * nq] : 0.0;
        if (!first) {
          pb[r] = ok ? src_plane(2)[off + r * nq] : 0.0;
          o[r] = ok ? src_plane(3)[off + r * nq] : 0.0;
        }
      }
    }
    if (first) {  // Pbar_L = d_L Lambda~, Pbar_{L+1} = 0
      const double2 cL = coef[p.L];
      const bool odd = p.L & 1;
      const double cs = odd ? sgn * cL.y : cL.x;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        pb[r] = cs * (odd ? lam_x[r] : lam_o[r]);
        o[r] = 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) sv[r] = 0.0;
    // the pf reads are complete before the next item's loads overwrite pf
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    if (it + (long)gridDim.x < items) prefetch(it + gridDim.x);

    // One term l >= 1 of parity P::value: Pbar_l = 2 G PB - O + d_l Lambda~
    // into O, P_{l-1} = 2 G X - Z into Z, the V sums; L0: the term l = 0.
    // cl = c_l (uniform; its real part for even l, imaginary for odd l)
    auto term = [&](auto par, const double* X, double* Z, const double* PB, double* O,
                    double2 cl, bool L0) {
      constexpr bool ODD = decltype(par)::value;
      const double cs = ODD ? sgn * cl.y : cl.x;
      const double xu = prev_lane_or_zero(X[R - 1]), xd = next_lane_or_zero(X[0]);
      const double pu = prev_lane_or_zero(PB[R - 1]), pd = next_lane_or_zero(PB[0]);
      const double hw = L0 ? 0.5 : 1.0;
#pragma unroll
      for (int r = 0; r < R; ++r) sv[r] = fma(hw * PB[r], X[r], sv[r]);
      if (!L0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double lo = r > 0 ? X[r - 1] : xu, hi = r < R - 1 ? X[r + 1] : xd;
          const double gl = r > 0 ? g2[r - 1] : gm2;
          double t = fma(d2r[r], X[r], -Z[r]);
          t = fma(gl, lo, t);
          Z[r] = fma(g2[r], hi, t);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double lo = r > 0 ? PB[r - 1] : pu, hi = r < R - 1 ? PB[r + 1] : pd;
          const double gl = r > 0 ? g2[r - 1] : gm2;
          double t = fma(d2r[r], PB[r], -O[r]);
          t = fma(gl, lo, t);
          t = fma(g2[r], hi, t);
          O[r] = fma(cs, ODD ? lam_x[r] : lam_o[r], t);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double lo = r > 0 ? PB[r - 1] : pu, hi = r < R - 1 ? PB[r + 1] : pd;
          const double gl = r > 0 ? g2[r - 1] : gm2;
          double hh = d2r[r] * PB[r];
          hh = fma(gl, lo, hh);
          hh = fma(g2[r], hi, hh);
          const double t = fma(0.5, hh, -O[r]);
          O[r] = fma(cs, ODD ? lam_x[r] : lam_o[r], t);
        }
      }
    };
    auto finish = [&](double* X, double* Z, double* PB, double* O) {
      if (p.lo == 0) term(Parity<0>{}, X, Z, PB, O, coef[0], true);
      long off2 = off;
      asm volatile("" : "+v"(off2));
      if (!own_lane) return;
      if (p.lo == 0) {
        double* v = p.lam_out + part * plane + off2;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (base + r < n) v[r * nq] = O[r];
      } else {
        double* v = p.out + part * plane + off2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (base + r < n) {
            v[r * nq] = X[r];
            v[2 * plane + r * nq] = Z[r];
            v[4 * plane + r * nq] = PB[r];
            v[6 * plane + r * nq] = O[r];
          }
        }
      }
    };
    // the coefficients of the next pair are loaded one pair ahead, so the
    // scalar loads' latency hides behind a pair of terms
    auto run = [&](double* X, double* Z, double* PB, double* O, int l) {
      double2 ca = coef[l], cb = coef[l >= 1 ? l - 1 : 0];
      for (; l - 1 >= lmin; l -= 2) {
        const double2 na = coef[l >= 2 ? l - 2 : 0], nb = coef[l >= 3 ? l - 3 : 0];
        term(Parity<0>{}, X, Z, PB, O, ca, false);
        term(Parity<1>{}, Z, X, O, PB, cb, false);
        ca = na;
        cb = nb;
      }
      if (l >= lmin) {
        term(Parity<0>{}, X, Z, PB, O, ca, false);
        finish(Z, X, O, PB);
      } else {
        finish(X, Z, PB, O);
      }
    };
    if constexpr (HI_ODD) {
      term(Parity<1>{}, x, z, pb, o, coef[p.hi], false);
      run(z, x, o, pb, p.hi - 1);
    } else {
      run(x, z, pb, o, p.hi);
    }
    if (own_lane) {
      const double* vq = tab + 2 * n16 + q;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (base + r < n) gsum = fma(vq[r * nq], sv[r], gsum);
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) gsum += __shfl_xor(gsum, m);
  if (lane == 0) atomicAdd(p.grad + 2 * (blockIdx.x % kAdjSlots), 2.0 * gsum);
}

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

hipError_t launch_tridiag_adj_table(const TridiagAdjStream& p, int k, bool plain_lambda,
                                    double* tab, hipStream_t s) {
  const long blocks = (p.n16 + 255) / 256;
  hipLaunchKernelGGL(tridiag_adj_table_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, k,
                     plain_lambda ? 1 : 0, tab);
  return hipGetLastError();
}

hipError_t launch_tridiag_lam_pack(const void* ubar, bool c64, long n, long ncols, long n16,
                                   double* out, hipStream_t s) {
  const long blocks = (n16 * ncols + 255) / 256;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tridiag_lam_pack_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ubar,
                     c64 ? 1 : 0, n, ncols, n16, out);
  return hipGetLastError();
}

hipError_t launch_tridiag_adj_stream(const TridiagAdjStream& p, const double* tab, bool with_k,
                                     hipStream_t s) {
  const long grid = p.ncols * p.nblk;
  if (p.n < 1 || p.ncols < 1 || p.K < 16 || p.K % 16 || p.B < 16 || p.B % 16 ||
      p.B + 2L * p.K != tridiag_stream_rows(1) || p.nblk != (p.n + p.B - 1) / p.B ||
      p.n16 != (p.n + 15) / 16 * 16 || p.plane < p.n16 * p.ncols || p.L < 1 || p.lo < 0 ||
      p.hi < p.lo || p.hi > p.L - 1 || p.hi - p.lo + 1 > p.K || grid > 0x7fffffffL ||
      !tab || !p.lam || !p.grad || (p.hi == p.L - 1 ? !p.seg : !p.in) ||
      (p.lo == 0 ? !p.lam_out : !p.out))
    return hipErrorInvalidValue;
  const double2* coef = reinterpret_cast<const double2*>(p.coef);
  const dim3 g((unsigned)grid), b(128);
  const bool odd = p.hi & 1;
  if (with_k && odd)
    hipLaunchKernelGGL((tridiag_adj_stream_kernel<true, true>), g, b, 0, s, p, tab, coef);
  else if (with_k)
    hipLaunchKernelGGL((tridiag_adj_stream_kernel<true, false>), g, b, 0, s, p, tab, coef);
  else if (odd)
    hipLaunchKernelGGL((tridiag_adj_stream_kernel<false, true>), g, b, 0, s, p, tab, coef);
  else
    hipLaunchKernelGGL((tridiag_adj_stream_kernel<false, false>), g, b, 0, s, p, tab, coef);
  return hipGetLastError();
}

hipError_t launch_tridiag_lam_gauge(const TridiagAdjStream& p, const double* tab, double* lam,
                                    hipStream_t s) {
  const long blocks = (p.plane + 255) / 256;
  if (p.n16 < 16 || p.plane < p.n16 || p.plane % p.n16 || !tab || !lam || blocks > 0x7fffffffL)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(tridiag_lam_gauge_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p.n16,
                     p.plane, tab, lam);
  return hipGetLastError();
}

hipError_t launch_tridiag_adj_persist(const TridiagAdjStream& p, const double* tab,
                                      hipStream_t s) {
  const long items = p.ncols * p.nblk;
  if (p.n < 1 || p.ncols < 1 || p.K < 16 || p.K % 16 || p.B < 16 || p.B % 16 ||
      p.B + 2L * p.K != tridiag_stream_rows(1) || p.nblk != (p.n + p.B - 1) / p.B ||
      p.n16 != (p.n + 15) / 16 * 16 || p.plane < p.n16 * p.ncols || p.L < 1 || p.lo < 0 ||
      p.hi < p.lo || p.hi > p.L - 1 || p.hi - p.lo + 1 > p.K || items > 0x7fffffffL ||
      !tab || !p.lam || !p.grad || (p.hi == p.L - 1 ? !p.seg : !p.in) ||
      (p.lo == 0 ? !p.lam_out : !p.out))
    return hipErrorInvalidValue;
  // two workgroups per CU (one wave per SIMD: the kernel holds more than 256
  // registers per lane; 64 KiB of LDS each)
  static int cus[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (cus[dev] == 0) {
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    cus[dev] = v > 0 ? v : 1;
  }
  const long grid = std::min(items, 2L * cus[dev]);
  const double2* coef = reinterpret_cast<const double2*>(p.coef);
  if (p.hi & 1)
    hipLaunchKernelGGL((tridiag_adj_persist_kernel<true>), dim3((unsigned)grid), dim3(128), 0, s, p,
                       tab, coef);
  else
    hipLaunchKernelGGL((tridiag_adj_persist_kernel<false>), dim3((unsigned)grid), dim3(128), 0, s,
                       p, tab, coef);
  return hipGetLastError();
}

}  // namespace fq
