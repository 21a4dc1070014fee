// Host FP64 numerics of the setup stage: Gauss-Legendre node times, Bessel
// expansion weights, the choice of the Chebyshev order, and Sturm-sequence
// bisection for extreme eigenvalues of Hermitian tridiagonal matrices.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "internal.h"

namespace fq {

void gl2_node_times(double T, int M, double* t_out) {
  // Nodes 1/2 -/+ sqrt(3)/6 of the two-point Gauss-Legendre rule on each step
  // [t_{k-1}, t_k], t_k = k T / M (Sec. 2, Eq. (9) grid).
  const double h = T / M;
  const double c1 = 0.5 - std::sqrt(3.0) / 6.0;
  const double c2 = 0.5 + std::sqrt(3.0) / 6.0;
  for (int k = 0; k < M; ++k) {
    t_out[2 * k] = (k + c1) * h;
    t_out[2 * k + 1] = (k + c2) * h;
  }
}

void gl3_node_times(double T, int M, double* t_out) {
  // Nodes 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10 of the three-point
  // Gauss-Legendre rule on each step, for the sixth-order scheme (Sec. 3, Eq. (14)).
  const double h = T / M;
  const double d = std::sqrt(15.0) / 10.0;
  for (int k = 0; k < M; ++k) {
    t_out[3 * k] = (k + 0.5 - d) * h;
    t_out[3 * k + 1] = (k + 0.5) * h;
    t_out[3 * k + 2] = (k + 0.5 + d) * h;
  }
}

// J_0(x) .. J_lmax(x) by Miller's backward recurrence
//   J_{l-1}(x) = (2 l / x) J_l(x) - J_{l+1}(x),
// started far above max(lmax, x) from (0, tiny) and normalised with the
// Neumann identity J_0(x) + 2 sum_{k>=1} J_{2k}(x) = 1. The forward recurrence
// is unstable for l > x; the backward one is stable (J. C. P. Miller, 1952;
// Abramowitz & Stegun, Sec. 9.12).
void bessel_j_table(double x, int lmax, std::vector<double>& out) {
  out.assign(static_cast<size_t>(lmax) + 1, 0.0);
  if (x == 0.0) {
    out[0] = 1.0;
    return;
  }
  const double big = std::max<double>(lmax, x);
  int start = static_cast<int>(big + 30.0 + 10.0 * std::cbrt(big) + 2.0 * std::sqrt(big));
  start += start & 1;  // even start so the normalisation sum sees every J_2k
  // x86-64 long double (64-bit significand) keeps the recurrence and the
  // normalisation sum well below double rounding for arguments in the
  // thousands, where the sum has many terms of alternating sign.
  using real = long double;
  std::vector<real> j(static_cast<size_t>(start) + 2, 0.0L);
  const real xl = x;
  real jp1 = 0.0L, jc = 1e-300L;
  j[start + 1] = jp1;
  j[start] = jc;
  for (int l = start; l >= 1; --l) {
    const real jm1 = (2.0L * l / xl) * jc - jp1;
    jp1 = jc;
    jc = jm1;
    j[l - 1] = jc;
    if (fabsl(jc) > 1e250L) {  // rescale to keep the recurrence in range
      for (int m = l - 1; m <= start + 1; ++m) j[m] *= 1e-250L;
      jp1 *= 1e-250L;
      jc *= 1e-250L;
    }
  }
  real norm = j[0];
  for (int m = 2; m <= start; m += 2) norm += 2.0L * j[m];
  for (int l = 0; l <= lmax; ++l) out[l] = static_cast<double>(j[l] / norm);
}

int choose_order(double R, double tol) {
  // Smallest L with 2 sum_{l>L} |J_l(R)| <= tol: a rigorous bound of the
  // truncation error when the rescaled spectrum lies in [-1, 1] (|T_l| <= 1).
  const int lmax = static_cast<int>(R + 40.0 + 12.0 * std::cbrt(std::max(R, 1.0))) + 64;
  std::vector<double> j;
  bessel_j_table(R, lmax, j);
  std::vector<double> tail(static_cast<size_t>(lmax) + 2, 0.0);
  for (int l = lmax; l >= 0; --l) tail[l] = tail[l + 1] + 2.0 * std::fabs(j[l]);
  for (int L = 1; L < lmax; ++L)
    if (tail[L + 1] <= tol) return L;
  return -1;
}

// Number of eigenvalues < x of the Hermitian tridiagonal matrix (d, e_abs),
// from the signs of the pivots of the LDL^T factorisation of T - x 1
// (Sylvester's law of inertia; the "Sturm count").
static long sturm_count(long n, const double* d, const double* e2, double x, double pivmin) {
  // A pivot that vanishes is replaced by -pivmin before its sign is taken, so
  // the count and the next pivot see the same value.
  long count = 0;
  double q = d[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++count;
  for (long i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++count;
  }
  return count;
}

void tridiag_extremes(long n, const double* d, const double* e_abs, double* lo_out,
                      double* hi_out) {
  if (n == 1) {
    *lo_out = *hi_out = d[0];
    return;
  }
  std::vector<double> e2(n - 1);
  double glo = d[0], ghi = d[0], e2max = 1.0;
  for (long i = 0; i < n; ++i) {
    const double r = (i > 0 ? e_abs[i - 1] : 0.0) + (i + 1 < n ? e_abs[i] : 0.0);
    glo = std::min(glo, d[i] - r);
    ghi = std::max(ghi, d[i] + r);
    if (i + 1 < n) {
      e2[i] = e_abs[i] * e_abs[i];
      e2max = std::max(e2max, e2[i]);
    }
  }
  const double pivmin = std::numeric_limits<double>::min() * e2max;
  const double span = std::max(ghi - glo, std::max(std::fabs(glo), std::fabs(ghi)) * 1e-300);
  glo -= 1e-14 * span + 1e-300;
  ghi += 1e-14 * span + 1e-300;
  // lambda_min: smallest x with count(x) >= 1; lambda_max: smallest x with count(x) >= n.
  auto bisect = [&](long target) {
    double a = glo, b = ghi;
    for (int it = 0; it < 200; ++it) {
      const double m = 0.5 * (a + b);
      if (m <= a || m >= b) break;
      if (sturm_count(n, d, e2.data(), m, pivmin) >= target)
        b = m;
      else
        a = m;
    }
    return std::make_pair(a, b);
  };
  auto lo = bisect(1);
  auto hi = bisect(n);
  *lo_out = lo.first;   // count(a) < 1 <= count(b): lambda_min in [a, b)
  *hi_out = hi.second;  // count(a) < n <= count(b): lambda_max in [a, b)
}

// A Hermitian tridiagonal matrix with couplings e_i = H[i][i+1] is unitarily
// similar, through D = diag(w), to the real one with couplings |e_i|:
// (D^+ H D)[i][i+1] = conj(w_i) e_i w_{i+1} = |e_i| when w_{i+1} = w_i conj(e_i) / |e_i|.
// The prefix product runs sequentially in 80-bit arithmetic and every factor
// is renormalised, so each ratio w_{i+1} / w_i matches conj(e_i / |e_i|) to
// one rounding however long the chain. For the Magnus-4 step operator
// e_i = h_i (1 - i b (v_{i+1} - v_i)) (the 1/dE scale does not change phases).
void tridiag_gauge(long n, const double* h0_off, const double* v_diag, double b, double* w_out) {
  long double wr = 1.0L, wi = 0.0L;
  w_out[0] = 1.0;
  w_out[1] = 0.0;
  for (long i = 0; i + 1 < n; ++i) {
    const long double hr = h0_off[2 * i], hi = h0_off[2 * i + 1];
    const long double q = (long double)b * ((long double)v_diag[i + 1] - v_diag[i]);
    const long double er = hr + hi * q, ei = hi - hr * q;  // h (1 - i q)
    const long double m = sqrtl(er * er + ei * ei);
    long double ur = 1.0L, ui = 0.0L;
    if (m > 0.0L) {
      ur = er / m;
      ui = ei / m;
    }
    const long double nr = wr * ur + wi * ui, ni = wi * ur - wr * ui;  // w conj(u)
    const long double nm = sqrtl(nr * nr + ni * ni);
    wr = nr / nm;
    wi = ni / nm;
    w_out[2 * (i + 1)] = (double)wr;
    w_out[2 * (i + 1) + 1] = (double)wi;
  }
}

}  // namespace fq
