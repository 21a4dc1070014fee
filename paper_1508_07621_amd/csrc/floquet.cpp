// C-ABI driver of libfloquet: argument checks, host FP64 setup, workspace
// layout and the step loops that enqueue the HIP kernels on one stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "context.h"

using fq::ChebTerm;

namespace {

thread_local std::string g_err;

fq_status fail(fq_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define FQ_HIP(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      if (ctx) (ctx)->broken = true;                                                       \
      return fail(FQ_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));             \
    }                                                                                      \
  } while (0)

#define FQ_TRY(expr)                 \
  do {                               \
    fq_status s_ = (expr);           \
    if (s_ != FQ_OK) return s_;      \
  } while (0)

// Zero `bytes` (a multiple of 8) of device memory with a fill kernel on the
// context's stream (a kernel rather than hipMemsetAsync, so that the same
// sequence can be recorded into a graph by a caller).
hipError_t zero_async(hipStream_t s, void* p, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  return fq::launch_fill_zero(static_cast<double*>(p), (long)(bytes / sizeof(double)), s);
}

// Device-to-host or host-to-device copy ordered on the context's stream and
// complete on return (the caller's stream may be a non-blocking stream, which
// the legacy null stream of a plain hipMemcpy does not wait for).
hipError_t copy_sync(hipStream_t s, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

constexpr size_t kAlign = 256;
constexpr int kMaxOrder = 65535;       // capacity of the device coefficient table
// Lanczos steps for the dense covers and the relative widening of their Ritz
// extremes (see lanczos_ritz): with a start vector uniform on the sphere, k
// steps leave an extreme Ritz value more than a fraction eps of the spread
// inside the spectrum with probability at most 1.648 sqrt(n) exp(-sqrt(eps) (2k - 1))
// (Kuczynski and Wozniakowski, SIAM J. Matrix Anal. Appl. 13 (1992)); at
// eps = 0.01, k = 200 this is below 1e-14 for n up to 10^6.
constexpr int kLanczosSteps = 200;
constexpr double kDenseMargin = 0.01;
// A build whose max |(U^dagger U - 1)_ij| exceeds this is reported as diverged.
constexpr double kDivergence = 1e-3;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

long dense_tile(long n) { return n >= 1024 ? 128 : 64; }
long pad_to(long x, long t) { return (x + t - 1) / t * t; }

// Terms per pass of the streamed tridiagonal gradient (a multiple of 16;
// windows of tridiag_stream_rows(1) rows hold 2K ghost and B = rows - 2K owned
// rows): the K that minimises passes x windows x (overhead + terms per pass)
// for `terms` terms per step over columns of n rows. The overhead is a pass
// window's cost beyond its terms, in terms, measured on the 10^4-row dimer
// (24-step gradients with K = 112, 128, 144): 60 for the reverse pass. A short
// last window costs a full one, which is why K = 128 (14 windows, the last
// with 16 owned rows) lost 3 % against K = 144 there. kmax: the reverse pass
// with the K contraction stages at most 128 of its coefficients in LDS.
int stream_pass_terms(long n, int terms, double overhead, int kmax) {
  const long rows = fq::tridiag_stream_rows(1);
  int best = 64;
  double best_cost = 0.0;
  for (int K = 64; K <= kmax && rows - 2L * K >= 256; K += 16) {
    const long B = rows - 2L * K;
    const long passes = (terms + K - 1) / K, windows = (n + B - 1) / B;
    const double cost = (double)passes * (double)windows * (overhead + (double)terms / passes);
    if (best_cost == 0.0 || cost < best_cost) {
      best_cost = cost;
      best = K;
    }
  }
  return best;
}
constexpr double kStreamOverheadRev = 60.0;

bool is_finite(double x) { return std::isfinite(x); }

int nodes_per_step(int scheme) { return scheme == FQ_MAGNUS6 ? 3 : 2; }

// Layouts served by the dense path (H0 given densely or by its eigenvalues).
bool dense_like(int layout) { return layout == FQ_DENSE || layout == FQ_DENSE_EIGEN; }

// Drive terms S and the matrices J of the drive block (see fq_ctx).
int drive_terms(const fq_system* sys) { return sys->n_drive >= 2 ? sys->n_drive : 1; }
int drive_block(int S, int scheme) {
  if (S == 1) return 2;
  return scheme == FQ_CF4 ? S : 2 * S + S * (S - 1) / 2;
}

// Exponentials per step: FQ_CF4 runs each step as two half-steps. Inside the
// library M, h, the checkpoint spacing and every table count these substeps;
// the entry points map step indices of the caller to them.
int substeps_per_step(int scheme) { return scheme == FQ_CF4 ? 2 : 1; }

// FQ_CF4: weights of f1, f2 in the Hmod coefficient of the first and the second
// half-step, 2 (a1, a2) and 2 (a2, a1) with a1,2 = 1/4 +/- sqrt(3)/6.
constexpr double kCf4P = 0.5 + 0.57735026918962576451;  // 1/2 + sqrt(3)/3
constexpr double kCf4Q = 0.5 - 0.57735026918962576451;  // 1/2 - sqrt(3)/3

// Number of nested commutators in the sixth-order effective Hamiltonian.
constexpr int kComm6 = 9;

struct Layout {
  size_t total = 0;
  size_t off_h0 = 0, off_v = 0, off_k = 0, off_ht = 0, off_x = 0, off_y = 0, off_pa = 0,
         off_pb = 0, off_pc = 0, off_htx = 0, off_tape = 0, off_small = 0, off_ab = 0, off_coef = 0,
         off_seg = 0, off_stack = 0, off_lam = 0, off_grad = 0, off_gauge = 0, off_stream = 0,
         off_adj = 0,
         off_comm6 = 0, off_vec = 0, off_drive32 = 0;
  long np = 0;
  int n_tape = 0;
};

// The tridiagonal gradient of columns longer than one workgroup holds runs as
// streamed passes (tridiag_adjoint_streamed). FQ_TRIDIAG_STREAMED_ADJOINT=1 in
// the environment selects that form for every n (it gives the same derivative
// as the per-column sweep; tests compare the two).
bool streamed_adjoint(const fq_system* sys, const fq_params* par) {
  if (sys->layout != FQ_TRIDIAG || par->checkpoint_every <= 0) return false;
  if (sys->n > fq::tridiag_adjoint_max_n()) return true;
  const char* e = std::getenv("FQ_TRIDIAG_STREAMED_ADJOINT");
  return e && e[0] == '1' && e[1] == 0;
}

Layout plan(const fq_system* sys, const fq_params* par) {
  Layout lay;
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    size_t o = cur;
    cur = align_up(cur + bytes);
    return o;
  };
  const long n = sys->n;
  // substeps and checkpoint spacing as the library runs them
  const int spp = substeps_per_step(par->scheme);
  const long Ms = (long)par->M * spp, cks = (long)par->checkpoint_every * spp;
  const int J = drive_block(drive_terms(sys), par->scheme);
  if (dense_like(sys->layout)) {
    lay.np = pad_to(n, dense_tile(n));
    const size_t plane2 = 2 * sizeof(double) * (size_t)lay.np * (size_t)lay.np;
    lay.off_h0 = take(plane2);
    // The drive block (Hmod and K, or the drive matrices and their commutators)
    // is laid out re(B_0), re(B_1), ..., im(B_0), im(B_1), ..., so that
    // [B_0; B_1; ...] is one J np-row operand for the gradient contraction.
    lay.off_v = take((size_t)J * plane2);
    lay.off_k = lay.off_v;
    lay.off_ht = take(plane2);
    lay.off_x = take(plane2);
    lay.off_y = take(plane2);
    // P buffers hold FP64 planes, or the product format (BF16X3: six 16-bit planes)
    const size_t pbytes = par->precision == FQ_BF16X3
                              ? std::max(plane2, sizeof(uint16_t) * fq::BF3_PLANES *
                                                     (size_t)lay.np * (size_t)lay.np)
                              : plane2;
    lay.off_pa = take(pbytes);
    lay.off_pb = take(pbytes);
    if (par->precision != FQ_FP64) lay.off_pc = take(pbytes);
    if (par->precision != FQ_FP64) lay.off_htx = take(pbytes);
    if (par->scheme == FQ_MAGNUS6) lay.off_comm6 = take(kComm6 * plane2);
    if (par->checkpoint_every > 0) {
      lay.n_tape = (Ms + cks - 1) / cks + 1;
      lay.off_tape = take(plane2 * (size_t)lay.n_tape);
      lay.off_seg = take(3 * plane2 * (size_t)cks);
      lay.off_stack = take(4 * plane2);
      lay.off_lam = take(plane2);
      lay.off_grad = take((size_t)J * sizeof(double) * (size_t)Ms);
      if (par->precision == FQ_FP32)  // the drive block in FP32 planes for the reverse products
        lay.off_drive32 = take((size_t)J * 2 * sizeof(float) * (size_t)lay.np * (size_t)lay.np);
    }
  } else {
    lay.np = pad_to(n, dense_tile(n));
    const size_t plane2 = 2 * sizeof(double) * (size_t)lay.np * (size_t)lay.np;
    lay.off_x = take(plane2);  // planar copy of U_T for the unitarity check
    if (par->reorthonormalize) {  // Newton-Schulz scratch: X X^dagger, X^T, next X
      lay.off_pa = take(plane2);
      lay.off_pb = take(plane2);
      lay.off_y = take(plane2);
    }
    lay.off_gauge = take(2 * sizeof(double) * (size_t)n * (size_t)Ms);
    const bool streamed_grad = streamed_adjoint(sys, par);
    const size_t n16 = (size_t)(n + 15) / 16 * 16;
    const size_t splane = sizeof(double) * n16 * (size_t)n;  // one state plane
    if (n > fq::tridiag_resident_max_n() || streamed_grad)  // two 8-plane states, per-step rows
      lay.off_stream = take(2 * 8 * splane + sizeof(double) * 6 * n16);
    if (par->checkpoint_every > 0) {  // X_{j ckpt} per column; segment buffers
      const size_t vec = 2 * sizeof(double) * (size_t)n;
      lay.n_tape = (Ms + cks - 1) / cks + 1;
      lay.off_tape = take(vec * (size_t)n * (size_t)lay.n_tape);
      if (streamed_grad) {
        // per step of a segment P_{L-1}, P_L (4 planes); two 8-plane pass
        // states, two 2-plane Lambdas and the per-step tables; slotted sums
        lay.off_seg = take(4 * splane * (size_t)cks);
        lay.off_adj = take(20 * splane + sizeof(double) * 7 * n16);
        lay.off_grad = take(2 * sizeof(double) * fq::kAdjSlots * (size_t)Ms);
      } else {  // per column: X_k, P_{L-1}, P_L of every step of a segment
        lay.off_seg = take(vec * (size_t)n * 3 * (size_t)cks);
        lay.off_grad = take(2 * sizeof(double) * (size_t)Ms);
      }
    }
  }
  lay.off_small = take(64 * sizeof(double));
  lay.off_vec = take(3 * sizeof(double) * (size_t)n);
  lay.off_ab = take(2 * sizeof(double) * (size_t)Ms);
  lay.off_coef = take(2 * sizeof(double) * (size_t)(kMaxOrder + 1));
  lay.total = cur;
  return lay;
}

fq_status validate(const fq_system* sys, const fq_params* par) {
  if (!sys || !par) return fail(FQ_ERR_ARG, "null system or params");
  if (sys->n < 1) return fail(FQ_ERR_ARG, "n must be >= 1 (got %lld)", (long long)sys->n);
  if (sys->n_drive < 0 || sys->n_drive > 4)
    return fail(FQ_ERR_ARG, "n_drive must be in [0, 4] (got %d)", sys->n_drive);
  if (sys->n_drive >= 2) {
    if (!dense_like(sys->layout))
      return fail(FQ_ERR_UNSUPPORTED, "several drive terms need a dense layout");
    if (!sys->hmods) return fail(FQ_ERR_ARG, "n_drive >= 2 needs hmods");
    for (int d = 0; d < sys->n_drive; ++d)
      if (!sys->hmods[d]) return fail(FQ_ERR_ARG, "hmods[%d] is null", d);
  }
  if (sys->layout == FQ_DENSE) {
    if (!sys->h0 || (!sys->hmod && sys->n_drive < 2))
      return fail(FQ_ERR_ARG, "dense layout needs h0 and hmod");
    if (sys->n > 46336) return fail(FQ_ERR_ARG, "n too large for 32-bit tile indexing");
  } else if (sys->layout == FQ_DENSE_EIGEN) {
    if (!sys->h0_diag || (!sys->hmod && sys->n_drive < 2))
      return fail(FQ_ERR_ARG, "eigenbasis layout needs h0_diag (eigenvalues of H0) and hmod");
    if (sys->n > 46336) return fail(FQ_ERR_ARG, "n too large for 32-bit tile indexing");
  } else if (sys->layout == FQ_TRIDIAG) {
    if (!sys->h0_diag || !sys->hmod_diag || (sys->n > 1 && !sys->h0_off))
      return fail(FQ_ERR_ARG, "tridiagonal layout needs h0_diag, h0_off and hmod_diag");
  } else {
    return fail(FQ_ERR_ARG, "unknown layout %d", sys->layout);
  }
  if (!is_finite(par->T) || par->T <= 0) return fail(FQ_ERR_ARG, "T must be finite and > 0");
  if (par->M < 1) return fail(FQ_ERR_ARG, "M must be >= 1");
  if (!par->f_nodes) return fail(FQ_ERR_ARG, "f_nodes is null");
  if (par->scheme != FQ_MAGNUS4 && par->scheme != FQ_MAGNUS6 && par->scheme != FQ_CF4)
    return fail(FQ_ERR_ARG, "scheme must be FQ_MAGNUS4, FQ_MAGNUS6 or FQ_CF4");
  if (par->M > 0x3fffffff / substeps_per_step(par->scheme)) return fail(FQ_ERR_ARG, "M too large");
  if (drive_terms(sys) > 1 && par->scheme == FQ_MAGNUS6)
    return fail(FQ_ERR_UNSUPPORTED, "FQ_MAGNUS6 takes one drive term");
  for (int i = 0; i < nodes_per_step(par->scheme) * par->M * drive_terms(sys); ++i)
    if (!is_finite(par->f_nodes[i])) return fail(FQ_ERR_NONFINITE, "f_nodes[%d] is not finite", i);
  if (par->L < 0 || par->L > kMaxOrder) return fail(FQ_ERR_ARG, "L out of range [0, %d]", kMaxOrder);
  if (par->L == 0 && (!is_finite(par->tol) || par->tol <= 0))
    return fail(FQ_ERR_ARG, "tol must be finite and > 0 when L == 0");
  const bool nmin = std::isnan(par->e_min), nmax = std::isnan(par->e_max);
  if (nmin != nmax) return fail(FQ_ERR_ARG, "give both e_min and e_max, or neither (NaN)");
  if (!nmin) {
    if (!is_finite(par->e_min) || !is_finite(par->e_max))
      return fail(FQ_ERR_NONFINITE, "spectral interval is not finite");
    if (!(par->e_max > par->e_min)) return fail(FQ_ERR_SPECTRUM, "need e_max > e_min");
  }
  if (par->precision < FQ_FP64 || par->precision > FQ_BF16X3)
    return fail(FQ_ERR_ARG, "unknown precision %d", par->precision);
  if (!is_finite(par->mixed_tol) || par->mixed_tol < 0)
    return fail(FQ_ERR_ARG, "mixed_tol must be finite and >= 0");
  if (par->n_term_formats < 0 || (par->n_term_formats > 0) != (par->term_formats != nullptr))
    return fail(FQ_ERR_ARG, "term_formats and n_term_formats must be given together");
  if (par->n_term_formats > 0) {
    if (par->precision != FQ_BF16X3)
      return fail(FQ_ERR_ARG, "term_formats apply to FQ_BF16X3 builds only");
    bool f64_run = true;
    for (int l = 0; l < par->n_term_formats; ++l) {
      const int f = par->term_formats[l];
      if (f < FQ_TERM_FP64 || f > FQ_TERM_BF16X1)
        return fail(FQ_ERR_ARG, "term_formats[%d] = %d is not an fq_term_format", l, f);
      if (f == FQ_TERM_FP64 && !f64_run)
        return fail(FQ_ERR_ARG, "FQ_TERM_FP64 only on a leading run of terms (term_formats[%d])", l);
      f64_run = f64_run && f == FQ_TERM_FP64;
    }
  }
  if (par->grad_pair_sums != 0 && par->grad_pair_sums != 1)
    return fail(FQ_ERR_ARG, "grad_pair_sums must be 0 or 1");
  if (par->checkpoint_every < 0) return fail(FQ_ERR_ARG, "checkpoint_every must be >= 0");
  if (par->profile != 0 && par->profile != 1) return fail(FQ_ERR_ARG, "profile must be 0 or 1");
  if (par->reorthonormalize != 0 && par->reorthonormalize != 1)
    return fail(FQ_ERR_ARG, "reorthonormalize must be 0 or 1");
  if (par->dtype != FQ_C128 && par->dtype != FQ_C64)
    return fail(FQ_ERR_ARG, "dtype must be FQ_C128 or FQ_C64");
  if (par->scheme == FQ_MAGNUS6) {
    if (!dense_like(sys->layout))
      return fail(FQ_ERR_UNSUPPORTED, "FQ_MAGNUS6 needs a dense layout (its nested "
                                      "commutators of a tridiagonal H0 are not tridiagonal)");
    if (par->checkpoint_every > 0)
      return fail(FQ_ERR_UNSUPPORTED, "the gradient tape is implemented for FQ_MAGNUS4 only");
  }
  if (sys->layout == FQ_TRIDIAG) {
    if (par->precision != FQ_FP64)
      return fail(FQ_ERR_UNSUPPORTED, "tridiagonal layout runs in FP64 only");
    // beyond one workgroup's column (4096 rows) the streamed passes keep two
    // 8-plane n x n FP64 states in the workspace (128 n^2 bytes)
    if (sys->n > 40000)
      return fail(FQ_ERR_UNSUPPORTED, "tridiagonal n > 40000 not supported");
  }
  return FQ_OK;
}

// ---- the sixth-order scheme -------------------------------------------------------------------
//
// For H(t) = H0 + f(t) V and A = -i H, the three-point Gauss-Legendre alphas of
// Eq. (14) are alpha_1 = -i (h H0 + a V), alpha_2 = -i g2 V, alpha_3 = -i g3 V with
//   a = h f2,  g2 = (sqrt(15) h / 3)(f3 - f1),  g3 = (10 h / 3)(f3 - 2 f2 + f1).
// Writing K1 = [H0, V] (anti-Hermitian) and expanding C_1, C_2 and the bracket,
// every term is a real multiple of one of the Hermitian matrices
//   B1 = i K1,          B2 = [H0, K1],        B3 = [V, K1],
//   B4 = i [H0, B2],    B5 = i [H0, B3],      B6 = i [V, B2],    B7 = i [V, B3],
//   B8 = [K1, B2],      B9 = [K1, B3],
// and H_eff = i Omega / h = H0 + (f2 + g3 / (12 h)) V + sum_j w_j B_j with
//   w1 = g2 / 12,                 w2 = -g3 h / 360,
//   w3 = (g2^2 - (20 a + g3) g3 / 30) / 240,
//   w4 = h^2 g2 / 720,            w5 = h a g2 / 720,
//   w6 = (20 a + g3) h g2 / 14400, w7 = (20 a + g3) a g2 / 14400,
//   w8 = -h^2 g2^2 / 14400,       w9 = -h a g2^2 / 14400.
// (A constant drive gives g2 = g3 = 0 and H_eff = H0 + f V.)
void magnus6_weights(double h, double f1, double f2, double f3, double* wv, double* w) {
  const double a = h * f2;
  const double g2 = std::sqrt(15.0) * h / 3.0 * (f3 - f1);
  const double g3 = 10.0 * h / 3.0 * (f3 - 2.0 * f2 + f1);
  const double q = 20.0 * a + g3;
  *wv = f2 + g3 / (12.0 * h);
  w[0] = g2 / 12.0;
  w[1] = -g3 * h / 360.0;
  w[2] = (g2 * g2 - q * g3 / 30.0) / 240.0;
  w[3] = h * h * g2 / 720.0;
  w[4] = h * a * g2 / 720.0;
  w[5] = q * h * g2 / 14400.0;
  w[6] = q * a * g2 / 14400.0;
  w[7] = -h * h * g2 * g2 / 14400.0;
  w[8] = -h * a * g2 * g2 / 14400.0;
}

// B = s i [P, Q] for Hermitian P, Q on FP64 matrix cores: (P Q)(i, j) =
// sum_k P(i, k) conj(Q(j, k)), and likewise Q P.
fq_status hermitian_commutator(fq_ctx* c, const double* pr, const double* pi, const double* qr,
                               const double* qi, double s, double* br, double* bi) {
  const int np = (int)c->np;
  if (c->h0_eigen && pr == c->h0r) {  // [diag(E), Q] elementwise
    FQ_HIP(c, fq::launch_diag_commutator(c->sys.h0_diag, c->n, np, qr, qi, s, br, bi, c->stream));
    return FQ_OK;
  }
  FQ_HIP(c, fq::launch_zgemm_nt_f64(pr, pi, false, qr, qi, true, br, bi, np, np, np, np, 0.0, s,
                                    0.0, 0.0, c->stream));
  FQ_HIP(c, fq::launch_zgemm_nt_f64(qr, qi, false, pr, pi, true, br, bi, np, np, np, np, 0.0, -s,
                                    1.0, 0.0, c->stream));
  return FQ_OK;
}

// The nine B_j of the sixth-order scheme from the planar H0 and V.
fq_status magnus6_commutators(fq_ctx* c) {
  const size_t plane = (size_t)c->np * (size_t)c->np;
  auto re = [&](int j) { return c->comm6 + 2 * plane * j; };
  auto im = [&](int j) { return c->comm6 + 2 * plane * j + plane; };
  // K1 = -i B1, so [X, K1] = -i [X, B1] and [K1, Y] = -i [B1, Y]
  FQ_TRY(hermitian_commutator(c, c->h0r, c->h0i, c->vr, c->vi, 1.0, re(0), im(0)));   // B1
  FQ_TRY(hermitian_commutator(c, c->h0r, c->h0i, re(0), im(0), -1.0, re(1), im(1)));  // B2
  FQ_TRY(hermitian_commutator(c, c->vr, c->vi, re(0), im(0), -1.0, re(2), im(2)));    // B3
  FQ_TRY(hermitian_commutator(c, c->h0r, c->h0i, re(1), im(1), 1.0, re(3), im(3)));   // B4
  FQ_TRY(hermitian_commutator(c, c->h0r, c->h0i, re(2), im(2), 1.0, re(4), im(4)));   // B5
  FQ_TRY(hermitian_commutator(c, c->vr, c->vi, re(1), im(1), 1.0, re(5), im(5)));     // B6
  FQ_TRY(hermitian_commutator(c, c->vr, c->vi, re(2), im(2), 1.0, re(6), im(6)));     // B7
  FQ_TRY(hermitian_commutator(c, re(0), im(0), re(1), im(1), -1.0, re(7), im(7)));    // B8
  FQ_TRY(hermitian_commutator(c, re(0), im(0), re(2), im(2), -1.0, re(8), im(8)));    // B9
  return FQ_OK;
}

// Into (outr, outi): sum_j w6[k][j] B_j, plus H0 + a_k V when with_base.
fq_status magnus6_sum(fq_ctx* c, int k, bool with_base, double* outr, double* outi) {
  const size_t plane = (size_t)c->np * (size_t)c->np;
  fq::WeightedSum ws{};
  int t = 0;
  if (with_base) {
    ws.re[t] = c->h0r; ws.im[t] = c->h0i; ws.w[t++] = 1.0;
    ws.re[t] = c->vr;  ws.im[t] = c->vi;  ws.w[t++] = c->a[k];
  }
  for (int j = 0; j < kComm6; ++j) {
    ws.re[t] = c->comm6 + 2 * plane * j;
    ws.im[t] = c->comm6 + 2 * plane * j + plane;
    ws.w[t++] = c->w6[(size_t)kComm6 * k + j];
  }
  ws.count = t;
  FQ_HIP(c, fq::launch_weighted_sum(ws, (long)plane, outr, outi, c->stream));
  return FQ_OK;
}

// Several drive terms: into (outr, outi) sum_j wS[k][j] B_j over the drive
// block, plus H0 when with_base (the (sub)step's H_eff).
fq_status drive_sum(fq_ctx* c, int k, bool with_base, double* outr, double* outi) {
  const size_t plane = (size_t)c->np * (size_t)c->np;
  fq::WeightedSum ws{};
  int t = 0;
  if (with_base) {
    ws.re[t] = c->h0r; ws.im[t] = c->h0i; ws.w[t++] = 1.0;
  }
  for (int j = 0; j < c->J; ++j) {
    ws.re[t] = c->vr + (size_t)j * plane;
    ws.im[t] = c->vi + (size_t)j * plane;
    ws.w[t++] = c->wS[(size_t)c->J * k + j];
  }
  ws.count = t;
  FQ_HIP(c, fq::launch_weighted_sum(ws, (long)plane, outr, outi, c->stream));
  return FQ_OK;
}

// ---- spectral interval ------------------------------------------------------------------------

using cd = std::complex<double>;
using Matvec = std::function<fq_status(const std::vector<cd>&, std::vector<cd>&)>;

// y = A x for a dense complex128 device matrix, through the device scratch
// (the Y planes are free during setup).
fq_status device_matvec(fq_ctx* ctx, const void* A, const std::vector<cd>& x, std::vector<cd>& y) {
  const long n = ctx->n;
  void* dx = ctx->yr;
  void* dy = ctx->yr + 2 * n;
  y.resize(n);
  FQ_HIP(ctx, hipMemcpyAsync(dx, x.data(), n * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
  FQ_HIP(ctx, fq::launch_zgemv(A, n, dx, dy, ctx->stream));
  FQ_HIP(ctx, hipMemcpyAsync(y.data(), dy, n * sizeof(cd), hipMemcpyDeviceToHost, ctx->stream));
  FQ_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return FQ_OK;
}

// y = A x for a planar (re, im) device matrix with row stride np.
fq_status device_matvec_planar(fq_ctx* ctx, const double* ar, const double* ai,
                               const std::vector<cd>& x, std::vector<cd>& y) {
  const long n = ctx->n;
  void* dx = ctx->yr;
  void* dy = ctx->yr + 2 * n;
  y.resize(n);
  FQ_HIP(ctx, hipMemcpyAsync(dx, x.data(), n * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
  FQ_HIP(ctx, fq::launch_zgemv_planar(ar, ai, n, ctx->np, dx, dy, ctx->stream));
  FQ_HIP(ctx, hipMemcpyAsync(y.data(), dy, n * sizeof(cd), hipMemcpyDeviceToHost, ctx->stream));
  FQ_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return FQ_OK;
}

// Extreme Ritz values of a Hermitian operator after k Lanczos steps. The start
// vector is drawn from a generator seeded with a hash of A x0 for a fixed x0,
// so it is not fixed in advance of the operator (no operator can be chosen with
// its extreme eigenvector orthogonal to a known start) and the same operator
// always gets the same start (reproducible covers). Ritz values lie inside
// [lambda_min, lambda_max] and converge to its ends fastest; the probability
// bound above applies to starts uniform on the sphere, which complex Gaussian
// components give after normalisation.
fq_status lanczos_extremes(long n, const Matvec& mv, double* lo, double* hi) {
  std::vector<cd> q(n), qp(n, 0.0), w(n);
  // hash of A x0, x0 = (1, 1, ..., 1) / sqrt(n)
  for (long i = 0; i < n; ++i) q[i] = cd(1.0 / std::sqrt((double)n), 0.0);
  fq_status st = mv(q, w);
  if (st != FQ_OK) return st;
  uint64_t s = 0x9E3779B97F4A7C15ull ^ (uint64_t)n;
  for (long i = 0; i < n; ++i) {
    uint64_t bits[2];
    std::memcpy(bits, &w[i], sizeof bits);
    for (uint64_t b : bits) {
      s ^= b + 0x9E3779B97F4A7C15ull + (s << 6) + (s >> 2);
      s *= 0xBF58476D1CE4E5B9ull;
      s ^= s >> 31;
    }
  }
  if (s == 0) s = 1;
  auto next = [&]() {  // xorshift64, then uniform in (0, 1)
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return ((double)(s >> 11) + 0.5) / 9007199254740992.0;
  };
  double nrm = 0.0;
  for (long i = 0; i < n; ++i) {  // complex Gaussian components (Box-Muller)
    const double r = std::sqrt(-2.0 * std::log(next())), t = 6.283185307179586 * next();
    q[i] = cd(r * std::cos(t), r * std::sin(t));
    nrm += std::norm(q[i]);
  }
  nrm = std::sqrt(nrm);
  for (auto& v : q) v /= nrm;
  const int ksteps = (int)std::min<long>(n, kLanczosSteps);
  std::vector<double> alpha, beta;
  double bprev = 0.0;
  for (int j = 0; j < ksteps; ++j) {
    st = mv(q, w);
    if (st != FQ_OK) return st;
    double a = 0.0;
    for (long i = 0; i < n; ++i) a += std::real(std::conj(q[i]) * w[i]);
    double b2 = 0.0;
    for (long i = 0; i < n; ++i) {
      w[i] -= a * q[i] + bprev * qp[i];
      b2 += std::norm(w[i]);
    }
    alpha.push_back(a);
    const double b = std::sqrt(b2);
    if (j + 1 == ksteps || b <= 1e-13 * (std::fabs(a) + bprev + 1e-300)) break;
    beta.push_back(b);
    for (long i = 0; i < n; ++i) {
      qp[i] = q[i];
      q[i] = w[i] / b;
    }
    bprev = b;
  }
  fq::tridiag_extremes((long)alpha.size(), alpha.data(), beta.data(), lo, hi);
  return FQ_OK;
}

fq_status lanczos_ritz(fq_ctx* ctx, const Matvec& mv, double* lo, double* hi) {
  return lanczos_extremes(ctx->n, mv, lo, hi);
}

// Ritz extremes of one of the context's fixed operators (key: its device
// pointer), computed once per context: fq_set_drive reuses them.
fq_status cached_ritz(fq_ctx* ctx, const void* key, const Matvec& mv, double* lo, double* hi) {
  for (const auto& e : ctx->ritz_cache)
    if (e.first == key) {
      *lo = e.second.first;
      *hi = e.second.second;
      return FQ_OK;
    }
  FQ_TRY(lanczos_ritz(ctx, mv, lo, hi));
  ctx->ritz_cache.push_back({key, {*lo, *hi}});
  return FQ_OK;
}

// Outer estimate of the union of spec(H_eff,k): Weyl's inequalities on the
// Lanczos extremes of H0 and Hmod (each widened by `margin` of its spread, as
// Ritz values approach the ends from inside) and ||K||_2 <= 2 ||H0|| ||Hmod||.
fq_status dense_cover(fq_ctx* ctx, double* lo_out, double* hi_out, double margin) {
  double l0, h0, lv, hv;
  Matvec mh0 = [&](const std::vector<cd>& x, std::vector<cd>& y) { return device_matvec(ctx, ctx->sys.h0, x, y); };
  Matvec mv = [&](const std::vector<cd>& x, std::vector<cd>& y) { return device_matvec(ctx, ctx->sys.hmod, x, y); };
  fq_status st = FQ_OK;
  if (ctx->h0_eigen) {  // the extremes of diag(E) are exact
    std::vector<double> e(ctx->n);
    FQ_HIP(ctx, copy_sync(ctx->stream, e.data(), ctx->sys.h0_diag, ctx->n * sizeof(double),
                          hipMemcpyDeviceToHost));
    l0 = *std::min_element(e.begin(), e.end());
    h0 = *std::max_element(e.begin(), e.end());
  } else {
    st = cached_ritz(ctx, ctx->sys.h0, mh0, &l0, &h0);
    if (st != FQ_OK) return st;
  }
  if (ctx->S > 1) {
    // Weyl over the drive terms with their Lanczos extremes; ||K_s|| <= 2 ||H0|| ||Hmod_s||,
    // ||K_st|| <= 2 ||Hmod_s|| ||Hmod_t||
    const int S = ctx->S, J = ctx->J;
    const double w0 = h0 - l0;
    l0 -= margin * w0;
    h0 += margin * w0;
    const double n0 = std::max(std::fabs(l0), std::fabs(h0));
    std::vector<double> ls(S), hs(S), nb(J, 0.0);
    for (int d = 0; d < S; ++d) {
      Matvec md = [&](const std::vector<cd>& x, std::vector<cd>& y) {
        return device_matvec(ctx, ctx->sys.hmods[d], x, y);
      };
      FQ_TRY(cached_ritz(ctx, ctx->sys.hmods[d], md, &ls[d], &hs[d]));
      const double wd = hs[d] - ls[d];
      ls[d] -= margin * wd;
      hs[d] += margin * wd;
      nb[d] = std::max(std::fabs(ls[d]), std::fabs(hs[d]));
    }
    if (ctx->scheme == FQ_MAGNUS4) {
      int q = 2 * S;
      for (int d = 0; d < S; ++d) {
        nb[S + d] = 2.0 * n0 * nb[d];
        for (int e = d + 1; e < S; ++e, ++q) nb[q] = 2.0 * nb[d] * nb[e];
      }
    }
    double lo = std::numeric_limits<double>::infinity(), hi = -lo;
    for (int k = 0; k < ctx->M; ++k) {
      const double* w = &ctx->wS[(size_t)J * k];
      double l = l0, u = h0;
      for (int d = 0; d < S; ++d) {
        l += std::min(w[d] * ls[d], w[d] * hs[d]);
        u += std::max(w[d] * ls[d], w[d] * hs[d]);
      }
      for (int j = S; j < J; ++j) {
        l -= std::fabs(w[j]) * nb[j];
        u += std::fabs(w[j]) * nb[j];
      }
      lo = std::min(lo, l);
      hi = std::max(hi, u);
    }
    *lo_out = lo;
    *hi_out = hi;
    return FQ_OK;
  }
  st = cached_ritz(ctx, ctx->sys.hmod, mv, &lv, &hv);
  if (st != FQ_OK) return st;
  const double w0 = h0 - l0, wv = hv - lv;
  l0 -= margin * w0;
  h0 += margin * w0;
  lv -= margin * wv;
  hv += margin * wv;
  const double kap = 2.0 * std::max(std::fabs(l0), std::fabs(h0)) * std::max(std::fabs(lv), std::fabs(hv));
  double lo = std::numeric_limits<double>::infinity(), hi = -lo;
  if (ctx->scheme == FQ_MAGNUS6) {
    // ||B_j|| from ||[X, Y]|| <= 2 ||X|| ||Y|| along the nesting of the B_j
    const double n0 = std::max(std::fabs(l0), std::fabs(h0)), nv = std::max(std::fabs(lv), std::fabs(hv));
    double nb[kComm6];
    nb[0] = kap;
    nb[1] = 2.0 * n0 * nb[0];
    nb[2] = 2.0 * nv * nb[0];
    nb[3] = 2.0 * n0 * nb[1];
    nb[4] = 2.0 * n0 * nb[2];
    nb[5] = 2.0 * nv * nb[1];
    nb[6] = 2.0 * nv * nb[2];
    nb[7] = 2.0 * nb[0] * nb[1];
    nb[8] = 2.0 * nb[0] * nb[2];
    for (int k = 0; k < ctx->M; ++k) {
      const double a = ctx->a[k];
      double r = 0.0;
      for (int j = 0; j < kComm6; ++j) r += std::fabs(ctx->w6[(size_t)kComm6 * k + j]) * nb[j];
      lo = std::min(lo, l0 + std::min(a * lv, a * hv) - r);
      hi = std::max(hi, h0 + std::max(a * lv, a * hv) + r);
    }
    *lo_out = lo;
    *hi_out = hi;
    return FQ_OK;
  }
  for (int k = 0; k < ctx->M; ++k) {
    const double a = ctx->a[k], b = std::fabs(ctx->b[k]);
    lo = std::min(lo, l0 + std::min(a * lv, a * hv) - b * kap);
    hi = std::max(hi, h0 + std::max(a * lv, a * hv) + b * kap);
  }
  *lo_out = lo;
  *hi_out = hi;
  return FQ_OK;
}

// Inner bounds for checking a caller's interval: Ritz values of H_eff,k at the
// steps with the smallest and the largest a_k. Each Ritz value lies in the
// spectrum's hull of its step, so an interval that misses one cannot contain
// that step's spectrum.
fq_status dense_inner_bounds(fq_ctx* ctx, double* lo_out, double* hi_out) {
  int kmin = 0, kmax = 0;
  for (int k = 1; k < ctx->M; ++k) {
    // one drive term: a_k; several: the weight of the first drive matrix
    const double ak = ctx->S > 1 ? ctx->wS[(size_t)ctx->J * k] : ctx->a[k];
    const double amin = ctx->S > 1 ? ctx->wS[(size_t)ctx->J * kmin] : ctx->a[kmin];
    const double amax = ctx->S > 1 ? ctx->wS[(size_t)ctx->J * kmax] : ctx->a[kmax];
    if (ak < amin) kmin = k;
    if (ak > amax) kmax = k;
  }
  double lo = std::numeric_limits<double>::infinity(), hi = -lo;
  for (int k : {kmin, kmax}) {
    const double a = ctx->a[k], b = ctx->b[k];
    if (ctx->scheme == FQ_MAGNUS6 || ctx->S > 1) {  // H_eff,k formed on the device
      if (ctx->S > 1)
        FQ_TRY(drive_sum(ctx, k, true, ctx->htr, ctx->hti));  // (Ht planes are free)
      else
        FQ_TRY(magnus6_sum(ctx, k, true, ctx->htr, ctx->hti));
      Matvec mz = [&](const std::vector<cd>& x, std::vector<cd>& y) {
        return device_matvec_planar(ctx, ctx->htr, ctx->hti, x, y);
      };
      double l, h;
      FQ_TRY(lanczos_ritz(ctx, mz, &l, &h));
      lo = std::min(lo, l);
      hi = std::max(hi, h);
      if (kmin == kmax) break;
      continue;
    }
    Matvec mv = [&](const std::vector<cd>& x, std::vector<cd>& y) {
      // H0 x + a Hmod x + b K x with K x = -i (H0 (Hmod x) - Hmod (H0 x))
      std::vector<cd> u1, u2, u3, u4;
      fq_status st = ctx->h0_eigen ? device_matvec_planar(ctx, ctx->h0r, ctx->h0i, x, u1)
                                   : device_matvec(ctx, ctx->sys.h0, x, u1);
      if (st == FQ_OK) st = device_matvec(ctx, ctx->sys.hmod, x, u2);
      if (st == FQ_OK && b != 0.0)
        st = ctx->h0_eigen ? device_matvec_planar(ctx, ctx->h0r, ctx->h0i, u2, u3)
                           : device_matvec(ctx, ctx->sys.h0, u2, u3);
      if (st == FQ_OK && b != 0.0) st = device_matvec(ctx, ctx->sys.hmod, u1, u4);
      if (st != FQ_OK) return st;
      y.resize(x.size());
      for (size_t i = 0; i < x.size(); ++i) {
        y[i] = u1[i] + a * u2[i];
        if (b != 0.0) y[i] += b * cd(0.0, -1.0) * (u3[i] - u4[i]);
      }
      return FQ_OK;
    };
    double l, h;
    fq_status st = lanczos_ritz(ctx, mv, &l, &h);
    if (st != FQ_OK) return st;
    lo = std::min(lo, l);
    hi = std::max(hi, h);
    if (kmin == kmax) break;
  }
  *lo_out = lo;
  *hi_out = hi;
  return FQ_OK;
}

fq_status tridiag_cover(fq_ctx* ctx, double* lo_out, double* hi_out) {
  const long n = ctx->n;
  std::vector<double> d0(n), v(n), off(2 * std::max<long>(n - 1, 0));
  FQ_HIP(ctx, copy_sync(ctx->stream, d0.data(), ctx->sys.h0_diag, n * sizeof(double),
                        hipMemcpyDeviceToHost));
  FQ_HIP(ctx, copy_sync(ctx->stream, v.data(), ctx->sys.hmod_diag, n * sizeof(double),
                        hipMemcpyDeviceToHost));
  if (n > 1)
    FQ_HIP(ctx, copy_sync(ctx->stream, off.data(), ctx->sys.h0_off, 2 * (n - 1) * sizeof(double),
                          hipMemcpyDeviceToHost));
  std::vector<double> d(n), e(std::max<long>(n - 1, 1));
  double lo = std::numeric_limits<double>::infinity(), hi = -lo;
  for (int k = 0; k < ctx->M; ++k) {
    const double a = ctx->a[k], b = ctx->b[k];
    for (long i = 0; i < n; ++i) d[i] = d0[i] + a * v[i];
    for (long i = 0; i + 1 < n; ++i) {
      // |h (1 - i b dv)| = |h| sqrt(1 + (b dv)^2)
      const double hm = std::hypot(off[2 * i], off[2 * i + 1]);
      e[i] = hm * std::hypot(1.0, b * (v[i + 1] - v[i]));
    }
    double l, h;
    fq::tridiag_extremes(n, d.data(), e.data(), &l, &h);
    lo = std::min(lo, l);
    hi = std::max(hi, h);
  }
  *lo_out = lo;
  *hi_out = hi;
  // gauge factors of every step, for the kernel's real-symmetric form of Ht_s
  std::vector<double> wtab(2 * (size_t)n * ctx->M);
  for (int k = 0; k < ctx->M; ++k)
    fq::tridiag_gauge(n, off.data(), v.data(), ctx->b[k], wtab.data() + 2 * (size_t)n * k);
  FQ_HIP(ctx, copy_sync(ctx->stream, ctx->d_gauge, wtab.data(), wtab.size() * sizeof(double),
                        hipMemcpyHostToDevice));
  return FQ_OK;
}

// ---- profile-mode event marks ----------------------------------------------------------------

// Record the event that opens the next launch (kind >= 0) or closes the last (kind < 0).
fq_status mark(fq_ctx* c, int kind) {
  if (!c->profile) return FQ_OK;
  if (c->n_events == c->events.size()) {
    hipEvent_t e;
    FQ_HIP(c, hipEventCreate(&e));
    c->events.push_back(e);
    c->event_kind.push_back(-1);
  }
  FQ_HIP(c, hipEventRecord(c->events[c->n_events], c->stream));
  c->event_kind[c->n_events] = kind;
  ++c->n_events;
  return FQ_OK;
}

#define FQ_MARK(c, kind)               \
  do {                                 \
    fq_status s_ = mark((c), (kind));  \
    if (s_ != FQ_OK) return s_;        \
  } while (0)

// Sum the per-launch intervals into the report (after the stream has drained).
fq_status collect_profile(fq_ctx* c) {
  for (int i = 0; i < FQ_K_SLOTS; ++i) {
    c->last.ms_kernel[i] = 0.0;
    c->last.n_kernel[i] = 0;
  }
  if (!c->profile || c->n_events < 2) return FQ_OK;
  FQ_HIP(c, hipEventSynchronize(c->events[c->n_events - 1]));
  for (size_t i = 0; i + 1 < c->n_events; ++i) {
    const int k = c->event_kind[i];
    if (k < 0 || k >= FQ_K_SLOTS) continue;
    float ms = 0.f;
    FQ_HIP(c, hipEventElapsedTime(&ms, c->events[i], c->events[i + 1]));
    c->last.ms_kernel[k] += ms;
    c->last.n_kernel[k] += 1;
  }
  return FQ_OK;
}

// ---- dense step loop ----------------------------------------------------------------------------

fq_status dense_heff(fq_ctx* c, int k) {
  FQ_MARK(c, FQ_K_HEFF);
  if (c->scheme == FQ_MAGNUS6) FQ_TRY(magnus6_sum(c, k, false, c->kr, c->ki));  // K slot
  // H0 + a V + b K, or with several drive terms the whole sum, formed first in
  // the P planes (free at a step start) and passed as H0 with a = b = 0
  const double *h0r = c->h0r, *h0i = c->h0i;
  if (c->S > 1) {
    FQ_TRY(drive_sum(c, k, true, c->par, c->pai));
    h0r = c->par;
    h0i = c->pai;
  }
  if (c->precision == FQ_FP64) {
    FQ_HIP(c, fq::launch_heff_f64(h0r, h0i, c->vr, c->vi, c->kr, c->ki, c->a[k], c->b[k],
                                  c->beta, c->dE, c->n, c->np, c->htr, c->hti, c->stream));
  } else {
    FQ_HIP(c, fq::launch_heff_mixed(h0r, h0i, c->vr, c->vi, c->kr, c->ki, c->a[k],
                                    c->b[k], c->beta, c->dE, c->n, c->np, c->htr, c->hti, c->htx,
                                    c->precision, c->stream));
  }
  return FQ_OK;
}

// One FP64 Chebyshev product. a, p, o are the first planes of their buffers
// (real part first; the imaginary planes follow).
fq_status cheb_launch(fq_ctx* c, int kind, int mrows, double* a, double* p, double* o,
                      std::complex<double> c0, std::complex<double> cl) {
  const int np = (int)c->np;
  const long plane = c->np * c->np;
  static const int slot[4] = {FQ_K_FIRST, FQ_K_FIRST_LAST, FQ_K_MID, FQ_K_LAST};
  FQ_MARK(c, slot[kind]);
  ChebTerm t{};
  t.kind = kind;
  t.a_re = a; t.a_im = a + plane;
  t.b_re = c->htr; t.b_im = c->hti;
  t.p_re = p; t.p_im = p + plane;
  t.y_re = c->yr; t.y_im = c->yi;
  t.o_re = o; t.o_im = o + plane;
  t.c0r = c0.real(); t.c0i = c0.imag(); t.cr = cl.real(); t.ci = cl.imag();
  t.phr = c->phr; t.phi = c->phi;
  if (c->save_pl && (kind == fq::CHEB_LAST || kind == fq::CHEB_FIRST_LAST)) {
    t.save_re = c->save_pl;
    t.save_im = c->save_pl + plane;
  }
  FQ_HIP(c, fq::launch_cheb_f64(t, mrows, np, c->stream));
  return FQ_OK;
}

fq_status dense_cheb_step_mixed(fq_ctx* c, int mrows);

// One step on the state-major block held in the X planes: X <- E_k X.
// FP64 builds: X, Y, Pa and Pb hold FP64 planes (mixed builds: see
// dense_cheb_step_mixed).

fq_status dense_cheb_step(fq_ctx* c, int mrows) {
  if (c->precision != FQ_FP64) return dense_cheb_step_mixed(c, mrows);
  const int L = c->L;
  const size_t p2bytes = 2 * sizeof(double) * (size_t)c->np * (size_t)c->np;
  auto C = [&](int l) { return std::complex<double>(c->coef[2 * l], c->coef[2 * l + 1]); };
  if (c->save_plm1 && L == 1)  // P_{L-1} = P_0 = X
    FQ_HIP(c, hipMemcpyAsync(c->save_plm1, c->xr, p2bytes, hipMemcpyDeviceToDevice, c->stream));
  if (L == 1) {  // X_new = ph (c0 X + c1 Ht X), written to Y, then the roles swap
    FQ_TRY(cheb_launch(c, fq::CHEB_FIRST_LAST, mrows, c->xr, c->xr, c->yr, C(0), C(1)));
    std::swap(c->xr, c->yr);
    std::swap(c->xi, c->yi);
    return FQ_OK;
  }
  // l = 0: P1 -> Pa, Y = c0 X + c1 P1
  FQ_TRY(cheb_launch(c, fq::CHEB_FIRST, mrows, c->xr, c->xr, c->par, C(0), C(1)));
  double* prv = c->xr;  // P_{l-1}
  double* cur = c->par;  // P_l
  for (int l = 1; l <= L - 1; ++l) {
    const bool last = (l == L - 1);
    double* out;
    if (last) {
      out = c->xr;  // X is free once P_2 exists (or is P_0 itself, updated in place)
    } else if (l == 1) {
      out = c->pbr;  // keep X intact until P_2 is formed
    } else {
      out = prv;  // in place over P_{l-1}
    }
    if (last && c->save_plm1)
      FQ_HIP(c, hipMemcpyAsync(c->save_plm1, cur, p2bytes, hipMemcpyDeviceToDevice, c->stream));
    FQ_TRY(cheb_launch(c, last ? fq::CHEB_LAST : fq::CHEB_MID, mrows, cur, prv, out, C(0),
                       C(l + 1)));
    if (!last) {
      prv = cur;
      cur = out;
    }
  }
  return FQ_OK;
}

// ---- mixed-precision builds: one format per Chebyshev term -----------------------------------
//
// The rounding error of term l enters a step's sum weighted by |c_l| =
// 2 |J_l(R)| (Eq. (12)), which falls off fast once l exceeds R, so each term
// gets the cheapest format whose contribution stays within the error target.
// Relative error (RMS over a column, relative to its norm) of one product per
// format, u = 2^-24, nk blocks of 16 in the contraction. Leading terms from
// the rounding analysis, constants measured on MI355X (one product of dense
// orthonormal columns, and whole random-matrix builds at N = 1024 and 4096):
// FP64 ~ 0; three pieces with FP64 sums per block: the 24-bit operands plus a
// term that still grows as sqrt(nk); three pieces with FP32 running sums: the
// FP32 roundings of the running sums, growing as sqrt(nk); two and one pieces:
// their 16 and 8 significant bits; FP32 products (16x16x4 matrix cores): one
// rounding of the running sum per 4 columns. The FP64-sum constants are those
// fitted with 16-column partial sums, divided by 1.4: with the 64-column
// partials of the product kernel, whole builds of the random-matrix model
// measured 1.66x below the estimate at both N = 4096 (2.7e-7 against 4.5e-7)
// and N = 10^4 (4.0e-7 against 6.5e-7), so 1.4 keeps a 1.2x margin at both.
constexpr double kErrAcc0 = 0.5 / 1.4, kErrAccN = 0.2 / 1.4;
constexpr double kErrX30 = 1.0, kErrX3N = 0.55;
constexpr double kErrX2 = 0.15;
constexpr double kErrX1 = 0.6;
constexpr double kErrF320 = 1.0, kErrF32N = 0.25;
constexpr double kMixedTolDefault = 5e-7;  // half the 1e-6 bar of the mixed path

double term_error(int tf, long nk) {
  const double u = std::ldexp(1.0, -24), r = std::sqrt((double)nk);
  switch (tf) {
    case fq::TF_F64: return 0.0;
    case fq::TF_ACC: return (kErrAcc0 + kErrAccN * r) * u;
    case fq::TF_X3: return (kErrX30 + kErrX3N * r) * u;
    case fq::TF_X2: return kErrX2 * std::ldexp(1.0, -16);
    case fq::TF_F32: return (kErrF320 + kErrF32N * 2.0 * r) * u;
    default: return kErrX1 * std::ldexp(1.0, -8);
  }
}

// Formats of terms 1..L of a mixed build: the caller's, or the cheapest
// schedule found as follows. Random rounding errors of the terms add in
// quadrature over terms and steps, so the estimate for U_T is
// sqrt(sum_l (w_l eps_l)^2 M) with w_l the effective weight below. Each term takes the cheapest format whose own
// contribution |c_l| eps_l sqrt(M) is within a per-term allowance, starting at
// the whole target and shrinking until the total meets it; FP64 terms are then
// extended to a leading run (the step converts from FP64 planes to the low
// format once).
void choose_schedule(fq_ctx* c) {
  const int L = c->L;
  const bool f32 = c->precision == FQ_FP32;
  c->term_fmt.assign(L + 1, f32 ? fq::TF_F32 : fq::TF_X3);
  const long nk = c->np / 16;
  const double tol = c->mixed_tol > 0 ? c->mixed_tol : kMixedTolDefault;
  const double sm = std::sqrt((double)c->M);
  // An error in P_l also enters every later term through the recurrence, as a
  // Chebyshev polynomial of the second kind of degree l' - l (norm at most
  // l' - l + 1 on the spectrum), so term l's effective weight is
  // |c_l| + sum_{l' > l} (l' - l + 1) |c_l'| (its own weight when R is small,
  // several times it when R is large).
  std::vector<double> weff(L + 1, 0.0);
  for (int l = 1; l <= L; ++l)
    for (int q = l; q <= L; ++q) weff[l] += (q - l + 1) * std::fabs(c->weights[q]);
  auto contribution = [&](int l, int f) { return weff[l] * sm * term_error(f, nk); };
  auto total = [&]() {
    double e2 = 0.0;
    for (int l = 1; l <= L; ++l) {
      const double e = contribution(l, c->term_fmt[l]);
      e2 += e * e;
    }
    return std::sqrt(e2);
  };
  const int nf = (int)c->term_formats.size();
  if (nf > 0) {
    for (int l = 1; l <= L; ++l) c->term_fmt[l] = c->term_formats[std::min(l, nf) - 1];
  } else {
    double allowance = tol;
    for (int pass = 0; pass < 64; ++pass, allowance *= 0.7) {
      // FQ_FP32: FP32 products after a leading FP64 run of at least one term
      int last_f64 = f32 ? 1 : 0;
      for (int l = 1; l <= L; ++l) {
        int f = fq::TF_F64;
        if (f32) {
          if (contribution(l, fq::TF_F32) <= allowance) f = fq::TF_F32;
        } else {
          for (int cand : {fq::TF_X1, fq::TF_X2, fq::TF_X3, fq::TF_ACC})
            if (contribution(l, cand) <= allowance) {
              f = cand;
              break;
            }
        }
        c->term_fmt[l] = f;
        if (f == fq::TF_F64) last_f64 = l;
      }
      for (int l = 1; l <= std::min(last_f64, L); ++l) c->term_fmt[l] = fq::TF_F64;
      if (total() <= tol) break;
    }
  }
  c->mixed_err_est = total();
}

// One mixed-precision step on the state-major block in the X planes:
// X <- E_k X. FP64 terms (a leading run of h terms) rotate FP64 planes through
// Pa and Pb; the output of the last one goes to Pc and is rounded into the low
// format (BF16X3 or FP32) for the next product's A operand; low-format terms
// then run in place over P_{l-2} whenever it is in the low format too. The
// last term writes X.
fq_status dense_cheb_step_mixed(fq_ctx* c, int mrows) {
  const int L = c->L, np = (int)c->np;
  const long plane = c->np * c->np;
  auto C = [&](int l) { return std::complex<double>(c->coef[2 * l], c->coef[2 * l + 1]); };
  int h = 0;
  while (h < L && c->term_fmt[h + 1] == fq::TF_F64) ++h;
  struct Buf {
    double* p;
    bool f64;
  };
  auto kind_of = [&](int l) {  // position of term l (1-based) in the step
    if (l == 1) return L == 1 ? fq::CHEB_FIRST_LAST : fq::CHEB_FIRST;
    return l == L ? fq::CHEB_LAST : fq::CHEB_MID;
  };
  // term l from A = a (P_{l-1}; X for l = 1), prev = p (P_{l-2}; X for l <= 2)
  const bool f32 = c->precision == FQ_FP32;
  const int low = f32 ? fq::FMT_F32 : fq::FMT_BF16X3;  // storage of the non-FP64 terms
  auto term = [&](int l, Buf a, Buf p, Buf o) -> fq_status {
    const int kind = kind_of(l), tf = c->term_fmt[l];
    // split-BF16 builds time products by format, FP32 builds by position
    static const int slot[4] = {FQ_K_FIRST, FQ_K_FIRST_LAST, FQ_K_MID, FQ_K_LAST};
    FQ_MARK(c, f32 ? slot[kind] : FQ_K_TERM_FP64 + tf);
    if (tf == fq::TF_F64) {
      ChebTerm t{};
      t.kind = kind;
      t.a_re = a.p; t.a_im = a.p + plane;
      t.b_re = c->htr; t.b_im = c->hti;
      t.p_re = p.p; t.p_im = p.p + plane;
      t.y_re = c->yr; t.y_im = c->yi;
      t.o_re = o.p; t.o_im = o.p + plane;
      t.c0r = C(0).real(); t.c0i = C(0).imag(); t.cr = C(l).real(); t.ci = C(l).imag();
      t.phr = c->phr; t.phi = c->phi;
      FQ_HIP(c, fq::launch_cheb_f64(t, mrows, np, c->stream));
      return FQ_OK;
    }
    fq::ChebTermX t{};
    t.kind = kind;
    t.a_fmt = low;
    t.p_fmt = p.f64 ? fq::FMT_F64 : low;
    t.o_fmt = o.f64 ? fq::FMT_F64 : low;
    t.plane = plane;
    t.a = a.p; t.b = c->htx; t.p = p.p; t.o = o.p;
    t.y_re = c->yr; t.y_im = c->yi;
    t.c0r = C(0).real(); t.c0i = C(0).imag(); t.cr = C(l).real(); t.ci = C(l).imag();
    t.phr = c->phr; t.phi = c->phi;
    if (f32)
      FQ_HIP(c, fq::launch_cheb_mixed(t, FQ_FP32, mrows, np, c->stream));
    else
      FQ_HIP(c, fq::launch_cheb_bf16(t, tf, mrows, np, c->stream));
    return FQ_OK;
  };
  auto convert = [&](double* src, double* dst) -> fq_status {
    FQ_MARK(c, FQ_K_CONVERT);
    FQ_HIP(c, fq::launch_to_product(src, src + plane, dst, low, mrows, np, c->stream));
    return FQ_OK;
  };
  const Buf X{c->xr, true};
  Buf A{c->par, true}, B{c->pbr, true}, S{c->pcr, true};
  if (h == L) {  // every term in FP64: the FP64 rotation through A and B
    if (L == 1) {  // X_new = ph (c0 X + c1 Ht X) to Y (A = X is read by every tile), then swap
      FQ_TRY(term(1, X, X, Buf{c->yr, true}));
      std::swap(c->xr, c->yr);
      std::swap(c->xi, c->yi);
      return FQ_OK;
    }
    FQ_TRY(term(1, X, X, A));
    Buf prv = X, cur = A;
    for (int l = 2; l <= L; ++l) {
      const Buf out = l == L ? X : (l == 2 ? B : prv);
      FQ_TRY(term(l, cur, prv, out));
      prv = cur;
      cur = out;
    }
    return FQ_OK;
  }
  Buf prv, cur;  // P_{l-2}, P_{l-1} before term l
  int l0;        // first BF16 term
  if (h == 0) {
    // X's BF16 copy for the first product's A operand, in B (free until term 2)
    FQ_TRY(convert(c->xr, B.p));
    const Buf xb{B.p, false};
    if (L == 1) return term(1, xb, X, X);
    A.f64 = false;
    FQ_TRY(term(1, xb, X, A));
    prv = X;
    cur = A;
    B.f64 = false;
    l0 = 2;
  } else {
    // FP64 terms 1..h; term h writes S, rounded into the buffer term h read as
    // P_{h-2} (B for h = 1 and h = 2), which is free from then on
    Buf p2 = X, p1 = X;  // P_{l-2}, P_{l-1}
    for (int l = 1; l <= h; ++l) {
      Buf out = l == h ? S : (l == 1 ? A : (l == 2 ? B : p2));
      FQ_TRY(term(l, p1, p2, out));
      p2 = p1;
      p1 = out;
    }
    // p1 = S holds P_h (FP64); p2 holds P_{h-1} (FP64)
    Buf dst = (h <= 2) ? B : (p2.p == A.p ? B : A);
    FQ_TRY(convert(S.p, dst.p));
    dst.f64 = false;
    prv = p2;   // P_{h-1}, FP64 (X when h = 1)
    cur = dst;  // P_h, BF16
    S.f64 = false;
    l0 = h + 1;
    // the FP64 buffers that no longer hold a live term become BF16 scratch
    if (dst.p == B.p) B = dst; else A = dst;
  }
  for (int l = l0; l <= L; ++l) {
    Buf out;
    if (l == L) {
      out = X;
    } else if (!prv.f64) {
      out = prv;  // in place over P_{l-2}
    } else {
      // P_{l-2} is FP64 (X, or the last FP64 term): a BF16 buffer that is neither operand
      Buf cands[3] = {Buf{A.p, false}, Buf{B.p, false}, Buf{S.p, false}};
      out = cands[0];
      for (const Buf& q : cands)
        if (q.p != cur.p && q.p != prv.p) {
          out = q;
          break;
        }
    }
    FQ_TRY(term(l, cur, prv, out));
    prv = cur;
    cur = out;
  }
  return FQ_OK;
}

// The one-launch chain of small_chain_kernel serves FP64 steps of one drive
// term whose Ht is H0 + a_k V + b_k K (Magnus-4, commutator-free) at np = 64,
// without tape, snapshots or saved terms. FQ_SMALL_CHAIN=0 in the environment
// (read at fq_create) keeps the launch-per-product form instead.
bool small_chain_ok(const fq_ctx* c, bool record_tape) {
  return c->small_chain && c->precision == FQ_FP64 && c->np == fq::small_chain_max_n() &&
         c->scheme != FQ_MAGNUS6 && c->S == 1 && !record_tape && !c->snap && !c->save_pl &&
         !c->save_plm1;
}

fq_status dense_steps(fq_ctx* c, int k0, int k1, int mrows, bool record_tape) {
  const size_t plane2 = 2 * (size_t)c->np * (size_t)c->np;
  if (small_chain_ok(c, record_tape)) {
    fq::SmallChain sc{};
    sc.h0r = c->h0r; sc.h0i = c->h0i;
    sc.vr = c->vr; sc.vi = c->vi;
    sc.kr = c->kr; sc.ki = c->ki;
    sc.ab = c->d_ab;
    sc.coef = c->d_coef;
    sc.xr = c->xr; sc.xi = c->xi;
    sc.ld = c->np;
    sc.n = (int)c->n;
    sc.L = c->L;
    sc.k0 = k0;
    sc.k1 = k1;
    sc.beta = c->beta;
    sc.inv_dE = 1.0 / c->dE;
    sc.phr = c->phr;
    sc.phi = c->phi;
    FQ_MARK(c, FQ_K_CHAIN);
    FQ_HIP(c, fq::launch_small_chain(sc, mrows, c->stream));
    return FQ_OK;
  }
  if (record_tape && k0 == 0)
    FQ_HIP(c, hipMemcpyAsync(c->tape, c->xr, plane2 / 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (record_tape && k0 == 0)
    FQ_HIP(c, hipMemcpyAsync(c->tape + plane2 / 2, c->xi, plane2 / 2 * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
  for (int k = k0; k < k1; ++k) {
    fq_status st = dense_heff(c, k);
    if (st != FQ_OK) return st;
    st = dense_cheb_step(c, mrows);
    if (st != FQ_OK) return st;
    if (c->snap && (k + 1 - c->snap_k0) % c->snap_every == 0) {  // X_{k+1} to the user's buffer
      const long j = (k + 1 - c->snap_k0) / c->snap_every - 1;
      char* dst = static_cast<char*>(c->snap) +
                  (size_t)j * (c->c64 ? 8 : 16) * (size_t)c->n * (size_t)c->snap_ncols;
      FQ_HIP(c, fq::launch_unpack_planar_t(c->xr, c->xi, c->np, c->n, c->snap_ncols, dst,
                                           c->snap_ncols, c->c64, c->stream));
    }
    if (record_tape && ((k + 1) % c->ckpt == 0 || k + 1 == c->M)) {
      const int slot = (k + 1 + c->ckpt - 1) / c->ckpt;
      double* dst = c->tape + (size_t)slot * plane2;
      FQ_HIP(c, hipMemcpyAsync(dst, c->xr, plane2 / 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      FQ_HIP(c, hipMemcpyAsync(dst + plane2 / 2, c->xi, plane2 / 2 * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream));
    }
  }
  return FQ_OK;
}

fq_status unitarity(fq_ctx* c, const double* xr, const double* xi) {
  FQ_HIP(c, zero_async(c->stream, c->small, 2 * sizeof(double)));
  FQ_HIP(c, fq::launch_unitarity_f64(xr, xi, (int)c->n, (int)c->np, c->small, c->stream));
  double h[2];
  FQ_HIP(c, hipMemcpyAsync(h, c->small, sizeof h, hipMemcpyDeviceToHost, c->stream));
  FQ_HIP(c, hipStreamSynchronize(c->stream));
  c->last.unitarity_max = h[0];
  c->last.unitarity_fro = std::sqrt(h[1]);
  c->last.diverged = !(h[0] <= kDivergence);  // also NaN
  return FQ_OK;
}

// Polar factor of U_T by Newton-Schulz steps X <- X (3 - X^dagger X) / 2, in
// the state-major planes A = U^T: A <- 1.5 A - 0.5 (A A^dagger) A, where
// (A A^dagger) A is the NT product of A A^dagger with the transpose of A.
// Quadratic convergence from ||U^dagger U - 1|| < 1; two steps take the
// build's residual (1e-8 for BF16x3, 1e-12 for FP64) to round-off.
fq_status reorthonormalize(fq_ctx* c) {
  const int np = (int)c->np;
  const size_t p2bytes = 2 * sizeof(double) * (size_t)c->np * (size_t)c->np;
  for (int it = 0; it < 2; ++it) {
    FQ_HIP(c, fq::launch_zgemm_nt_f64(c->xr, c->xi, false, c->xr, c->xi, true, c->par, c->pai, np,
                                      np, np, np, 1.0, 0.0, 0.0, 0.0, c->stream));
    FQ_HIP(c, fq::launch_transpose_planar(c->xr, c->xi, c->pbr, c->pbi, c->np, c->stream));
    FQ_HIP(c, hipMemcpyAsync(c->yr, c->xr, p2bytes, hipMemcpyDeviceToDevice, c->stream));
    FQ_HIP(c, fq::launch_zgemm_nt_f64(c->par, c->pai, false, c->pbr, c->pbi, false, c->yr, c->yi,
                                      np, np, np, np, -0.5, 0.0, 1.5, 0.0, c->stream));
    std::swap(c->xr, c->yr);
    std::swap(c->xi, c->yi);
  }
  return FQ_OK;
}

// Re-orthonormalise the planar U_T, write it to U_out and measure it again;
// the build's own unitarity stays in unitarity_max / unitarity_fro.
fq_status finish_reortho(fq_ctx* c, void* U_out) {
  const double umax = c->last.unitarity_max, ufro = c->last.unitarity_fro;
  FQ_TRY(reorthonormalize(c));
  FQ_HIP(c, fq::launch_unpack_planar_t(c->xr, c->xi, c->np, c->n, c->n, U_out, c->n, c->c64,
                                       c->stream));
  FQ_TRY(unitarity(c, c->xr, c->xi));
  c->last.unitarity_max_after = c->last.unitarity_max;
  c->last.unitarity_fro_after = c->last.unitarity_fro;
  c->last.unitarity_max = umax;
  c->last.unitarity_fro = ufro;
  return FQ_OK;
}

void fill_report(fq_ctx* c) {
  for (int l = 0; l < FQ_TERM_SLOTS; ++l)
    c->last.term_format[l] =
        l < c->L && !c->term_fmt.empty() ? c->term_fmt[l + 1] : -1;
  c->last.mixed_err_est = c->mixed_err_est;
  c->last.L = c->L;
  c->last.M = c->M_user;
  c->last.R = c->R;
  c->last.dE = c->dE;
  c->last.beta = c->beta;
  c->last.e_min = c->e_min;
  c->last.e_max = c->e_max;
}

fq_status tridiag_run(fq_ctx* c, const void* x0, long ncols, int k0, int k1, void* x_out) {
  fq::TridiagJob job{};
  job.n = c->n;
  job.ncols = ncols;
  job.h0_diag = c->sys.h0_diag;
  job.h0_off = reinterpret_cast<const double*>(c->sys.h0_off);
  job.v_diag = c->sys.hmod_diag;
  job.ab = c->d_ab;
  job.coef = c->d_coef;
  job.gauge = c->d_gauge;
  job.L = c->L;
  job.k0 = k0;
  job.k1 = k1;
  job.beta = c->beta;
  job.inv_dE = 1.0 / c->dE;
  job.phr = c->phr;
  job.phi = c->phi;
  job.x0 = x0;
  job.ld_x0 = ncols;
  job.x_out = x_out;
  job.ld_out = ncols;
  job.c64 = c->c64 ? 1 : 0;
  if (c->snap) {
    job.snap = static_cast<double*>(c->snap);
    job.snap_every = c->snap_every;
  }
  // a build (identity, all steps) with a gradient tape records X_{j ckpt}
  if (c->tape && x0 == nullptr && k0 == 0 && k1 == c->M && ncols == c->n) {
    job.tape = c->tape;
    job.ckpt = c->ckpt;
  }
  if (c->n <= fq::tridiag_resident_max_n()) {
    FQ_MARK(c, FQ_K_TRIDIAG);
    FQ_HIP(c, fq::launch_tridiag_resident(job, c->stream));
    return FQ_OK;
  }
  // Longer columns: k-term passes with ghost rows, state ping-ponged through HBM.
  const int K = 128, G = 1;  // 768 owned rows per workgroup
  if (x0 && x0 == x_out && k1 - k0 == 1 && c->L + 1 <= K) {
    // One pass both reads X0 (with ghost rows) and writes X_out (owned rows):
    // in place, a workgroup could overwrite rows its neighbour still reads.
    // The state planes are unused by a single pass; stage X0 there.
    const size_t bytes = (size_t)c->n * (size_t)ncols * (c->c64 ? 8 : 16);
    FQ_HIP(c, hipMemcpyAsync(c->d_stream, x0, bytes, hipMemcpyDeviceToDevice, c->stream));
    job.x0 = c->d_stream;
  }
  fq::TridiagStream st{};
  st.G = G;
  st.n16 = (c->n + 15) / 16 * 16;
  st.plane = st.n16 * ncols;
  st.K = K;
  st.B = fq::tridiag_stream_rows(G) - 2L * K;
  st.nblk = (c->n + st.B - 1) / st.B;
  const size_t state = 8 * (size_t)st.n16 * (size_t)c->n;
  double* buf[2] = {c->d_stream, c->d_stream + state};
  double* stepc = c->d_stream + 2 * state;
  st.stepc = stepc;
  int cur = 0;
  for (int s = k0; s < k1; ++s) {
    st.s = s;
    st.last_step = (s + 1 == k1);
    FQ_MARK(c, FQ_K_HEFF);  // rows of 2 Ht_s and the gauge factors of the step
    FQ_HIP(c, fq::launch_tridiag_stream_step(job, st, stepc, c->stream));
    for (int l0 = 0; l0 <= c->L; l0 += K) {
      st.l0 = l0;
      st.l1 = std::min(l0 + K, c->L + 1);
      st.first_step = (s == k0 && l0 == 0);
      st.in = buf[cur];
      st.out = buf[cur ^ 1];
      FQ_MARK(c, FQ_K_TRIDIAG);
      FQ_HIP(c, fq::launch_tridiag_stream(job, st, c->stream));
      cur ^= 1;
    }
  }
  return FQ_OK;
}

// ---- adjoint ---------------------------------------------------------------------------------
//
// One step maps X to X' = phi sum_l c_l P_l with P_0 = X, P_1 = Ht X,
// P_{l+1} = 2 Ht P_l - P_{l-1}, phi = exp(-i beta h). For a real loss with
// Lambda = dL/dRe X' + i dL/dIm X', the chain rule gives (Ht Hermitian):
//   Pbar_L = d_L Lambda,  Pbar_{L-1} = 2 Ht Pbar_L + d_{L-1} Lambda,
//   Pbar_l = 2 Ht Pbar_{l+1} - Pbar_{l+2} + d_l Lambda   (1 <= l <= L-2),
//   Pbar_0 = Ht Pbar_1 - Pbar_2 + d_0 Lambda = dL/dRe X + i dL/dIm X,
// with d_l = conj(phi c_l), and
//   dL/da_k = Re sum_l w_l <Pbar_{l+1}, Hmod P_l> / dE,  w_0 = 1, w_l = 2,
// likewise dL/db_k with K. The P_l are regenerated backwards from P_{L-1},
// P_L by P_{l-1} = 2 Ht P_l - P_{l+1}, in the same product as the Pbar_l
// (stacked operand [P_l; Pbar_{l+1}]). X_{k-1}, P_{L-1}, P_L of each step come
// from recomputing its segment forward from the tape.

fq_status adjoint_step(fq_ctx* c, int k, int slot, bool with_k) {
  const int L = c->L;
  const int np = (int)c->np;
  const long plane = c->np * c->np;
  const size_t pbytes = sizeof(double) * (size_t)plane;
  hipStream_t s = c->stream;
  double* seg_x = c->seg + (size_t)slot * 6 * plane;
  double* seg_lm1 = seg_x + 2 * plane;
  double* seg_l = seg_x + 4 * plane;
  auto D = [&](int l) {  // conj(phi c_l)
    const std::complex<double> ph(c->phr, c->phi), cl(c->coef[2 * l], c->coef[2 * l + 1]);
    return std::conj(ph * cl);
  };
  // stack views: re plane (2np x np) then im plane; top = P, bottom = Pbar
  auto top_re = [&](int i) { return c->stack[i]; };
  auto top_im = [&](int i) { return c->stack[i] + 2 * plane; };
  auto bot_re = [&](int i) { return c->stack[i] + plane; };
  auto bot_im = [&](int i) { return c->stack[i] + 3 * plane; };
  double* lr = c->lam;
  double* li = c->lam + plane;
  double* gk = c->d_grad + (size_t)c->J * k;
  // contractions with the drive block: [Hmod; K] (K skipped when only the
  // node-pair sums are asked for), or all J matrices for several drive terms
  const int dot_cols = c->S > 1 ? c->J * np : (with_k ? 2 * np : np);
  auto copy2 = [&](double* dre, double* dim, const double* src) -> fq_status {
    FQ_HIP(c, hipMemcpyAsync(dre, src, pbytes, hipMemcpyDeviceToDevice, s));
    FQ_HIP(c, hipMemcpyAsync(dim, src + plane, pbytes, hipMemcpyDeviceToDevice, s));
    return FQ_OK;
  };
  // FQ_FP32 contexts run the reverse products on FP32 matrix cores (operands
  // rounded while staged; FP64 epilogues and contraction sums)
  const bool f32 = c->adj_f32;
  const float* ht32 = static_cast<const float*>(c->htx);
  auto dot = [&](int i, double w) -> fq_status {
    if (f32)
      FQ_HIP(c, fq::launch_adj_dot_f32(top_re(i), 2 * plane, c->drive32, (long)c->J * plane,
                                       dot_cols, bot_re(i), bot_im(i), w, gk, np, s));
    else
      FQ_HIP(c, fq::launch_adj_dot(top_re(i), top_im(i), c->vr, c->vi, dot_cols, bot_re(i),
                                   bot_im(i), w, gk, np, s));
    return FQ_OK;
  };
  // A = [P_l; Pbar_{l+1}] rows from a_re (imaginary plane two planes on), Ht
  auto rev = [&](double* a_re, double* a_im, int mrows, int o, std::complex<double> dl, double fac,
                 int row_off) -> fq_status {
    FQ_MARK(c, FQ_K_ADJ_REV);
    if (f32)
      FQ_HIP(c, fq::launch_adj_step_f32(a_re, mrows, 2 * plane, ht32, top_re(o), top_im(o), lr, li,
                                        dl.real(), dl.imag(), fac, row_off, np, s));
    else
      FQ_HIP(c, fq::launch_adj_step(a_re, a_im, mrows, c->htr, c->hti, top_re(o), top_im(o), lr,
                                    li, dl.real(), dl.imag(), fac, row_off, np, s));
    FQ_MARK(c, -1);
    return FQ_OK;
  };
  // Pbar_L = d_L Lambda over P_{L-1} in stack 0; P_L over zero in stack 1
  std::complex<double> d = D(L);
  FQ_TRY(copy2(top_re(0), top_im(0), seg_lm1));
  FQ_HIP(c, fq::launch_scale_planar(lr, li, d.real(), d.imag(), bot_re(0), bot_im(0), plane, s));
  FQ_TRY(copy2(top_re(1), top_im(1), seg_l));
  FQ_HIP(c, zero_async(s, bot_re(1), pbytes));
  FQ_HIP(c, zero_async(s, bot_im(1), pbytes));
  int cur = 0;
  for (int l = L - 1; l >= 1; --l) {
    const int o = 1 - cur;
    FQ_TRY(dot(cur, 2.0));  // <Pbar_{l+1}, D P_l>
    d = D(l);
    if (l >= 2) {
      FQ_TRY(rev(top_re(cur), top_im(cur), 2 * np, o, d, 2.0, 0));
    } else {  // l = 1: Pbar_1 only; P_0 = X_{k-1} from the segment store
      FQ_TRY(rev(bot_re(cur), bot_im(cur), np, o, d, 2.0, np));
      FQ_TRY(copy2(top_re(o), top_im(o), seg_x));
    }
    cur = o;
  }
  if (L == 1) {  // stack 0 = [P_0; Pbar_1]
    FQ_TRY(copy2(top_re(0), top_im(0), seg_x));
    cur = 0;
  }
  // l = 0: <Pbar_1, D P_0>, then Pbar_0 = Ht Pbar_1 - Pbar_2 + d_0 Lambda
  const int o = 1 - cur;
  FQ_TRY(dot(cur, 1.0));
  d = D(0);
  FQ_TRY(rev(bot_re(cur), bot_im(cur), np, o, d, 1.0, np));
  FQ_HIP(c, hipMemcpyAsync(lr, bot_re(o), pbytes, hipMemcpyDeviceToDevice, s));
  FQ_HIP(c, hipMemcpyAsync(li, bot_im(o), pbytes, hipMemcpyDeviceToDevice, s));
  return FQ_OK;
}

// Chain rule from dL/da, dL/db per (sub)step (g, contractions with the
// unscaled Hmod and K, hence the 1/dE) to the drive samples.
void grad_to_nodes(const fq_ctx* c, const std::vector<double>& g, double* grad_f_nodes) {
  if (c->S > 1) {  // g holds J values per (sub)step; output [step][node][term]
    const int S = c->S, J = c->J;
    const double w = std::sqrt(3.0) * c->h / 12.0;
    for (int k = 0; k < c->M_user; ++k) {
      double* o1 = grad_f_nodes + (size_t)(2 * k) * S;
      double* o2 = grad_f_nodes + (size_t)(2 * k + 1) * S;
      if (c->scheme == FQ_CF4) {
        const double* g1 = &g[(size_t)J * (2 * k)];
        const double* g2 = &g[(size_t)J * (2 * k + 1)];
        for (int d = 0; d < S; ++d) {
          o1[d] = (kCf4P * g1[d] + kCf4Q * g2[d]) / c->dE;
          o2[d] = (kCf4Q * g1[d] + kCf4P * g2[d]) / c->dE;
        }
        continue;
      }
      const double* gk = &g[(size_t)J * k];
      const double* f1 = &c->f_nodes[(size_t)(2 * k) * S];
      const double* f2 = &c->f_nodes[(size_t)(2 * k + 1) * S];
      for (int d = 0; d < S; ++d) {
        o1[d] = (0.5 * gk[d] + w * gk[S + d]) / c->dE;
        o2[d] = (0.5 * gk[d] - w * gk[S + d]) / c->dE;
      }
      int q = 2 * S;  // weight w (f_d2 f_e1 - f_e2 f_d1) of K_de
      for (int d = 0; d < S; ++d)
        for (int e = d + 1; e < S; ++e, ++q) {
          const double gq = w * gk[q] / c->dE;
          o1[d] -= gq * f2[e];
          o2[d] += gq * f1[e];
          o1[e] += gq * f2[d];
          o2[e] -= gq * f1[d];
        }
    }
    return;
  }
  if (c->scheme == FQ_CF4) {  // a of the half-steps: (P f1 + Q f2, Q f1 + P f2)
    for (int k = 0; k < c->M_user; ++k) {
      const double g1 = g[4 * k] / c->dE, g2 = g[4 * k + 2] / c->dE;
      grad_f_nodes[2 * k] = kCf4P * g1 + kCf4Q * g2;
      grad_f_nodes[2 * k + 1] = kCf4Q * g1 + kCf4P * g2;
    }
    return;
  }
  const double w = std::sqrt(3.0) * c->h / 12.0;  // b = sqrt(3) h (f1 - f2) / 12
  for (int k = 0; k < c->M; ++k) {
    const double ga = g[2 * k] / c->dE, gb = g[2 * k + 1] / c->dE;
    grad_f_nodes[2 * k] = 0.5 * ga + w * gb;
    grad_f_nodes[2 * k + 1] = 0.5 * ga - w * gb;
  }
}

fq_status adjoint(fq_ctx* c, const void* U_bar, double* grad_f_nodes) {
  const int M = c->M, s = c->ckpt;
  const long plane = c->np * c->np;
  const size_t p2bytes = 2 * sizeof(double) * (size_t)plane;
  FQ_HIP(c, fq::launch_pack_planar_t(U_bar, c->n, c->n, c->n, c->lam, c->lam + plane, c->np,
                                     c->np, c->c64, c->stream));
  FQ_HIP(c, zero_async(c->stream, c->d_grad, (size_t)c->J * sizeof(double) * (size_t)M));
  // dL/db_k is needed for the node derivatives even where b_k = 0; it cancels
  // in the node-pair sums
  const bool with_k = !c->pair_sums;
  const int nseg = (M + s - 1) / s;
  c->n_events = 0;  // profile mode: the recompute and reverse products go to the report
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int k0 = sg * s, k1 = std::min(M, k0 + s);
    // regenerate the segment forward in FP64 from its checkpoint
    FQ_MARK(c, -1);
    FQ_HIP(c, hipMemcpyAsync(c->xr, c->tape + (size_t)sg * 2 * plane, p2bytes,
                             hipMemcpyDeviceToDevice, c->stream));
    for (int k = k0; k < k1; ++k) {
      double* slot = c->seg + (size_t)(k - k0) * 6 * plane;
      FQ_HIP(c, hipMemcpyAsync(slot, c->xr, p2bytes, hipMemcpyDeviceToDevice, c->stream));
      c->save_plm1 = slot + 2 * plane;
      c->save_pl = slot + 4 * plane;
      FQ_TRY(dense_heff(c, k));
      FQ_TRY(dense_cheb_step(c, (int)c->np));
      c->save_pl = c->save_plm1 = nullptr;
    }
    for (int k = k1 - 1; k >= k0; --k) {
      if (c->adj_f32) {  // Ht also in the FP32 product format for the reverse products
        c->precision = FQ_FP32;
        const fq_status hs = dense_heff(c, k);
        c->precision = FQ_FP64;
        FQ_TRY(hs);
      } else {
        FQ_TRY(dense_heff(c, k));
      }
      FQ_TRY(adjoint_step(c, k, k - k0, with_k));
    }
  }
  FQ_MARK(c, -1);
  std::vector<double> g((size_t)c->J * M);
  FQ_HIP(c, hipMemcpyAsync(g.data(), c->d_grad, g.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  FQ_HIP(c, hipStreamSynchronize(c->stream));
  grad_to_nodes(c, g, grad_f_nodes);
  return collect_profile(c);
}

// The reverse sweep in streamed passes (columns longer than one workgroup
// holds, or on request): per checkpoint segment, last first, the steps are
// recomputed by the forward passes from the segment's checkpoint, which leave
// the gauge-frame P_{L-1}, P_L of every step in the segment buffer; then each
// step is reversed in passes of at most K terms (P_0 regenerated with the
// other terms), Lambda passing from step to step as Pbar_0 in the gauge frame
// of the step it came from.
fq_status tridiag_adjoint_streamed(fq_ctx* c, const void* U_bar, double* grad_f_nodes) {
  const int M = c->M, L = c->L, ckpt = c->ckpt;
  const long n = c->n;
  const bool with_k = !c->pair_sums;
  // one pass length for the recompute and the reverse passes, chosen for the
  // reverse passes (two thirds of the sweep)
  const int K = stream_pass_terms(n, L, kStreamOverheadRev, with_k ? 128 : 256);
  const long n16 = (n + 15) / 16 * 16;
  const size_t plane = (size_t)n16 * (size_t)n;  // doubles per state plane

  // forward passes of the recompute: the build's job and pass geometry
  fq::TridiagJob job{};
  job.n = n;
  job.ncols = n;
  job.h0_diag = c->sys.h0_diag;
  job.h0_off = reinterpret_cast<const double*>(c->sys.h0_off);
  job.v_diag = c->sys.hmod_diag;
  job.ab = c->d_ab;
  job.coef = c->d_coef;
  job.gauge = c->d_gauge;
  job.L = L;
  job.beta = c->beta;
  job.inv_dE = 1.0 / c->dE;
  job.phr = c->phr;
  job.phi = c->phi;
  job.ld_x0 = n;
  job.c64 = c->c64 ? 1 : 0;
  fq::TridiagStream st{};
  st.G = 1;
  st.n16 = n16;
  st.plane = (long)plane;
  st.K = K;
  st.B = fq::tridiag_stream_rows(1) - 2L * K;
  st.nblk = (n + st.B - 1) / st.B;
  double* fbuf[2] = {c->d_stream, c->d_stream + 8 * plane};
  double* stepc = c->d_stream + 16 * plane;
  st.stepc = stepc;

  fq::TridiagAdjStream p{};
  p.n = n;
  p.ncols = n;
  p.n16 = n16;
  p.plane = (long)plane;
  p.K = K;
  p.B = st.B;
  p.nblk = st.nblk;
  p.L = L;
  p.coef = c->d_coef;
  p.phr = c->phr;
  p.phi = c->phi;
  p.h0_diag = c->sys.h0_diag;
  p.h0_off = reinterpret_cast<const double*>(c->sys.h0_off);
  p.v_diag = c->sys.hmod_diag;
  p.gauge = c->d_gauge;
  p.beta = c->beta;
  p.inv_dE = 1.0 / c->dE;
  double* rset[2] = {c->d_adj, c->d_adj + 8 * plane};
  double* lam[2] = {c->d_adj + 16 * plane, c->d_adj + 18 * plane};
  double* tab = c->d_adj + 20 * plane;
  auto seg = [&](int j) { return c->seg + (size_t)j * 4 * plane; };
  // tape entry j: X_{j ckpt}; column-major complex128 from the per-column
  // build, or (n > tridiag_resident_max_n()) the snapshot store of the streamed
  // build, row-major in the state type from entry 1 on (entry 0: identity)
  const bool tape_rows = n > fq::tridiag_resident_max_n();
  auto tape_entry = [&](int j) -> const void* {
    if (!tape_rows) return c->tape + (size_t)j * 2 * (size_t)n * (size_t)n;
    if (j == 0) return nullptr;
    const size_t esz = c->c64 ? 8 : 16;
    return reinterpret_cast<const char*>(c->tape) + 16 * (size_t)n * (size_t)n +
           (size_t)(j - 1) * (size_t)n * (size_t)n * esz;
  };

  FQ_HIP(c, zero_async(c->stream, c->d_grad, 2 * sizeof(double) * fq::kAdjSlots * (size_t)M));
  FQ_HIP(c, fq::launch_tridiag_lam_pack(U_bar, c->c64, n, n, n16, lam[0], c->stream));
  c->n_events = 0;  // profile mode: the passes' times go to the report
  int lam_cur = 0;
  const int nseg = (M + ckpt - 1) / ckpt;
  // FQ_PROGRESS=1: a line on stderr after each segment (long sweeps)
  const char* prog = std::getenv("FQ_PROGRESS");
  const bool progress = prog && prog[0] == '1';
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int k0 = sg * ckpt, k1 = std::min(k0 + ckpt, M);
    job.x0 = tape_entry(sg);
    job.x0_colmajor = tape_rows ? 0 : 1;
    int cur = 0;
    for (int k = k0; k < k1; ++k) {  // forward recompute, keeping P_{L-1}, P_L
      st.s = k;
      st.last_step = (k + 1 == M);  // the step rows: no gauge of a step M
      FQ_MARK(c, FQ_K_HEFF);
      FQ_HIP(c, fq::launch_tridiag_stream_step(job, st, stepc, c->stream));
      st.last_step = 0;  // X~_{k+1} stays in the pass state (unused after step M - 1)
      for (int l0 = 0; l0 <= L; l0 += K) {
        st.l0 = l0;
        st.l1 = std::min(l0 + K, L + 1);
        st.first_step = (k == k0 && l0 == 0);
        st.in = fbuf[cur];
        st.out = fbuf[cur ^ 1];
        st.save = st.l1 > L ? seg(k - k0) : nullptr;
        FQ_MARK(c, FQ_K_ADJ_FWD);
        FQ_HIP(c, fq::launch_tridiag_stream(job, st, c->stream));
        cur ^= 1;
      }
    }
    st.save = nullptr;
    for (int k = k1 - 1; k >= k0; --k) {  // reverse
      p.a = c->a[k];
      p.b = c->b[k];
      FQ_MARK(c, FQ_K_HEFF);
      FQ_HIP(c, fq::launch_tridiag_adj_table(p, k, k == M - 1, tab, c->stream));
      p.lam = lam[lam_cur];
      p.lam_out = lam[lam_cur ^ 1];
      // without the K contraction the passes read Lambda' = f Lambda (f of
      // the step's table), formed once here in place
      if (!with_k) FQ_HIP(c, fq::launch_tridiag_lam_gauge(p, tab, lam[lam_cur], c->stream));
      p.seg = seg(k - k0);
      p.grad = c->d_grad + 2 * (size_t)fq::kAdjSlots * (size_t)k;
      int rc = 0;
      for (int hi = L - 1; hi >= 0; hi -= K) {
        p.hi = hi;
        p.lo = std::max(hi - K + 1, 0);
        p.in = rset[rc];
        p.out = rset[rc ^ 1];
        FQ_MARK(c, FQ_K_ADJ_REV);
        FQ_HIP(c, with_k ? fq::launch_tridiag_adj_stream(p, tab, true, c->stream)
                         : fq::launch_tridiag_adj_persist(p, tab, c->stream));
        rc ^= 1;
      }
      lam_cur ^= 1;
    }
    if (progress) {
      FQ_HIP(c, hipStreamSynchronize(c->stream));
      std::fprintf(stderr, "floquet_grad: segment %d of %d reversed (steps %d..%d)\n",
                   nseg - sg, nseg, k0, k1 - 1);
      std::fflush(stderr);
    }
  }
  FQ_MARK(c, -1);
  std::vector<double> slots(2 * (size_t)fq::kAdjSlots * (size_t)M);
  FQ_HIP(c, hipMemcpyAsync(slots.data(), c->d_grad, slots.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  FQ_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<double> g(2 * (size_t)M, 0.0);
  for (int k = 0; k < M; ++k)
    for (int j = 0; j < fq::kAdjSlots; ++j) {
      g[2 * k] += slots[(size_t)(k * fq::kAdjSlots + j) * 2];
      g[2 * k + 1] += slots[(size_t)(k * fq::kAdjSlots + j) * 2 + 1];
    }
  grad_to_nodes(c, g, grad_f_nodes);
  return collect_profile(c);
}

// Gradient of the tridiagonal chain: one reverse-sweep launch over all columns
// (each workgroup recomputes its column's segments from the tape), then the
// chain rule to the node samples as in the dense case; streamed passes when
// the context holds their buffers.
fq_status tridiag_adjoint(fq_ctx* c, const void* U_bar, double* grad_f_nodes) {
  if (c->d_adj) return tridiag_adjoint_streamed(c, U_bar, grad_f_nodes);
  const int M = c->M;
  fq::TridiagAdjJob job{};
  job.n = c->n;
  job.ncols = c->n;
  job.h0_diag = c->sys.h0_diag;
  job.h0_off = reinterpret_cast<const double*>(c->sys.h0_off);
  job.v_diag = c->sys.hmod_diag;
  job.ab = c->d_ab;
  job.coef = c->d_coef;
  job.L = c->L;
  job.M = M;
  job.ckpt = c->ckpt;
  job.any_b = c->pair_sums ? 0 : 1;
  job.beta = c->beta;
  job.inv_dE = 1.0 / c->dE;
  job.phr = c->phr;
  job.phi = c->phi;
  job.tape = c->tape;
  job.u_bar = U_bar;
  job.c64 = c->c64 ? 1 : 0;
  job.seg = c->seg;
  job.grad = c->d_grad;
  FQ_HIP(c, zero_async(c->stream, c->d_grad, 2 * sizeof(double) * (size_t)M));
  FQ_HIP(c, fq::launch_tridiag_adjoint(job, c->stream));
  std::vector<double> g(2 * (size_t)M);
  FQ_HIP(c, hipMemcpyAsync(g.data(), c->d_grad, g.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  FQ_HIP(c, hipStreamSynchronize(c->stream));
  grad_to_nodes(c, g, grad_f_nodes);
  return FQ_OK;
}

}  // namespace

// ---- static scratch of the allocation-free one-shot build ------------------------------------
//
// floquet_build_UT_static places the whole workspace of its temporary context
// in this array instead of caller memory. Each GPU the library runs on holds
// its own copy (allocated when the code object loads on that device, kept
// until the process ends). In host code `scratch` names a host-side stand-in,
// not the device array: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// handed to kernels and copies.
constexpr size_t kStaticScratchBytes = size_t(256) << 20;  // 256 MiB
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of the current device's scratch array.
fq_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(FQ_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(FQ_ERR_UNSUPPORTED, "device index %d beyond the %d devices with static scratch",
                dev, kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FQ_ERR_HIP, "hipGetSymbolAddress of the static scratch failed: %s",
                  hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return FQ_OK;
}

}  // namespace

extern "C" {

const char* fq_last_error(void) { return g_err.c_str(); }

fq_status fq_node_times(double T, int32_t M, double* t_out) {
  if (!is_finite(T) || T <= 0) return fail(FQ_ERR_ARG, "T must be finite and > 0");
  if (M < 1) return fail(FQ_ERR_ARG, "M must be >= 1");
  if (!t_out) return fail(FQ_ERR_ARG, "t_out is null");
  fq::gl2_node_times(T, M, t_out);
  return FQ_OK;
}

fq_status fq_node_times_magnus6(double T, int32_t M, double* t_out) {
  if (!is_finite(T) || T <= 0) return fail(FQ_ERR_ARG, "T must be finite and > 0");
  if (M < 1) return fail(FQ_ERR_ARG, "M must be >= 1");
  if (!t_out) return fail(FQ_ERR_ARG, "t_out is null");
  fq::gl3_node_times(T, M, t_out);
  return FQ_OK;
}

fq_status fq_bessel_weights(double R, int32_t L, double* out) {
  if (!is_finite(R) || R < 0) return fail(FQ_ERR_ARG, "R must be finite and >= 0");
  if (L < 0 || L > kMaxOrder) return fail(FQ_ERR_ARG, "L out of range");
  if (!out) return fail(FQ_ERR_ARG, "out is null");
  std::vector<double> j;
  fq::bessel_j_table(R, L, j);
  for (int l = 0; l <= L; ++l) out[l] = (l == 0 ? 1.0 : 2.0) * j[l];
  return FQ_OK;
}

fq_status fq_choose_order(double R, double tol, int32_t* L_out) {
  if (!is_finite(R) || R < 0) return fail(FQ_ERR_ARG, "R must be finite and >= 0");
  if (!is_finite(tol) || tol <= 0) return fail(FQ_ERR_ARG, "tol must be finite and > 0");
  if (!L_out) return fail(FQ_ERR_ARG, "L_out is null");
  const int L = fq::choose_order(R, tol);
  if (L < 1 || L > kMaxOrder) return fail(FQ_ERR_UNSUPPORTED, "required order exceeds %d", kMaxOrder);
  *L_out = L;
  return FQ_OK;
}

fq_status fq_tridiag_extremes(int64_t n, const double* d, const double* e_abs, double* lam_min,
                              double* lam_max) {
  if (n < 1 || !d || (n > 1 && !e_abs) || !lam_min || !lam_max)
    return fail(FQ_ERR_ARG, "bad arguments");
  for (int64_t i = 0; i < n; ++i)
    if (!is_finite(d[i]) || (i + 1 < n && !is_finite(e_abs[i])))
      return fail(FQ_ERR_NONFINITE, "non-finite entry");
  fq::tridiag_extremes((long)n, d, e_abs, lam_min, lam_max);
  return FQ_OK;
}

fq_status fq_hermitian_cover(int64_t n, const void* a, double* lo, double* hi) {
  if (n < 1 || !a || !lo || !hi) return fail(FQ_ERR_ARG, "need n >= 1 and non-null pointers");
  const cd* A = static_cast<const cd*>(a);
  for (int64_t i = 0; i < n * n; ++i)
    if (!std::isfinite(A[i].real()) || !std::isfinite(A[i].imag()))
      return fail(FQ_ERR_NONFINITE, "matrix entry %lld is not finite", (long long)i);
  Matvec mv = [&](const std::vector<cd>& x, std::vector<cd>& y) {
    y.assign(n, cd(0.0, 0.0));
    for (int64_t i = 0; i < n; ++i) {
      cd acc(0.0, 0.0);
      for (int64_t j = 0; j < n; ++j) acc += A[i * n + j] * x[j];
      y[i] = acc;
    }
    return FQ_OK;
  };
  double l, h;
  fq_status st = lanczos_extremes(n, mv, &l, &h);
  if (st != FQ_OK) return st;
  const double w = h - l;
  *lo = l - kDenseMargin * w;
  *hi = h + kDenseMargin * w;
  return FQ_OK;
}

fq_status fq_workspace_bytes(const fq_system* sys, const fq_params* par, size_t* bytes) {
  fq_status st = validate(sys, par);
  if (st != FQ_OK) return st;
  if (!bytes) return fail(FQ_ERR_ARG, "bytes is null");
  *bytes = plan(sys, par).total;
  return FQ_OK;
}

// Everything that follows from the drive samples: the per-(sub)step weights,
// the spectral interval (the caller's, checked against the drive's bounds, or
// the library's cover), beta, dE, R, the order L (unless fixed), the Bessel
// coefficients, the mixed schedule, the step phase, and the device step
// tables. Run by fq_create and again by fq_set_drive.
fq_status apply_drive(fq_ctx* c, const double* f_nodes) {
  c->f_nodes.assign(f_nodes, f_nodes + nodes_per_step(c->scheme) * c->M_user * c->S);
  // per (sub)step: H_eff = H0 + a Hmod + b K
  c->a.resize(c->M);
  c->b.resize(c->M);
  if (c->S > 1) {  // weights of the drive block per (sub)step; a, b unused
    const int S = c->S, J = c->J;
    c->wS.assign((size_t)J * c->M, 0.0);
    const double w = std::sqrt(3.0) * c->h / 12.0;
    for (int k = 0; k < c->M_user; ++k) {
      const double* f1 = &c->f_nodes[(size_t)(2 * k) * S];
      const double* f2 = &c->f_nodes[(size_t)(2 * k + 1) * S];
      if (c->scheme == FQ_CF4) {
        double* w1 = &c->wS[(size_t)J * (2 * k)];
        double* w2 = &c->wS[(size_t)J * (2 * k + 1)];
        for (int d = 0; d < S; ++d) {
          w1[d] = kCf4P * f1[d] + kCf4Q * f2[d];
          w2[d] = kCf4Q * f1[d] + kCf4P * f2[d];
        }
      } else {
        // Magnus-4: a_s, b_s = sqrt(3) h (f_s1 - f_s2) / 12 for K_s, and from
        // [A2, A1] the weight of K_st: sqrt(3) h (f_s2 f_t1 - f_t2 f_s1) / 12
        double* wk = &c->wS[(size_t)J * k];
        int q = 2 * S;
        for (int d = 0; d < S; ++d) {
          wk[d] = 0.5 * (f1[d] + f2[d]);
          wk[S + d] = w * (f1[d] - f2[d]);
          for (int e = d + 1; e < S; ++e, ++q) wk[q] = w * (f2[d] * f1[e] - f2[e] * f1[d]);
        }
      }
    }
    for (int k = 0; k < c->M; ++k) c->a[k] = c->b[k] = 0.0;
  } else if (c->scheme == FQ_MAGNUS6) {
    c->w6.resize((size_t)kComm6 * c->M);
    for (int k = 0; k < c->M; ++k) {
      const double* f = &c->f_nodes[3 * k];
      magnus6_weights(c->h, f[0], f[1], f[2], &c->a[k], &c->w6[(size_t)kComm6 * k]);
      c->b[k] = 1.0;  // the K slot holds the step's commutator sum
    }
  } else if (c->scheme == FQ_CF4) {
    for (int k = 0; k < c->M_user; ++k) {
      const double f1 = c->f_nodes[2 * k], f2 = c->f_nodes[2 * k + 1];
      c->a[2 * k] = kCf4P * f1 + kCf4Q * f2;      // first half-step
      c->a[2 * k + 1] = kCf4Q * f1 + kCf4P * f2;  // second half-step
      c->b[2 * k] = c->b[2 * k + 1] = 0.0;
    }
  } else {
    for (int k = 0; k < c->M; ++k) {
      const double f1 = c->f_nodes[2 * k], f2 = c->f_nodes[2 * k + 1];
      c->a[k] = 0.5 * (f1 + f2);
      c->b[k] = std::sqrt(3.0) * c->h * (f1 - f2) / 12.0;
    }
  }
  // spectral interval
  double lo, hi;
  const bool given = c->interval_given;
  fq_status st;
  if (c->layout == FQ_DENSE)
    st = given ? dense_inner_bounds(c, &lo, &hi) : dense_cover(c, &lo, &hi, kDenseMargin);
  else
    st = tridiag_cover(c, &lo, &hi);
  if (st != FQ_OK) return st;
  if (given) {
    const double slack = 1e-9 * std::max({1.0, std::fabs(lo), std::fabs(hi)});
    if (c->e_min_given > lo + slack || c->e_max_given < hi - slack)
      return fail(FQ_ERR_SPECTRUM,
                  "interval [%.17g, %.17g] does not contain the bounds [%.17g, %.17g]",
                  c->e_min_given, c->e_max_given, lo, hi);
    lo = c->e_min_given;
    hi = c->e_max_given;
  }
  if (!(hi > lo)) {  // a constant H: any positive half-width gives the exact phase
    const double s = std::max(1.0, std::fabs(lo)) * 1e-8;
    lo -= s;
    hi += s;
  }
  c->e_min = lo;
  c->e_max = hi;
  c->beta = 0.5 * (hi + lo);
  c->dE = 0.5 * (hi - lo);
  c->R = c->h * c->dE;
  if (c->L_given > 0) {
    c->L = c->L_given;
  } else {
    c->L = fq::choose_order(c->R, c->tol);
    if (c->L < 1 || c->L > kMaxOrder)
      return fail(FQ_ERR_UNSUPPORTED, "required Chebyshev order exceeds %d (R = %g)", kMaxOrder, c->R);
  }
  std::vector<double> j;
  fq::bessel_j_table(c->R, c->L, j);
  c->weights.resize(c->L + 1);
  c->coef.resize(2 * (c->L + 1));
  for (int l = 0; l <= c->L; ++l) {
    const double w = (l == 0 ? 1.0 : 2.0) * j[l];
    c->weights[l] = w;
    // (-i)^l w
    const int q = l & 3;
    c->coef[2 * l] = (q == 0) ? w : (q == 2 ? -w : 0.0);
    c->coef[2 * l + 1] = (q == 1) ? -w : (q == 3 ? w : 0.0);
  }
  if (c->precision != FQ_FP64 && c->layout == FQ_DENSE) choose_schedule(c);
  c->phr = std::cos(c->beta * c->h);
  c->phi = -std::sin(c->beta * c->h);
  std::vector<double> ab(2 * c->M);
  for (int k = 0; k < c->M; ++k) {
    ab[2 * k] = c->a[k];
    ab[2 * k + 1] = c->b[k];
  }
  if (hipMemcpyAsync(c->d_ab, ab.data(), ab.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->d_coef, c->coef.data(), c->coef.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(FQ_ERR_HIP, "upload of the step tables failed");
  c->tape_valid = false;
  fill_report(c);
  return FQ_OK;
}

fq_status fq_create(fq_ctx** out, const fq_system* sys, const fq_params* par, void* workspace,
                    size_t ws_bytes, void* stream) {
  if (!out) return fail(FQ_ERR_ARG, "out is null");
  *out = nullptr;
  fq_status st = validate(sys, par);
  if (st != FQ_OK) return st;
  const Layout lay = plan(sys, par);
  if (!workspace) return fail(FQ_ERR_ARG, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(FQ_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
  if (ws_bytes < lay.total)
    return fail(FQ_ERR_ARG, "workspace too small: %zu < %zu bytes", ws_bytes, lay.total);

  fq_ctx* c = new (std::nothrow) fq_ctx();
  if (!c) return fail(FQ_ERR_ARG, "out of host memory");
  c->n = sys->n;
  c->layout = dense_like(sys->layout) ? FQ_DENSE : sys->layout;
  c->h0_eigen = sys->layout == FQ_DENSE_EIGEN;
  c->sys = *sys;
  c->T = par->T;
  c->spp = substeps_per_step(par->scheme);
  c->M_user = par->M;
  c->M = par->M * c->spp;
  c->h = par->T / c->M;
  c->tol = par->tol;
  c->precision = par->precision;
  c->ckpt = par->checkpoint_every * c->spp;
  c->profile = par->profile != 0;
  c->reortho = par->reorthonormalize != 0;
  c->c64 = par->dtype == FQ_C64;
  {
    const char* e = std::getenv("FQ_SMALL_CHAIN");
    c->small_chain = !(e && e[0] == '0' && e[1] == 0);
  }
  c->scheme = par->scheme;
  c->pair_sums = par->grad_pair_sums == 1;
  c->S = drive_terms(sys);
  c->J = drive_block(c->S, par->scheme);
  c->mixed_tol = par->mixed_tol;
  if (par->n_term_formats > 0)
    c->term_formats.assign(par->term_formats, par->term_formats + par->n_term_formats);
  c->interval_given = !std::isnan(par->e_min);
  c->e_min_given = par->e_min;
  c->e_max_given = par->e_max;
  c->L_given = par->L;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char*>(workspace);
  c->ws_bytes = ws_bytes;
  c->np = lay.np;
  auto P = [&](size_t off) { return reinterpret_cast<double*>(c->ws + off); };
  const size_t plane = (size_t)lay.np * (size_t)lay.np;
  c->small = P(lay.off_small);
  c->d_vec = P(lay.off_vec);
  c->d_ab = P(lay.off_ab);
  c->d_coef = P(lay.off_coef);
  c->xr = P(lay.off_x);
  if (sys->layout == FQ_TRIDIAG) {
    if (par->reorthonormalize) {
      c->par = P(lay.off_pa); c->pai = c->par + plane;
      c->pbr = P(lay.off_pb); c->pbi = c->pbr + plane;
      c->yr = P(lay.off_y);   c->yi = c->yr + plane;
    }
    c->d_gauge = P(lay.off_gauge);
    if (lay.off_stream) c->d_stream = P(lay.off_stream);
    if (lay.n_tape > 0) {
      c->tape = P(lay.off_tape);
      c->n_tape = lay.n_tape;
      c->seg = P(lay.off_seg);
      c->d_grad = P(lay.off_grad);
      if (lay.off_adj) c->d_adj = P(lay.off_adj);
    }
  }
  c->xi = c->xr + plane;
  if (dense_like(sys->layout)) {
    c->h0r = P(lay.off_h0); c->h0i = c->h0r + plane;
    // drive block: re(B_0..B_{J-1}), then im; one term: B_0 = Hmod, B_1 = K
    c->vr = P(lay.off_v);   c->kr = c->vr + plane;
    c->vi = c->vr + (size_t)c->J * plane; c->ki = c->vi + plane;
    c->htr = P(lay.off_ht); c->hti = c->htr + plane;
    c->yr = P(lay.off_y);   c->yi = c->yr + plane;
    c->par = P(lay.off_pa); c->pai = c->par + plane;
    c->pbr = P(lay.off_pb); c->pbi = c->pbr + plane;
    if (par->precision != FQ_FP64) c->htx = P(lay.off_htx);
    if (par->precision != FQ_FP64) c->pcr = P(lay.off_pc);
    if (par->scheme == FQ_MAGNUS6) c->comm6 = P(lay.off_comm6);
    if (lay.n_tape > 0) {
      c->tape = P(lay.off_tape);
      c->n_tape = lay.n_tape;
      c->seg = P(lay.off_seg);
      c->stack[0] = P(lay.off_stack);
      c->stack[1] = c->stack[0] + 4 * plane;
      c->lam = P(lay.off_lam);
      c->d_grad = P(lay.off_grad);
      if (lay.off_drive32) {
        c->drive32 = reinterpret_cast<float*>(c->ws + lay.off_drive32);
        c->adj_f32 = true;
      }
    }
  }

  auto bail = [&](fq_status s) {
    delete c;
    return s;
  };
  if (zero_async(c->stream, c->ws, lay.total) != hipSuccess)
    return bail(fail(FQ_ERR_HIP, "zeroing the workspace failed"));

  const long n = c->n;
  if (c->layout == FQ_DENSE) {
    // planar H0 (diag(E) in the eigenbasis layout), the drive matrices, and their
    // commutators: K = -i [H0, Hmod] for one term; for S terms K_s = -i [H0, Hmod_s]
    // and K_st = -i [Hmod_s, Hmod_t] (FQ_MAGNUS4). Products on FP64 matrix cores,
    // (X Y)(i, j) = sum_k X(i, k) conj(Y(j, k)) for Hermitian Y; commutators with
    // diag(E) elementwise.
    const int np = (int)c->np;
    const size_t plane = (size_t)c->np * (size_t)c->np;
    auto bre = [&](int j) { return c->vr + (size_t)j * plane; };
    auto bim = [&](int j) { return c->vi + (size_t)j * plane; };
    hipError_t he = c->h0_eigen ? fq::launch_diag_planar(sys->h0_diag, n, np, c->h0r, c->stream)
                                : fq::launch_pack_planar(sys->h0, n, n, n, c->h0r, c->h0i, np,
                                                         c->stream);
    for (int d = 0; d < c->S && he == hipSuccess; ++d)
      he = fq::launch_pack_planar(c->S == 1 ? sys->hmod : sys->hmods[d], n, n, n, bre(d), bim(d),
                                  np, c->stream);
    if (he != hipSuccess)
      return bail(fail(FQ_ERR_HIP, "setup kernels failed: %s", hipGetErrorString(he)));
    if (c->S == 1) {
      st = hermitian_commutator(c, c->h0r, c->h0i, c->vr, c->vi, -1.0, c->kr, c->ki);
    } else if (c->scheme == FQ_MAGNUS4) {
      for (int d = 0; d < c->S && st == FQ_OK; ++d)
        st = hermitian_commutator(c, c->h0r, c->h0i, bre(d), bim(d), -1.0, bre(c->S + d),
                                  bim(c->S + d));
      int q = 2 * c->S;
      for (int d = 0; d < c->S; ++d)
        for (int e = d + 1; e < c->S && st == FQ_OK; ++e, ++q)
          st = hermitian_commutator(c, bre(d), bim(d), bre(e), bim(e), -1.0, bre(q), bim(q));
    }
    if (st == FQ_OK && c->scheme == FQ_MAGNUS6) st = magnus6_commutators(c);
    if (st != FQ_OK) return bail(st);
    if (c->drive32) {  // both planes of all J drive matrices, in their order
      he = fq::launch_f64_to_f32(c->vr, c->drive32, 2L * c->J * (long)plane, c->stream);
      if (he != hipSuccess)
        return bail(fail(FQ_ERR_HIP, "setup kernels failed: %s", hipGetErrorString(he)));
    }
  }

  st = apply_drive(c, par->f_nodes);
  if (st != FQ_OK) return bail(st);
  *out = c;
  return FQ_OK;
}

fq_status fq_destroy(fq_ctx* ctx) {
  delete ctx;
  return FQ_OK;
}

fq_status fq_set_drive(fq_ctx* c, const double* f_nodes) {
  if (!c || !f_nodes) return fail(FQ_ERR_ARG, "null argument");
  if (c->broken) return fail(FQ_ERR_HIP, "context unusable after an earlier HIP failure");
  const long cnt = (long)nodes_per_step(c->scheme) * c->M_user * c->S;
  for (long i = 0; i < cnt; ++i)
    if (!is_finite(f_nodes[i])) return fail(FQ_ERR_NONFINITE, "f_nodes[%ld] is not finite", i);
  const fq_status st = apply_drive(c, f_nodes);
  c->drive_ok = st == FQ_OK;
  return st;
}

fq_status fq_get_report(const fq_ctx* ctx, fq_report* rep) {
  if (!ctx || !rep) return fail(FQ_ERR_ARG, "null argument");
  *rep = ctx->last;
  return FQ_OK;
}

fq_status floquet_build_UT(fq_ctx* c, void* U_out, fq_report* rep) {
  if (!c || !U_out) return fail(FQ_ERR_ARG, "null argument");
  if (c->broken) return fail(FQ_ERR_HIP, "context unusable after an earlier HIP failure");
  if (!c->drive_ok) return fail(FQ_ERR_STATE, "the last fq_set_drive failed: set a valid drive first");
  // The build's two timing events live with the context (created once, freed
  // by fq_destroy), so that no return path leaks them.
  if (c->timed && !c->build_ev[0]) {
    FQ_HIP(c, hipEventCreate(&c->build_ev[0]));
    FQ_HIP(c, hipEventCreate(&c->build_ev[1]));
  }
  hipEvent_t e0 = c->build_ev[0], e1 = c->build_ev[1];
  fq_status st = FQ_OK;
  c->n_events = 0;
  if (c->layout == FQ_DENSE) {
    FQ_HIP(c, fq::launch_identity_rows(c->xr, c->xi, c->n, c->np, c->np, c->stream));
    if (e0) FQ_HIP(c, hipEventRecord(e0, c->stream));
    st = dense_steps(c, 0, c->M, (int)c->np, c->ckpt > 0);
    if (st != FQ_OK) return st;
    FQ_MARK(c, -1);
    if (e1) FQ_HIP(c, hipEventRecord(e1, c->stream));
    FQ_HIP(c, fq::launch_unpack_planar_t(c->xr, c->xi, c->np, c->n, c->n, U_out, c->n, c->c64,
                                       c->stream));
    c->tape_valid = c->ckpt > 0;
    st = unitarity(c, c->xr, c->xi);
    if (st == FQ_OK && c->reortho) st = finish_reortho(c, U_out);
  } else {
    if (e0) FQ_HIP(c, hipEventRecord(e0, c->stream));
    // Streamed columns record the checkpoints X_{j ckpt}, j >= 1, through the
    // snapshot store (row-major, tape entries 1, 2, ...); entry 0 is the identity.
    const bool snap_tape = c->ckpt > 0 && c->n > fq::tridiag_resident_max_n();
    if (snap_tape) {
      c->snap = c->tape + 2 * (size_t)c->n * (size_t)c->n;
      c->snap_every = c->ckpt;
      c->snap_k0 = 0;
      c->snap_ncols = c->n;
    }
    st = tridiag_run(c, nullptr, c->n, 0, c->M, U_out);
    c->snap = nullptr;
    if (st != FQ_OK) return st;
    FQ_MARK(c, -1);
    if (e1) FQ_HIP(c, hipEventRecord(e1, c->stream));
    c->tape_valid = c->ckpt > 0;
    FQ_HIP(c, fq::launch_pack_planar_t(U_out, c->n, c->n, c->n, c->xr, c->xi, c->np, c->np, c->c64,
                                       c->stream));
    st = unitarity(c, c->xr, c->xi);
    if (st == FQ_OK && c->reortho) st = finish_reortho(c, U_out);
  }
  if (st != FQ_OK) return st;
  float ms = 0.f;
  if (e1) {
    FQ_HIP(c, hipEventSynchronize(e1));
    FQ_HIP(c, hipEventElapsedTime(&ms, e0, e1));
  }
  c->last.ms_build = ms;
  st = collect_profile(c);
  if (st != FQ_OK) return st;
  fill_report(c);
  if (rep) *rep = c->last;
  return FQ_OK;
}

fq_status floquet_propagate(fq_ctx* c, const void* X0, int64_t ncols, int32_t k0, int32_t k1,
                            void* X_out, void* snapshots, int32_t snap_every) {
  if (!c || !X0 || !X_out) return fail(FQ_ERR_ARG, "null argument");
  if (c->broken) return fail(FQ_ERR_HIP, "context unusable after an earlier HIP failure");
  if (!c->drive_ok) return fail(FQ_ERR_STATE, "the last fq_set_drive failed: set a valid drive first");
  if (ncols < 1 || ncols > c->n) return fail(FQ_ERR_ARG, "ncols must be in [1, n]");
  if (k0 < 0 || k1 < k0 || k1 > c->M_user) return fail(FQ_ERR_ARG, "need 0 <= k0 <= k1 <= M");
  if (snapshots && snap_every < 1) return fail(FQ_ERR_ARG, "snap_every must be >= 1 with snapshots");
  if (!snapshots && snap_every != 0) return fail(FQ_ERR_ARG, "snap_every without a snapshot buffer");
  struct SnapReset {
    fq_ctx* c;
    ~SnapReset() { c->snap = nullptr; }
  } snap_reset{c};
  // the library's substeps (FQ_CF4: two per step)
  k0 *= c->spp;
  k1 *= c->spp;
  c->snap = snapshots;
  c->snap_every = snap_every * c->spp;
  c->snap_k0 = k0;
  c->snap_ncols = ncols;
  c->n_events = 0;
  if (k0 == k1) {  // no steps: X_out = X0 (and no snapshot falls in the empty range)
    const size_t bytes = (size_t)c->n * (size_t)ncols * (c->c64 ? 8 : 16);
    if (X_out != X0)
      FQ_HIP(c, hipMemcpyAsync(X_out, X0, bytes, hipMemcpyDeviceToDevice, c->stream));
    FQ_HIP(c, hipStreamSynchronize(c->stream));
    return collect_profile(c);
  }
  if (c->layout == FQ_DENSE) {
    const long mrows = pad_to(ncols, dense_tile(c->n));
    FQ_HIP(c, fq::launch_pack_planar_t(X0, c->n, ncols, ncols, c->xr, c->xi, c->np, mrows, c->c64,
                                       c->stream));
    fq_status st = dense_steps(c, k0, k1, (int)mrows, false);
    if (st != FQ_OK) return st;
    FQ_MARK(c, -1);
    FQ_HIP(c, fq::launch_unpack_planar_t(c->xr, c->xi, c->np, c->n, ncols, X_out, ncols, c->c64,
                                         c->stream));
  } else {
    fq_status st = tridiag_run(c, X0, ncols, k0, k1, X_out);
    if (st != FQ_OK) return st;
    FQ_MARK(c, -1);
  }
  FQ_HIP(c, hipStreamSynchronize(c->stream));
  return collect_profile(c);
}

// Period average of the energy (Sec. 3, Eq. (average) with A(t) = H(t)) by the
// rectangle rule on the step grid: avg_c = (1/M) sum_{k<M} <x_k|H(t_k)|x_k> / <x_k|x_k>,
// x_k = E_k ... E_1 x_0, t_k = k h. For a Floquet state the integrand is smooth
// and T-periodic, where this rule converges faster than any power of h.
fq_status floquet_period_average(fq_ctx* c, const void* X0, int64_t ncols, const double* f_grid,
                                 double* avg_out) {
  if (!c || !X0 || !f_grid || !avg_out) return fail(FQ_ERR_ARG, "null argument");
  if (c->broken) return fail(FQ_ERR_HIP, "context unusable after an earlier HIP failure");
  if (!c->drive_ok) return fail(FQ_ERR_STATE, "the last fq_set_drive failed: set a valid drive first");
  if (ncols < 1 || ncols > c->n) return fail(FQ_ERR_ARG, "ncols must be in [1, n]");
  for (int k = 0; k < c->M_user * c->S; ++k)
    if (!is_finite(f_grid[k])) return fail(FQ_ERR_NONFINITE, "f_grid[%d] is not finite", k);
  c->n_events = 0;
  c->snap = nullptr;
  const int spp = c->spp;
  const double w = 1.0 / c->M_user;
  double* avg = c->d_vec;
  double* num = c->d_vec + c->n;
  double* den = c->d_vec + 2 * c->n;
  FQ_HIP(c, fq::launch_fill_zero(c->d_vec, 3 * c->n, c->stream));
  if (c->layout == FQ_DENSE) {
    const int np = (int)c->np;
    const long mrows = pad_to(ncols, dense_tile(c->n));
    FQ_HIP(c, fq::launch_pack_planar_t(X0, c->n, ncols, ncols, c->xr, c->xi, c->np, mrows, c->c64,
                                       c->stream));
    for (int k = 0; k < c->M_user; ++k) {
      // H(t_k) into the Ht planes (free between steps), H(t_k) x into the P planes
      fq::WeightedSum ws{};
      ws.re[0] = c->h0r; ws.im[0] = c->h0i; ws.w[0] = 1.0;
      for (int d = 0; d < c->S; ++d) {  // drive matrices are the first S of the block
        ws.re[1 + d] = c->vr + (size_t)d * c->np * c->np;
        ws.im[1 + d] = c->vi + (size_t)d * c->np * c->np;
        ws.w[1 + d] = f_grid[(size_t)k * c->S + d];
      }
      ws.count = 1 + c->S;
      FQ_HIP(c, fq::launch_weighted_sum(ws, c->np * c->np, c->htr, c->hti, c->stream));
      FQ_HIP(c, fq::launch_zgemm_nt_f64(c->xr, c->xi, false, c->htr, c->hti, false, c->par,
                                        c->pai, (int)mrows, np, np, np, 1.0, 0.0, 0.0, 0.0,
                                        c->stream));
      FQ_HIP(c, fq::launch_energy_rows(c->xr, c->xi, c->par, c->pai, ncols, c->n, c->np, w, avg,
                                       c->stream));
      FQ_TRY(dense_steps(c, k * spp, (k + 1) * spp, (int)mrows, false));
    }
  } else {
    // the states in the user layout, propagated in place one step at a time
    void* x = c->xr;
    const size_t bytes = (size_t)c->n * (size_t)ncols * (c->c64 ? 8 : 16);
    FQ_HIP(c, hipMemcpyAsync(x, X0, bytes, hipMemcpyDeviceToDevice, c->stream));
    for (int k = 0; k < c->M_user; ++k) {
      FQ_HIP(c, fq::launch_tridiag_energy(x, c->c64, c->n, ncols, c->sys.h0_diag, c->sys.h0_off,
                                          c->sys.hmod_diag, f_grid[k], num, den, c->stream));
      FQ_HIP(c, fq::launch_energy_finish(num, den, ncols, w, avg, c->stream));
      FQ_TRY(tridiag_run(c, x, ncols, k * spp, (k + 1) * spp, x));
    }
  }
  FQ_MARK(c, -1);
  FQ_HIP(c, hipMemcpyAsync(avg_out, avg, ncols * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  FQ_HIP(c, hipStreamSynchronize(c->stream));
  return collect_profile(c);
}

fq_status floquet_grad(fq_ctx* c, const void* U_bar, double* grad_f_nodes) {
  if (!c || !U_bar || !grad_f_nodes) return fail(FQ_ERR_ARG, "null argument");
  if (c->broken) return fail(FQ_ERR_HIP, "context unusable after an earlier HIP failure");
  if (!c->drive_ok) return fail(FQ_ERR_STATE, "the last fq_set_drive failed: set a valid drive first");
  if (c->ckpt <= 0) return fail(FQ_ERR_STATE, "context was created without a gradient tape");
  if (!c->tape_valid) return fail(FQ_ERR_STATE, "no tape: call floquet_build_UT first");
  if (c->layout == FQ_TRIDIAG) return tridiag_adjoint(c, U_bar, grad_f_nodes);
  // The segment recomputation runs in FP64 whatever the build precision (the
  // sweep differentiates the FP64 Chebyshev map); the reverse products run in
  // FP64, or on FP32 matrix cores for FQ_FP32 contexts (adj_f32).
  struct Restore {
    fq_ctx* c;
    int prec;
    bool prof;
    ~Restore() {
      c->precision = prec;
      c->profile = prof;
      c->save_pl = c->save_plm1 = nullptr;
    }
  } restore{c, c->precision, c->profile};
  c->precision = FQ_FP64;
  fq_status st = adjoint(c, U_bar, grad_f_nodes);
  return st;
}

fq_status floquet_build_UT_static(const fq_system* sys, const fq_params* par, void* stream,
                                  void* U_out, fq_report* rep) {
  if (!U_out) return fail(FQ_ERR_ARG, "U_out is null");
  fq_status st = validate(sys, par);
  if (st != FQ_OK) return st;
  if (par->checkpoint_every != 0)
    return fail(FQ_ERR_UNSUPPORTED, "the one-shot build keeps no gradient tape "
                                    "(checkpoint_every must be 0)");
  if (par->profile != 0)
    return fail(FQ_ERR_UNSUPPORTED, "the one-shot build does not time kernels (profile must be 0)");
  const size_t need = plan(sys, par).total;
  if (need > kStaticScratchBytes)
    return fail(FQ_ERR_ARG, "this build needs %zu bytes of workspace, more than the %zu bytes of "
                "static scratch; create a context with a caller workspace instead",
                need, kStaticScratchBytes);
  void* ws = nullptr;
  st = static_scratch(&ws);
  if (st != FQ_OK) return st;
  fq_ctx* c = nullptr;
  st = fq_create(&c, sys, par, ws, kStaticScratchBytes, stream);
  if (st != FQ_OK) return st;
  c->timed = false;  // no events: ms_build is reported as 0
  st = floquet_build_UT(c, U_out, rep);
  delete c;
  return st;
}

}  // extern "C"
