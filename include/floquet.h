/*
 * floquet.h -- C ABI of the MI355X Floquet-operator library (libfloquet.so).
 *
 * The library builds the one-period propagator ("Floquet operator") U_T of
 *     i dX/dt = H(t) X,   H(t) = H0 + f(t) Hmod,   f(t + T) = f(t)
 * (Laptyeva et al., arXiv:1508.07621, Sec. 3, Eq. (13); propagator Sec. 2,
 * Eqs. (1) and (3); hbar = 1) as a chain of M single-step exponentials
 * (Sec. 2, Eq. (9)), each applied to all N columns at once (Sec. 3 and Sec. 5:
 * the identity is propagated as a block, so the work is matrix-matrix products).
 *
 * One step k (time t_{k-1} = (k-1) h to t_k, h = T / M):
 *   - Magnus-4 effective Hamiltonian from the drive at the two Gauss-Legendre
 *     nodes t_{k-1} + (1/2 -/+ sqrt(3)/6) h (values f1, f2; Sec. 2, Eq. (8)
 *     truncated after its commutator term):
 *         H_eff,k = H0 + a_k Hmod + b_k K,   K = -i [H0, Hmod],
 *         a_k = (f1 + f2) / 2,   b_k = sqrt(3) h (f1 - f2) / 12;
 *   - rescaling into [-1, 1] (Sec. 2, Eq. (11)):
 *         Ht = (H_eff,k - beta) / dE,  beta = (e_max + e_min) / 2,
 *         dE = (e_max - e_min) / 2,    R = h dE;
 *     or, with fq_params.scheme = FQ_MAGNUS6, the paper's own sixth-order
 *     scheme (Sec. 3, Eq. (14)) from the drive at the three Gauss-Legendre
 *     nodes t_{k-1} + (1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10) h (values
 *     f1, f2, f3), for the generator A(t) = -i H(t):
 *         alpha_1 = h A(f2), alpha_2 = (sqrt(15) h / 3)(A(f3) - A(f1)),
 *         alpha_3 = (10 h / 3)(A(f3) - 2 A(f2) + A(f1)),
 *         C_1 = [alpha_1, alpha_2], C_2 = -[alpha_1, 2 alpha_3 + C_1] / 60,
 *         Omega = alpha_1 + alpha_3 / 12
 *                 + [-20 alpha_1 - alpha_3 + C_1, alpha_2 + C_2] / 240,
 *         H_eff,k = i Omega / h
 *     (the alpha_j as quadrature combinations rather than scaled midpoint
 *     derivatives: with them the scheme has order six). H_eff,k is a real
 *     combination of H0, Hmod and nine nested commutators of H0 and Hmod,
 *     formed once per context (dense layout only);
 *   - Chebyshev expansion with Bessel weights (Sec. 2, Eqs. (10)-(12)), in the
 *     equivalent real-multiplier form
 *         P_0 = X, P_1 = Ht X, P_{l+1} = 2 Ht P_l - P_{l-1},
 *         X <- exp(-i beta h) sum_{l=0..L} c_l P_l,
 *         c_0 = J_0(R), c_l = 2 (-i)^l J_l(R).
 *
 * Conventions for every entry point:
 *   - complex numbers are complex128 (two float64, real part first), except
 *     the state blocks when fq_params.dtype = FQ_C64 (complex64);
 *   - dense matrices are row-major, element [i][j] = <i|A|j>; the columns of
 *     X, U_T and X0 are the propagated states;
 *   - "device" pointers are HIP device memory owned by the caller; the library
 *     never allocates or frees device memory (the caller hands in one
 *     workspace, sized by fq_workspace_bytes); "host" pointers are ordinary
 *     host memory owned by the caller;
 *   - all device work is enqueued on the stream given to fq_create; entry
 *     points that return host values synchronise that stream first;
 *   - every entry point returns fq_status; FQ_OK == 0. Arguments are checked
 *     before any device work; on a non-OK status the outputs are unspecified
 *     and fq_last_error() describes the failure (thread-local string). The
 *     context stays usable after every error except FQ_ERR_HIP.
 */
#ifndef FLOQUET_H
#define FLOQUET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FQ_OK = 0,
  FQ_ERR_ARG = 1,          /* invalid argument: size, null pointer, range, layout */
  FQ_ERR_NONFINITE = 2,    /* NaN / Inf in a host scalar or array argument */
  FQ_ERR_SPECTRUM = 3,     /* given interval does not contain the library's bounds */
  FQ_ERR_HIP = 4,          /* a HIP runtime call failed; the context is unusable */
  FQ_ERR_UNSUPPORTED = 5,  /* valid request the library does not implement */
  FQ_ERR_STATE = 6         /* call out of order (e.g. floquet_grad without a tape) */
} fq_status;

/* FQ_DENSE_EIGEN: the dense model written in the eigenbasis of H0 (Sec. 3,
 * Eq. (Ham2)): H0 = diag(E_i), given as h0_diag, and Hmod dense in that basis.
 * Every commutator with H0 is then elementwise, [H0, X]_ij = (E_i - E_j) X_ij,
 * and the extremes of H0 are exact; the Chebyshev products are the dense ones. */
typedef enum { FQ_DENSE = 0, FQ_TRIDIAG = 1, FQ_DENSE_EIGEN = 2 } fq_layout;

/* Arithmetic of the Chebyshev products. FQ_FP64: everything in float64.
 * FQ_FP32: products on FP32 matrix cores with FP32 accumulation (the first
 * product of a step on FP64 matrix cores); P_l stored FP32; X, the Chebyshev
 * sum and the step phase stay float64.
 * FQ_BF16X3: products on BF16 matrix cores with operands split into BF16
 * pieces, each term in its own fq_term_format chosen from its Bessel weight;
 * P_l stored as three BF16 pieces (about 24 bits); X and the Chebyshev sum
 * float64. Setup, coefficients and checks are always float64. */
typedef enum { FQ_FP64 = 0, FQ_FP32 = 1, FQ_BF16X3 = 2 } fq_precision;

/* Format of one Chebyshev product P_l = 2 Ht P_{l-1} - P_{l-2} (P_1 = Ht X) of
 * an FQ_BF16X3 build. Its rounding error enters the step's sum weighted by
 * |c_l| = 2 |J_l(R)| (Sec. 2, Eq. (12)), so the library picks for each term
 * the cheapest format whose estimated contribution stays within the error
 * target (fq_params.mixed_tol), unless the caller fixes them. */
typedef enum fq_term_format {
  FQ_TERM_FP64 = 0,          /* FP64 matrix cores on FP64 operands */
  FQ_TERM_BF16X3_F64ACC = 1, /* three BF16 pieces per operand, FP32 partial
                                sums of each 64-column block added in FP64:
                                about 24 significant bits, independent of N */
  FQ_TERM_BF16X3 = 2,        /* three BF16 pieces, FP32 accumulation */
  FQ_TERM_BF16X2 = 3,        /* two BF16 pieces (about 16 bits) */
  FQ_TERM_BF16X1 = 4,        /* one BF16 piece (about 8 bits) */
  FQ_TERM_FP32 = 5           /* FP32 matrix cores on FP32 operands: the
                                products of FQ_FP32 builds after their leading
                                FP64 run (not selectable in term_formats) */
} fq_term_format;

/* The time-independent operators of H(t) = H0 + f(t) Hmod (Sec. 3, Eq. (13)),
 * or of H(t) = H0 + sum_s f_s(t) Hmod_s with several drive terms (Sec. 3 notes
 * the generalisation): n_drive = S >= 2 drive matrices given by hmods. */
typedef struct fq_system {
  int64_t n;                 /* dimension N >= 1 */
  int32_t layout;            /* fq_layout */
  int32_t n_drive;           /* 0 or 1: one drive term (hmod / hmod_diag);
                                2..4: that many dense drive matrices in hmods
                                (dense layouts; FQ_MAGNUS4 or FQ_CF4). With S
                                terms every per-node array (f_nodes, the
                                gradient, f_grid) holds S values per entry, term
                                index fastest. */
  /* FQ_DENSE: device, n*n complex128, row-major, Hermitian (not checked).
   * FQ_DENSE_EIGEN: hmod as for FQ_DENSE (in H0's eigenbasis), h0 unused, and
   * h0_diag (below) holds the n eigenvalues E_i of H0. */
  const void* h0;
  const void* hmod;
  /* FQ_TRIDIAG: H0 Hermitian tridiagonal, Hmod real diagonal (the dimer of
   * Sec. 4 has exactly this structure in its Fock basis). Device pointers:
   * h0_diag n float64, h0_off n-1 complex128 with h0_off[i] = H0[i][i+1]
   * (H0[i+1][i] is its conjugate), hmod_diag n float64. */
  const double* h0_diag;
  const void* h0_off;
  const double* hmod_diag;
  /* n_drive >= 2: host array of n_drive device pointers, each an n*n
   * complex128 row-major Hermitian matrix (in H0's eigenbasis for
   * FQ_DENSE_EIGEN); hmod is then unused. */
  const void* const* hmods;
} fq_system;

/* Step operator. FQ_MAGNUS4: two Gauss-Legendre nodes, one commutator (fourth
 * order). FQ_MAGNUS6: the paper's Eq. (14) from three Gauss-Legendre nodes
 * (sixth order); dense layout, no gradient tape. FQ_CF4: commutator-free
 * (the variant the paper names as an improvement, Sec. 2 and Sec. 8): two
 * exponentials of linear combinations of H at the two Gauss-Legendre nodes,
 *     E_k = exp(-i h (a2 H(f1) + a1 H(f2))) exp(-i h (a1 H(f1) + a2 H(f2))),
 *     a1 = 1/4 + sqrt(3)/6, a2 = 1/4 - sqrt(3)/6 (fourth order),
 * each run as one Chebyshev propagation over h/2 of H0 + a Hmod; no commutator
 * is formed, so it serves both layouts and the gradient. */
typedef enum fq_scheme { FQ_MAGNUS4 = 0, FQ_MAGNUS6 = 1, FQ_CF4 = 2 } fq_scheme;

/* Storage of the state blocks that cross the boundary: U_T, X0, X_out, the
 * snapshots and U_bar. Operators stay complex128 / float64. */
typedef enum fq_dtype {
  FQ_C128 = 0,  /* complex128 (interleaved float64 pairs) */
  FQ_C64 = 1    /* complex64 (interleaved float32 pairs); the library still
                   propagates in its own working precision and rounds on output */
} fq_dtype;

/* Time grid, drive samples and method parameters. */
typedef struct fq_params {
  double T;                  /* period > 0 */
  int32_t M;                 /* steps per period >= 1; h = T / M */
  int32_t L;                 /* Chebyshev order; 0 = smallest L with
                                2 sum_{l>L} |J_l(R)| <= tol (FQ_CF4: R of the
                                half step, h dE / 2) */
  const double* f_nodes;     /* host, float64: f at the Gauss-Legendre nodes
                                of each step in time order, 2*M values for
                                FQ_MAGNUS4 and FQ_CF4 (fq_node_times gives the
                                times) or 3*M for FQ_MAGNUS6
                                (fq_node_times_magnus6) */
  double e_min, e_max;       /* spectral interval containing the spectrum of
                                every H_eff,k; both NaN = the library computes
                                it (tridiagonal: exact per-step extremes by
                                Sturm bisection; dense: Weyl cover from the
                                bounds fq_hermitian_cover gives for H0 and Hmod).
                                A given interval is rejected with
                                FQ_ERR_SPECTRUM when it misses a point known to
                                lie in some step's spectral hull (tridiagonal:
                                the exact extremes; dense: Ritz values of H_eff
                                at the steps with the smallest and largest
                                weight of Hmod; FQ_CF4: of each half-step's
                                operator). FQ_MAGNUS6 widens the dense
                                cover by sum_j |w_j| times a bound on the norm
                                of each nested commutator (||[A, B]|| <=
                                2 ||A|| ||B||) */
  double tol;                /* truncation tolerance used when L == 0 (> 0) */
  int32_t precision;         /* fq_precision (FQ_TRIDIAG supports FQ_FP64 only) */
  int32_t checkpoint_every;  /* > 0: floquet_build_UT keeps X_0, X_s, X_2s, ...
                                (s = checkpoint_every) for floquet_grad;
                                0 = no tape. FQ_MAGNUS4 only. */
  int32_t profile;           /* 1: time every kernel launch of a build with HIP
                                events on the library's stream and report the
                                per-kind sums in fq_report; 0: off */
  int32_t reorthonormalize;  /* 1: after the build replace U_T by its polar
                                factor U (U^dagger U)^(-1/2), the nearest
                                unitary matrix in the Frobenius norm, by two
                                FP64 Newton-Schulz steps
                                X <- X (3 - X^dagger X) / 2 on the device; the
                                report gives the unitarity before and after
                                (a correction of the result, not part of the
                                paper's method). 0: off */
  int32_t dtype;             /* fq_dtype of the state blocks */
  int32_t scheme;            /* fq_scheme; FQ_MAGNUS6 needs FQ_DENSE and
                                checkpoint_every == 0 (else
                                FQ_ERR_UNSUPPORTED) */
  double mixed_tol;          /* FQ_BF16X3 and FQ_FP32: target for the
                                rounding error the products add to U_T (worst
                                column 2-norm), from which each term's format
                                is chosen (FQ_FP32: FP64 or FP32, the first
                                term always FP64); 0 = 5e-7 */
  const int32_t* term_formats;  /* FQ_BF16X3, host, nullable: fq_term_format of
                                terms 1 .. n_term_formats (the last entry
                                repeats for later terms) instead of the
                                library's choice; FQ_TERM_FP64 only on a
                                leading run of terms */
  int32_t n_term_formats;    /* entries of term_formats (0 when NULL) */
  int32_t grad_pair_sums;    /* floquet_grad with one drive term: 0 = the
                                derivative with respect to every node sample;
                                1 = only the sums over each step's two nodes,
                                grad[2k] + grad[2k+1] = dLoss/dA_k for an
                                amplitude A_k moving both nodes of step k
                                together (the caller's drive need not be
                                constant over the step), returned as two equal
                                halves. The commutator K enters H_eff through
                                b_k, proportional to the node difference, so
                                its contraction cancels in these sums and is
                                skipped. Ignored with several drive terms. */
} fq_params;

/* Kernel kinds timed in profile mode (indices of fq_report.ms_kernel). */
enum {
  FQ_K_FIRST = 0,       /* first Chebyshev product of a step (P_1 = Ht X) */
  FQ_K_FIRST_LAST = 1,  /* the only product of a step when L == 1 */
  FQ_K_MID = 2,         /* products P_{l+1} = 2 Ht P_l - P_{l-1}, 1 <= l < L-1 */
  FQ_K_LAST = 3,        /* last product of a step, with the phase and hand-off */
  FQ_K_HEFF = 4,        /* per-step rescaled Hamiltonian */
  FQ_K_TRIDIAG = 5,     /* tridiagonal whole-chain kernel */
  FQ_K_ADJ_FWD = 6,     /* gradient, streamed tridiagonal: segment recompute pass */
  FQ_K_ADJ_REV = 7,     /* gradient: reverse-sweep products (dense) or reverse passes
                           (streamed tridiagonal); after floquet_grad the dense
                           segment recompute's products appear under FIRST / MID /
                           LAST / HEFF */
  /* FQ_BF16X3 builds time their products by format instead of position: */
  FQ_K_TERM_FP64 = 8,       /* FQ_TERM_FP64 products */
  FQ_K_TERM_F64ACC = 9,     /* FQ_TERM_BF16X3_F64ACC */
  FQ_K_TERM_X3 = 10,        /* FQ_TERM_BF16X3 */
  FQ_K_TERM_X2 = 11,        /* FQ_TERM_BF16X2 */
  FQ_K_TERM_X1 = 12,        /* FQ_TERM_BF16X1 */
  FQ_K_CONVERT = 13,        /* FP64 planes rounded into the BF16X3 format */
  FQ_K_CHAIN = 14,          /* dense N <= 64 in FP64: every step of the range in one
                               launch (Ht, all terms and the hand-off per step) */
  FQ_K_SLOTS = 16
};
#define FQ_TERM_SLOTS 16

/* Setup values and per-build measurements. */
typedef struct fq_report {
  int32_t L;                 /* Chebyshev order in use */
  int32_t M;
  double R, dE, beta;        /* R = h dE; beta = interval midpoint */
  double e_min, e_max;       /* interval in use */
  double unitarity_max;      /* max |(U^dagger U - 1)_ij| of the last build (FP64) */
  double unitarity_fro;      /* Frobenius norm of U^dagger U - 1 */
  double unitarity_max_after;  /* the same after re-orthonormalisation (0 if off) */
  double unitarity_fro_after;
  double ms_build;           /* device time of the last build, milliseconds */
  double ms_kernel[FQ_K_SLOTS];   /* profile mode: summed event time per kind */
  int32_t n_kernel[FQ_K_SLOTS];   /* profile mode: launches per kind */
  int32_t term_format[FQ_TERM_SLOTS];  /* FQ_BF16X3 and FQ_FP32: fq_term_format
                                          of terms 1 .. min(L, 16) (later terms
                                          are not listed); FQ_FP64 builds and
                                          unused entries: -1 */
  double mixed_err_est;           /* FQ_BF16X3 and FQ_FP32: the error estimate
                                     the schedule was chosen for (0 otherwise) */
  int32_t diverged;               /* 1 when the last build's max |(U^dagger U -
                                     1)_ij| exceeds 1e-3 (or is not finite): the
                                     Chebyshev series diverged, e.g. because a
                                     step's spectrum left the interval; 0
                                     otherwise */
} fq_report;

typedef struct fq_ctx fq_ctx;  /* opaque; host memory owned by the library */

/* Gauss-Legendre sampling times of the drive: t_out[2k] and t_out[2k+1] are
 * the earlier and later node of step k+1, i.e. (k + 1/2 -/+ sqrt(3)/6) h.
 * t_out: host, 2*M float64. */
fq_status fq_node_times(double T, int32_t M, double* t_out);

/* Three-point Gauss-Legendre sampling times for FQ_MAGNUS6: t_out[3k + j] =
 * (k + c_j) h with c = 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10.
 * t_out: host, 3*M float64. */
fq_status fq_node_times_magnus6(double T, int32_t M, double* t_out);

/* Expansion weights a_0 = J_0(R), a_l = 2 J_l(R), l = 1..L (Sec. 2, Eq. (12)),
 * by Miller's backward recurrence normalised with J_0 + 2 sum_k J_2k = 1.
 * R >= 0, L >= 0; out: host, L+1 float64. */
fq_status fq_bessel_weights(double R, int32_t L, double* out);

/* Smallest L >= 1 with 2 sum_{l > L} |J_l(R)| <= tol (R >= 0, tol > 0). */
fq_status fq_choose_order(double R, double tol, int32_t* L_out);

/* Extreme eigenvalues of the Hermitian tridiagonal matrix with diagonal d[n]
 * and off-diagonal moduli |e[i]| = e_abs[i] (n-1 values), by Sturm-sequence
 * bisection to full FP64 accuracy. Host pointers. */
fq_status fq_tridiag_extremes(int64_t n, const double* d, const double* e_abs,
                              double* lam_min, double* lam_max);

/* Outer estimate [lo, hi] of the spectrum of a dense Hermitian matrix, the
 * way the library bounds H0 and each Hmod for its dense spectral cover (the
 * paper's interval of Sec. 3, made to contain the spectrum): the extreme Ritz
 * values of 200 Lanczos steps, from a start vector drawn from a hash of
 * A (1, ..., 1), widened by 1 % of their spread on each side. For a start
 * uniform on the sphere an extreme Ritz value lies more than 1 % of the spread
 * inside the spectrum with probability below 1.648 sqrt(n) exp(-0.1 (2k - 1)),
 * k = min(n, 200) (Kuczynski and Wozniakowski, 1992): below 1e-14 for
 * n <= 10^6. a: host, n*n complex128 row-major (Hermitian, not checked);
 * lo, hi: host. Runs on the host. */
fq_status fq_hermitian_cover(int64_t n, const void* a, double* lo, double* hi);

/* Bytes of device workspace a context for (sys, par) needs (256-byte aligned
 * pointer expected). Checks the arguments like fq_create. */
fq_status fq_workspace_bytes(const fq_system* sys, const fq_params* par, size_t* bytes);

/* Create a context: validates, computes K (FQ_MAGNUS6: the nine nested
 * commutators), the spectral interval, R, L, the Bessel weights and the node
 * scalars (host FP64 except the commutators, which are formed on the device
 * with FP64 matrix products). The operator arrays of sys must stay valid and unchanged for
 * the life of the context. workspace: device, ws_bytes >= fq_workspace_bytes.
 * stream: a hipStream_t (NULL = default stream). */
fq_status fq_create(fq_ctx** out, const fq_system* sys, const fq_params* par,
                    void* workspace, size_t ws_bytes, void* stream);

fq_status fq_destroy(fq_ctx* ctx);

/* Replace the drive samples of a context (same layout as fq_params.f_nodes)
 * and redo what depends on them: the per-step weights of H_eff (Sec. 3),
 * the spectral interval (a caller's fixed interval is checked against the
 * new drive, FQ_ERR_SPECTRUM if it no longer contains it; a library interval
 * is recomputed, reusing the fixed operators' Lanczos extremes), beta, dE, R,
 * the order L unless fixed, the Bessel coefficients, the mixed-precision
 * schedule and the device step tables. The operators, commutators and the
 * workspace are kept, so a sequence of drives (an optimisation loop) costs no
 * setup beyond this. The gradient tape of the previous build is dropped
 * (floquet_grad then needs a new build). On any error the context refuses
 * builds, propagation and gradients (FQ_ERR_STATE) until a call succeeds. */
fq_status fq_set_drive(fq_ctx* ctx, const double* f_nodes);

/* Setup values (L, R, dE, beta, interval) and the last build's measurements. */
fq_status fq_get_report(const fq_ctx* ctx, fq_report* rep);

/* Build U_T = X_M from X_0 = identity (Sec. 3: the identity propagated over
 * one period). U_out: device, n*n complex (fq_params.dtype) row-major,
 * [i][j] = <i|U_T|j>.
 * rep (host, nullable) receives fq_get_report after the build, including the
 * FP64 unitarity measures of U_T. If checkpoint_every > 0 the tape for
 * floquet_grad is recorded. */
fq_status floquet_build_UT(fq_ctx* ctx, void* U_out, fq_report* rep);

/* Propagate ncols given states over steps k0+1 .. k1 (0 <= k0 <= k1 <= M):
 * X_out = E_k1 ... E_{k0+1} X0 (the second propagation round of Sec. 3, e.g.
 * Floquet states over one period, and its resumption from any step).
 * X0, X_out: device, n*ncols complex (fq_params.dtype), row-major (column c
 * is state c); they may alias. 1 <= ncols <= n. snapshots (device,
 * nullable): with snap_every >= 1, the states after steps k0 + j*snap_every,
 * j = 1 .. (k1 - k0) / snap_every, are written as n*ncols blocks of the same
 * dtype, block j-1 at snapshots + (j-1)*n*ncols elements; snap_every must be
 * 0 when snapshots is NULL. */
fq_status floquet_propagate(fq_ctx* ctx, const void* X0, int64_t ncols, int32_t k0, int32_t k1,
                            void* X_out, void* snapshots, int32_t snap_every);

/* Period average of the energy of ncols states (the second propagation round
 * of Sec. 3: Eq. (average) with A(t) = H(t), e.g. for the Floquet states
 * phi_mu(0), the eigenvectors of U_T, whose order by mean energy the paper
 * uses): with x_0 = column c of X0, x_k = E_k ... E_1 x_0 and t_k = k h,
 *     avg_out[c] = (1/M) sum_{k=0..M-1} <x_k| H0 + f_grid[k] Hmod |x_k> / <x_k|x_k>,
 * the rectangle rule on the step grid (for a Floquet state the integrand is
 * smooth and T-periodic, where it converges faster than any power of h).
 * X0: device, n*ncols complex (fq_params.dtype) row-major, 1 <= ncols <= n;
 * f_grid: host, M float64 (M x S with several drive terms), the drive at
 * t_k = k h (not at the quadrature nodes); avg_out: host, ncols float64. Steps use the context's scheme and
 * precision; the expectations are FP64. */
fq_status floquet_period_average(fq_ctx* ctx, const void* X0, int64_t ncols, const double* f_grid,
                                 double* avg_out);

/* Gradient of a real loss of U_T with respect to the 2*M drive samples (FQ_MAGNUS4), by
 * the reverse sweep through the Chebyshev recurrence of every step (beta, dE
 * and L held fixed), recomputing each segment from the tape of the last
 * floquet_build_UT. U_bar: device, n*n complex (fq_params.dtype) row-major with
 * U_bar[i][j] = dLoss/dRe U[i][j] + i dLoss/dIm U[i][j]. grad_f_nodes: host,
 * 2*M float64 (2*M*S with several drive terms), same order as f_nodes (with
 * fq_params.grad_pair_sums only each step's node sum is meaningful). Needs
 * checkpoint_every > 0. Dense layouts: every step of a checkpoint segment is
 * recomputed in FP64; the reverse products run in FP64, or, for FQ_FP32
 * contexts, on FP32 matrix cores (operands rounded to FP32 as they are
 * staged, FP64 epilogues and FP64 sums of the contractions: about FP32
 * accuracy in the derivative).
 * FQ_TRIDIAG: up to n = 2048 one workgroup reverses each state column;
 * longer columns run the same recurrences in streamed passes of K terms over
 * windows of rows with K ghost rows per side (K chosen per problem: at most
 * 256, at most 128 with the K contraction), one wave per real or imaginary
 * part (setting the environment variable FQ_TRIDIAG_STREAMED_ADJOINT=1 before
 * fq_workspace_bytes / fq_create selects the streamed form for any n; both
 * give the same derivative up to rounding). For n > 4096 the build records its
 * checkpoints in the state type (complex64 checkpoints round the recomputed
 * segments' starting states). In profile mode the report then holds the
 * streamed passes' times (FQ_K_ADJ_FWD: segment recompute, FQ_K_ADJ_REV:
 * reverse); with FQ_PROGRESS=1 in the environment the streamed sweep prints a
 * line on stderr per checkpoint segment. */
fq_status floquet_grad(fq_ctx* ctx, const void* U_bar, double* grad_f_nodes);

/* One-shot build of U_T that allocates nothing, for callers that cannot
 * allocate device memory (serving loops with a fixed memory budget, code that
 * must not call hipMalloc or a caching allocator). It does what fq_create,
 * floquet_build_UT and fq_destroy do in sequence, with the workspace taken
 * from a static device array of the library (256 MiB per GPU, held from the
 * first use on a device until the process ends) instead of caller memory;
 * it calls no hipMalloc or hipFree and creates no events. sys and par as for
 * fq_create, with checkpoint_every == 0 and profile == 0 (else
 * FQ_ERR_UNSUPPORTED); a problem whose fq_workspace_bytes exceeds 256 MiB is
 * rejected with FQ_ERR_ARG before any device work (dense Magnus-4 or
 * commutator-free: n up to 1408 in FP64 and 1280 in FP32 or split-BF16; the
 * tridiagonal chain: about 16 n^2 + 16 n M bytes, n up to about 3900).
 * stream: hipStream_t of the current device (NULL = default stream); U_out:
 * device, n*n complex (par->dtype) row-major, [i][j] = <i|U_T|j>; rep (host,
 * nullable) as for floquet_build_UT, with ms_build = 0. Returns after the
 * stream has drained. Every call on one GPU uses that GPU's single array
 * (each call clears what it needs): calls that overlap on one GPU, from
 * several host threads or on several streams, race and give wrong results. */
fq_status floquet_build_UT_static(const fq_system* sys, const fq_params* par, void* stream,
                                  void* U_out, fq_report* rep);

/* Thread-local description of the last non-OK status ("" if none). */
const char* fq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FLOQUET_H */
