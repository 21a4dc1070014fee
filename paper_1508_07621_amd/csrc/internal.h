// Internal declarations shared by the C-ABI driver and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/floquet.h"

namespace fq {

// ---- host numerics (host_numerics.cpp) ---------------------------------------------------
void gl2_node_times(double T, int M, double* t_out);
// Three-point Gauss-Legendre nodes t_{k-1} + (1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10) h.
void gl3_node_times(double T, int M, double* t_out);
void bessel_j_table(double x, int lmax, std::vector<double>& out);
int choose_order(double R, double tol);
void tridiag_extremes(long n, const double* d, const double* e_abs, double* lo, double* hi);

// ---- dense kernels (kernels_dense.hip) ---------------------------------------------------
// All dense working matrices are planar (separate real and imaginary float64
// planes), padded to np x np with zeros, row stride np. Column states are
// stored "state-major": row j of a plane holds state j (the transpose of the
// user's column layout), so every product is C(j, i) = sum_k A(j, k) B(i, k)
// with both operands contiguous along k.

// Epilogue kinds of the Chebyshev products (one launch = one term).
enum ChebKind : int {
  CHEB_FIRST = 0,       // P1 = acc; Y = c0 X + c1 P1
  CHEB_FIRST_LAST = 1,  // (L == 1) out = ph (c0 X + c1 acc)
  CHEB_MID = 2,         // P_{l+1} = 2 acc - P_{l-1}; Y += c P_{l+1}
  CHEB_LAST = 3         // P_L = 2 acc - P_{L-1}; out = ph (Y + c P_L)
};

struct ChebTerm {
  int kind;
  const double* a_re;  // A operand planes: P_l (state-major)
  const double* a_im;
  const double* b_re;  // B operand planes: rescaled H (row-major)
  const double* b_im;
  const double* p_re;  // previous term P_{l-1} (X for the first product)
  const double* p_im;
  double* y_re;        // Chebyshev sum
  double* y_im;
  double* o_re;        // output term or new X
  double* o_im;
  double c0r, c0i, cr, ci;  // coefficients (c0 only for the first product)
  double phr, phi;          // exp(-i beta h)
  double* save_re;          // optional: the last product also stores P_L here
  double* save_im;
};

// ---- adjoint products (kernels_dense.hip) ---------------------------------------------------
// Reverse term on a stack (rows [0, np) = P_l, [np, 2np) = Pbar_{l+1}) of mrows
// rows starting at A: P_{l-1} = 2 Ht P_l - P_{l+1} and
// Pbar_l = fac Ht Pbar_{l+1} - Pbar_{l+2} + d Lambda, in place over the output
// stack (P_{l+1} over Pbar_{l+2}); row_off = np when A holds only the adjoint half.
hipError_t launch_adj_step(const double* ar, const double* ai, int mrows, const double* htr,
                           const double* hti, double* sr, double* si, const double* lr,
                           const double* li, double dr, double di, double fac, int row_off, int np,
                           hipStream_t s);
// out[0] += w Re <Pbar, Hmod P>, out[1] += w Re <Pbar, K P> (ncols = 2np; np: Hmod only),
// with B = the planes [Hmod; K] stacked as 2np rows.
hipError_t launch_adj_dot(const double* pr, const double* pi, const double* dr, const double* di,
                          int ncols, const double* pbr, const double* pbi, double w, double* out,
                          int np, hipStream_t s);

// Whole chain of steps k0+1 .. k1 for np = 64 in one launch (FP64; Magnus-4 or
// commutator-free steps, one drive term): rows [0, mrows) of the state-major X
// planes (mrows a multiple of 16) are propagated in place, 16 states per
// workgroup, each forming every step's Ht in LDS from H0, V, K and a_k, b_k.
struct SmallChain {
  const double *h0r, *h0i, *vr, *vi, *kr, *ki;  // planar operators, row stride ld
  const double* ab;                            // device: a_k, b_k
  const double* coef;                          // device: c_l, complex interleaved
  double* xr;                                  // state-major X planes, in place
  double* xi;
  long ld;                                     // np (must be 64)
  int n, L, k0, k1;
  double beta, inv_dE, phr, phi;
};
long small_chain_max_n();
hipError_t launch_small_chain(const SmallChain& c, int mrows, hipStream_t s);

// The same two adjoint products on FP32 matrix cores (FQ_FP32 contexts): A in
// FP64 planes (re plane, im plane at + plane_a elements) rounded to FP32 while
// staged, B in FP32 planes (Ht in the FP32 product format; the drive block
// re planes then im planes at + plane_b), FP64 epilogues and contraction sums.
hipError_t launch_adj_step_f32(const double* ar, int mrows, long plane_a, const float* ht,
                               double* sr, double* si, const double* lr, const double* li, double dr,
                               double di, double fac, int row_off, int np, hipStream_t s);
hipError_t launch_adj_dot_f32(const double* pr, long plane_a, const float* drive, long plane_b,
                              int ncols, const double* pbr, const double* pbi, double w,
                              double* out, int np, hipStream_t s);
// dst[e] = (float)src[e], e < count.
hipError_t launch_f64_to_f32(const double* src, float* dst, long count, hipStream_t s);

// Launch one Chebyshev product over rows [0, mrows) of the state-major
// operands (mrows, np multiples of the tile size chosen by the launcher).
hipError_t launch_cheb_f64(const ChebTerm& t, int mrows, int np, hipStream_t s);

// ---- mixed-precision products (kernels_mixed.hip) ------------------------------------------
// Storage formats of a complex plane pair. F64 and F32: two planes (re, im).
// BF16X3: six k-blocked planes of 16-bit words (formats.h), the hi, mid and lo
// pieces of re and of im; hi + mid + lo carries about 24 significant bits. The
// product kernel forms the pieces of re + im (for three-product complex
// multiplication) while it stages a k-block into LDS, which holds nine planes.
enum Fmt : int { FMT_F64 = 0, FMT_F32 = 1, FMT_BF16X3 = 2 };
constexpr int BF3_PLANES = 6;
constexpr int BF3_LDS_PLANES = 9;

struct ChebTermX {
  int kind;
  int a_fmt, p_fmt, o_fmt;  // formats of A (P_l or X), P_{l-1} (or X), and the output
  long plane;               // elements per plane (np * np)
  const void* a;            // A planes (state-major)
  const void* b;            // B planes: rescaled H in the product format (F32 or BF16X3)
  const void* p;            // P_{l-1} (X for the first product)
  double* y_re;             // Chebyshev sum, F64
  double* y_im;
  void* o;                  // output planes
  double c0r, c0i, cr, ci, phr, phi;
};

// FP32 products P_{l+1} = 2 Ht P_l - P_{l-1} (l >= 1) with A = P_l in FP32
// (precision FQ_FP32; FP32 matrix cores).
hipError_t launch_cheb_mixed(const ChebTermX& t, int precision, int mrows, int np, hipStream_t s);

// Formats of the Chebyshev products of a mixed build, one per term,
// chosen on the host from the term's Bessel weight (fq_ctx::term_fmt):
// TF_F64: FP64 matrix cores on FP64 operands; TF_ACC: three BF16 pieces per
// operand with FP64 accumulation per k-block (about 24 bits independently of
// N); TF_X3 / TF_X2 / TF_X1: three / two / one BF16 pieces with FP32
// accumulation (about 24 bits less the accumulation error, 16 bits, 8 bits).
// FQ_FP32 builds use TF_F64 and TF_F32 (FP32 matrix cores, FP32 operands).
enum TermFmt : int { TF_F64 = 0, TF_ACC = 1, TF_X3 = 2, TF_X2 = 3, TF_X1 = 4, TF_F32 = 5 };

// Split-BF16 product of one term in term_fmt (TF_ACC .. TF_X1). A: BF16X3 (P_l,
// or X's BF16X3 copy for CHEB_FIRST / CHEB_FIRST_LAST); P_{l-1}: BF16X3 or FP64
// (X for the first product, for c_0 X); output BF16X3 (FIRST, MID) or FP64
// X_k (LAST, FIRST_LAST). mrows and np multiples of 64.
hipError_t launch_cheb_bf16(const ChebTermX& t, int term_fmt, int mrows, int np, hipStream_t s);
// FP64 planes (rows [0, mrows) of an np x np pair, row stride np) rounded into
// the product format `fmt` (FMT_F32 planar or FMT_BF16X3 k-blocked) at `out`.
// The first product of a mixed-precision step runs on FP64 matrix cores and
// its P_1 reaches the product format through this conversion.
hipError_t launch_to_product(const double* re, const double* im, void* out, int fmt, long mrows,
                             long np, hipStream_t s);
// Rescaled Hamiltonian, written both as FP64 planes (hr, hi) and in the
// product format of `precision` (out).
hipError_t launch_heff_mixed(const double* h0r, const double* h0i, const double* vr,
                             const double* vi, const double* kr, const double* ki, double a,
                             double b, double beta, double dE, long n, long ld, double* hr,
                             double* hi, void* out, int precision, hipStream_t s);

// C = alpha * (A op(B)^T) + beta * C with conjugation flags; planar fp64.
hipError_t launch_zgemm_nt_f64(const double* ar, const double* ai, bool conj_a, const double* br,
                               const double* bi, bool conj_b, double* cr, double* ci, int mrows,
                               int ncols, int kdim, int ld, double alr, double ali, double ber,
                               double bei, hipStream_t s);

// max |(A^H A - 1)_ij| (bit pattern, atomic max) and sum |.|^2 over an
// n x n Gram matrix of the first n state rows. out[0] = max (as double bits),
// out[1] = sum of squares; caller zeroes out first.
hipError_t launch_unitarity_f64(const double* xr, const double* xi, int n, int np,
                                double* out, hipStream_t s);

// Complex128 interleaved (rows x cols, row stride ld_src) -> planar planes (row stride ld).
hipError_t launch_pack_planar(const void* src, long rows, long cols, long ld_src, double* re,
                              double* im, long ld, hipStream_t s);
// Transposing pack: planes(j, i) = src(i, j) for i < rows, j < cols (src row stride ld_src);
// planes(j, i) = 0 elsewhere in [0, mrows) x [0, ld). src is complex64 when c64, else complex128.
hipError_t launch_pack_planar_t(const void* src, long rows, long cols, long ld_src, double* re,
                                double* im, long ld, long mrows, bool c64, hipStream_t s);
// Transposing unpack: dst(i, j) = planes(j, i) for i < rows, j < cols (dst row stride ld_dst),
// rounded to complex64 when c64.
hipError_t launch_unpack_planar_t(const double* re, const double* im, long ld, long rows,
                                  long cols, void* dst, long ld_dst, bool c64, hipStream_t s);
// Rows [0, m) x [0, ld) of the state-major planes set to the n x n identity (zero padding).
hipError_t launch_identity_rows(double* re, double* im, long n, long m, long ld, hipStream_t s);
// Rescaled Hamiltonian Ht = (H0 + a V + b K - beta 1) / dE on the n x n block.
hipError_t launch_heff_f64(const double* h0r, const double* h0i, const double* vr,
                           const double* vi, const double* kr, const double* ki, double a,
                           double b, double beta, double dE, long n, long ld, double* hr,
                           double* hi, hipStream_t s);
// dst = src^T for np x np planar pairs (dst must not alias src).
hipError_t launch_transpose_planar(const double* sr, const double* si, double* dr, double* di,
                                   long np, hipStream_t s);
// t = d * s elementwise on count planar complex elements.
hipError_t launch_scale_planar(const double* sr, const double* si, double dr, double di,
                               double* tr, double* ti, long count, hipStream_t s);
// y = A x for a dense complex128 row-major matrix (n x n) and vectors x, y (complex128).
hipError_t launch_zgemv(const void* A, long n, const void* x, void* y, hipStream_t s);
// y = A x for a planar (re, im) matrix with row stride ld; x, y interleaved complex, n rows.
hipError_t launch_zgemv_planar(const double* ar, const double* ai, long n, long ld, const void* x,
                               void* y, hipStream_t s);

// out = sum_j w_j M_j over planar matrices of `total` elements each (real weights).
constexpr int kMaxSumTerms = 16;
struct WeightedSum {
  const double* re[kMaxSumTerms];
  const double* im[kMaxSumTerms];
  double w[kMaxSumTerms];
  int count;
};
hipError_t launch_weighted_sum(const WeightedSum& ws, long total, double* outr, double* outi,
                               hipStream_t s);

// Energy expectations for the period average. Dense (state-major planes, row m
// = state m < rows, y = H x in the same layout): avg[m] += w Re<x_m, y_m> / |x_m|^2.
hipError_t launch_energy_rows(const double* xr, const double* xi, const double* yr,
                              const double* yi, long rows, long n, long ld, double w, double* avg,
                              hipStream_t s);
hipError_t launch_fill_zero(double* p, long count, hipStream_t s);
// H0 in its eigenbasis: diag(e) into zeroed planes; B = sgn i [diag(e), Q] elementwise.
hipError_t launch_diag_planar(const double* e, long n, long ld, double* re, hipStream_t s);
hipError_t launch_diag_commutator(const double* e, long n, long ld, const double* qr,
                                  const double* qi, double sgn, double* br, double* bi,
                                  hipStream_t s);
// Tridiagonal (user layout, complex128 or complex64 when c64), H = H0 + f Hmod:
// num[c] += Re<x_c, H x_c>, den[c] += |x_c|^2; finish: avg[c] += w num / den, num = den = 0.
hipError_t launch_tridiag_energy(const void* x, bool c64, long n, long ncols, const double* d,
                                 const void* off, const double* v, double f, double* num,
                                 double* den, hipStream_t s);
hipError_t launch_energy_finish(double* num, double* den, long ncols, double w, double* avg,
                                hipStream_t s);

// ---- tridiagonal kernels (kernels_tridiag.hip) --------------------------------------------
struct TridiagJob {
  long n;                // dimension
  long ncols;            // states propagated (one workgroup per state)
  const double* h0_diag; // device
  const double* h0_off;  // device, complex128 interleaved (n-1)
  const double* v_diag;  // device
  const double* ab;      // device, 2*M: a_k, b_k interleaved, for the steps in use
  const double* coef;    // device, 2*(L+1): c_l complex interleaved
  const double* gauge;   // device, M x n complex: w[s][i], D_s = diag(w[s]) makes D_s^+ Ht_s D_s real
  int L;
  int k0, k1;            // steps k0+1 .. k1
  double beta, inv_dE, phr, phi;
  const void* x0;        // device complex128 n x ncols row-major, or nullptr = identity
  long ld_x0;
  int x0_colmajor;       // streamed passes: x0 is complex128 column-major (col at col * n)
  void* x_out;           // device complex128 n x ncols row-major
  long ld_out;
  double* tape;          // optional (resident kernel): X_{j ckpt} as complex, slot j at
  int ckpt;              //   ((j * ncols + col) * n + i), written during the build
  double* snap;          // optional: X_{k0 + (j+1) snap_every}, complex n x ncols row-major
  int snap_every;        //   (block j at element j n ncols)
  int c64;               // x0, x_out and snap hold complex64 (else complex128)
};
// Returns hipErrorInvalidValue when n exceeds what one workgroup can hold.
hipError_t launch_tridiag_resident(const TridiagJob& job, hipStream_t s);
long tridiag_resident_max_n();

// Longer columns: one launch runs terms [l0, l1) of step s on blocks of B owned
// rows with K ghost rows per side (B + 2K = tridiag_stream_rows(G)), reading the
// state from `in` and writing it to `out` (8 planes of ncols x n16 doubles each),
// or, at the end of the last step (last_step and l1 == L + 1), X to job.x_out.
// first_step with l0 == 0 takes X from job.x0 (identity when null) instead of in.
// State planes between passes hold row i of a column at (i mod 16) nq + i / 16
// (nq = n16 / 16, n16 = n rounded up to 16), so that the 16 consecutive rows a
// lane owns are read and written with unit stride across the wave.
struct TridiagStream {
  const double* in;
  double* out;
  long plane;       // n16 * ncols
  long n16;         // rows per column in a state plane
  const double* stepc;  // per-step rows (same interleaved layout): 2 diag, 2 coupling,
                        // phase w_s (re, im), w_{s+1} (re, im); 6 n16 doubles
  int s;            // step index (0-based)
  int l0, l1;       // terms of this launch, l1 - l0 <= K, l0 != 1
  int first_step;
  int last_step;
  double* save;     // nullable: at the step's end, its last two terms P_{L-1}, P_L
                    // (4 planes [l & 1][part] in the state-plane layout)
  int K;            // ghost rows per side
  int G;            // waves per part: 1024 G rows per workgroup (the launcher takes G = 1)
  long B;           // owned rows per block
  long nblk;        // blocks per column = ceil(n / B)
};
long tridiag_stream_rows(int G);
hipError_t launch_tridiag_stream_step(const TridiagJob& job, const TridiagStream& st,
                                      double* stepc, hipStream_t s);

// Gradient of the tridiagonal chain, one workgroup per column (n <= 2048).
struct TridiagAdjJob {
  long n, ncols;
  const double* h0_diag;
  const double* h0_off;   // complex128 interleaved (n-1)
  const double* v_diag;
  const double* ab;       // a_k, b_k
  const double* coef;     // c_l complex interleaved
  int L, M, ckpt;
  int any_b;              // accumulate the K contraction
  double beta, inv_dE, phr, phi;
  const double* tape;     // X_{j ckpt} (forward build), complex, ((j * ncols + col) * n + i)
  const void* u_bar;      // Lambda_M, complex n x ncols row-major
  int c64;                // u_bar is complex64 (else complex128)
  double* seg;            // per column: ckpt x 3 complex vectors of n
  double* grad;           // 2 M accumulators: Re sum w_l <Pbar_{l+1}, D P_l>, D = Hmod, K
};
long tridiag_adjoint_max_n();
hipError_t launch_tridiag_adjoint(const TridiagAdjJob& job, hipStream_t s);

// One launch of the streamed reverse sweep for columns longer than one
// workgroup holds: terms l = hi .. lo of one step on the windows of the forward
// passes (B owned rows, K ghost rows per side, B + 2K = tridiag_stream_rows(1);
// both multiples of 16), in the gauge frame of the step. Vectors are planes of
// ncols x n16 doubles in the interleaved row layout of TridiagStream.
constexpr int kAdjSlots = 64;  // accumulator slots per step (workgroup b adds to b mod 64)
struct TridiagAdjStream {
  long n, ncols, n16, plane;  // plane = n16 * ncols (doubles)
  int K;
  long B, nblk;
  int L, lo, hi;              // hi - lo + 1 <= K, hi <= L - 1
  const double* coef;         // c_l complex interleaved
  double phr, phi;            // exp(-i beta h)
  // table inputs (launch_tridiag_adj_table)
  const double* h0_diag;
  const double* h0_off;       // complex interleaved (n-1)
  const double* v_diag;
  const double* gauge;        // M x n complex: w_k
  double a, b, beta, inv_dE;  // step scalars
  // pass state
  const double* lam;          // 2 planes (re, im): Lambda before the table's factor (after it: persistent pass)
  const double* seg;          // hi == L-1: P_{L-1}, P_L of the step (4 planes [l & 1][part])
  const double* in;           // hi < L-1: 8 planes [role][part]: P_l, P_{l+1}, Pbar_{l+1}, Pbar_{l+2}
  double* out;                // lo > 0: the same for the next launch (terms from lo - 1)
  double* lam_out;            // lo == 0: Pbar_0 in the step's gauge frame (2 planes)
  double* grad;               // the step's 2 x kAdjSlots accumulators: (V, K) per slot
};
// Per-step tables (7 n16 doubles): 2d, 2g, v, Lambda factor (re, im), K~ (re, im);
// plain_lambda: the step reads U_bar (factor conj(w_k)), else Pbar_0 of step k+1.
hipError_t launch_tridiag_adj_table(const TridiagAdjStream& p, int k, bool plain_lambda,
                                    double* tab, hipStream_t s);
// U_bar (n x ncols row-major, complex64 when c64) into two planes.
hipError_t launch_tridiag_lam_pack(const void* ubar, bool c64, long n, long ncols, long n16,
                                   double* out, hipStream_t s);
hipError_t launch_tridiag_adj_stream(const TridiagAdjStream& p, const double* tab, bool with_k,
                                     hipStream_t s);
// Lambda' = f Lambda in place (both planes), f the table's Lambda factor.
hipError_t launch_tridiag_lam_gauge(const TridiagAdjStream& p, const double* tab, double* lam,
                                    hipStream_t s);
// The reverse pass without the K contraction in its persistent form; p.lam
// holds Lambda' (launch_tridiag_lam_gauge), not Lambda.
hipError_t launch_tridiag_adj_persist(const TridiagAdjStream& p, const double* tab,
                                      hipStream_t s);
hipError_t launch_tridiag_stream(const TridiagJob& job, const TridiagStream& st, hipStream_t s);

// Unit gauge factors of step s (host FP64): w_0 = 1, w_{i+1} = w_i conj(u_i) with
// u_i = e_i / |e_i| the phase of Ht[i][i+1] (u_i = 1 where e_i = 0).
void tridiag_gauge(long n, const double* h0_off, const double* v_diag, double b, double* w_out);

}  // namespace fq
