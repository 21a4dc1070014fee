// The library context (fq_ctx): host-side state of one problem, used by the
// C-ABI driver only. The kernels see the launch structures of internal.h.
#pragma once

#include "internal.h"

// ---- the context ---------------------------------------------------------------------------
struct fq_ctx {
  // system
  int64_t n = 0;
  int layout = 0;
  fq_system sys{};
  // params
  double T = 0, h = 0, tol = 0;
  int M = 0, L = 0, precision = 0, ckpt = 0;
  std::vector<double> f_nodes, a, b;  // host
  // scheme: 0 = Magnus-4 (H0 + a V + b K); 1 = the sixth-order scheme, whose
  // H_eff,k = H0 + a_k V + sum_j w6[k][j] B_j over nine fixed Hermitian nested
  // commutators B_j (device planes comm6, 2 planes each); a_k as above, b_k = 1
  // for the K slot, which then holds each step's sum over the B_j.
  int scheme = 0;
  // FQ_CF4 runs every step as spp = 2 half-steps: M, h and ckpt above count
  // those; M_user is the caller's step count (API indices are scaled by spp).
  int spp = 1, M_user = 0;
  // dense model given in H0's eigenbasis (sys.h0_diag = E_i): H0 planes hold
  // diag(E), and commutators with H0 are taken elementwise
  bool h0_eigen = false;
  // drive terms: S matrices Hmod_s; the drive block holds J planar matrices B_j
  // (re planes of all J, then im planes): one term -> [Hmod, K]; S >= 2 ->
  // [Hmod_s..., and for FQ_MAGNUS4 K_s = -i [H0, Hmod_s]..., K_st = -i [Hmod_s, Hmod_t]
  // (s < t)]; wS (M x J) are the per-(sub)step weights of the B_j when S >= 2.
  int S = 1, J = 2;
  bool pair_sums = false;             // floquet_grad: node-pair sums only (no K contraction)
  // the parameters the drive-dependent setup needs again on fq_set_drive
  double mixed_tol = 0.0;
  std::vector<int> term_formats;      // caller's term formats (empty: the library's schedule)
  bool interval_given = false;        // the caller fixed [e_min, e_max]
  double e_min_given = 0.0, e_max_given = 0.0;
  int L_given = 0;                    // the caller fixed L (> 0)
  bool drive_ok = true;               // false after a failed fq_set_drive
  // Ritz extremes of the fixed operators (H0, Hmod, ...), by operator pointer
  std::vector<std::pair<const void*, std::pair<double, double>>> ritz_cache;
  std::vector<double> wS;
  std::vector<double> w6;             // M x 9
  double* comm6 = nullptr;
  double e_min = 0, e_max = 0, beta = 0, dE = 0, R = 0;
  std::vector<double> weights;        // a_l = (2 - delta_l0) J_l(R), l = 0..L
  std::vector<double> coef;           // c_l = (2 - delta_l0) (-i)^l J_l(R), interleaved
  double phr = 1, phi = 0;            // exp(-i beta h)
  // device
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  long np = 0;                        // padded dimension (dense)
  // dense planes
  double *h0r = nullptr, *h0i = nullptr, *vr = nullptr, *vi = nullptr, *kr = nullptr, *ki = nullptr;
  double *htr = nullptr, *hti = nullptr;
  double *xr = nullptr, *xi = nullptr, *yr = nullptr, *yi = nullptr;
  double *par = nullptr, *pai = nullptr, *pbr = nullptr, *pbi = nullptr;
  void* htx = nullptr;                // mixed builds: rescaled H in the product format
  double* pcr = nullptr;              // mixed builds: a third P buffer (format changes)
  std::vector<int> term_fmt;          // mixed builds: TermFmt of terms 1..L (index 0 unused)
  double mixed_err_est = 0.0;         // the schedule's estimate of the error it adds to U_T
  double* tape = nullptr;             // checkpoints, each 2 planes
  int n_tape = 0;
  // gradient: per segment step X_{k-1}, P_{L-1}, P_L; two stacks; Lambda; d/da, d/db per step
  double* seg = nullptr;
  double* stack[2] = {nullptr, nullptr};
  double* lam = nullptr;
  double* d_grad = nullptr;
  float* drive32 = nullptr;           // FQ_FP32 gradient: the drive block in FP32 planes
  bool adj_f32 = false;               // reverse-sweep products on FP32 matrix cores
  double* save_pl = nullptr;          // when set, a step also stores P_L and P_{L-1} here
  double* save_plm1 = nullptr;
  double* small = nullptr;            // 64 doubles of reduction scratch
  double* d_ab = nullptr;             // 2*M
  double* d_coef = nullptr;           // 2*(L+1)
  double* d_gauge = nullptr;          // tridiagonal: M x n complex gauge factors
  double* d_stream = nullptr;         // tridiagonal n > resident size: two 8-plane states
  double* d_adj = nullptr;            // streamed reverse sweep: 10 complex n x n vectors
  double* d_vec = nullptr;            // 3 n doubles: period-average accumulators
  // state
  bool tape_valid = false;
  bool broken = false;
  fq_report last{};
  // profile mode: one event before every launch of a build (and one after the
  // last); launch i took the time between events i and i+1.
  bool profile = false;
  bool reortho = false;               // polar factor of U_T after the build
  bool small_chain = true;            // np = 64 FP64 steps in one launch (small_chain_kernel)
  bool c64 = false;                   // user state blocks (U, X, W, snapshots) in complex64
  void* snap = nullptr;               // propagate: snapshot buffer, every snap_every steps
  int snap_every = 0, snap_k0 = 0;
  long snap_ncols = 0;
  std::vector<hipEvent_t> events;
  std::vector<int> event_kind;
  size_t n_events = 0;
  // device time of a whole build (ms_build); off for the allocation-free
  // one-shot build, which creates no events
  bool timed = true;
  hipEvent_t build_ev[2] = {nullptr, nullptr};
  ~fq_ctx() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipEvent_t e : build_ev)
      if (e) (void)hipEventDestroy(e);
  }
};
