#!/usr/bin/env python3
"""Seconds per Floquet-operator build on one MI355X, with the dominant kernel's
roofline fraction and the FP64 CPU oracle timed beside it.

A "step" is one complete build of U_T from the identity over one period: every
per-step Hamiltonian, every Chebyshev product, the phase hand-off, the chain of
M steps, and the FP64 unitarity check of the result. Inputs (operators, drive
samples) are resident in HBM before the timed region; setup (commutator,
spectral interval, coefficients) is done once before it.

    python bench.py [--steps K] [--warmup W] [--workload gue4096|dimer1000|gue64|gue4096m6|...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X datasheet peaks used for the roofline fractions.
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP64_VECTOR_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

#: algorithmic real flops per element and Chebyshev term of the tridiagonal
#: pass: two complex-by-complex couplings (6 each), a real diagonal (2), two
#: complex adds (4), 2 t - P_{l-1} (4) and the Bessel-weighted accumulation (4).
TRIDIAG_FLOPS_PER_ELEMENT_TERM = 26

#: longest column the library keeps resident in one workgroup; longer ones run
#: as streamed passes with ghost rows
TRIDIAG_RESIDENT_MAX_N = 4096

#: algorithmic real flops per element and term of the streamed reverse pass in
#: the gauge frame (real couplings): Pbar_l = w G Pbar_{l+1} - Pbar_{l+2} + d_l Lambda
#: (G on a complex value 12, scale and subtract 4, complex source 8),
#: P_{l-1} = 2 G P_l - P_{l+1} (16) and the contraction w v_i Re(conj(Pbar) P) (6)
TRIDIAG_ADJ_REV_FLOPS_PER_ELEMENT_TERM = 46

WORKLOAD_TEXT = {
    "gue4096": "random-matrix model N=4096 (GUE H0, V), f=cos t, T=2pi, M=200 Magnus-4 steps, "
               "Chebyshev order for 1e-12 per step",
    "dimer1000": "Bose-Hubbard dimer, 999 bosons (N=1000, tridiagonal), J=1, U=0.01, "
                 "eps=0.5+1.5cos t, T=2pi, M=500",
    "gue64": "random-matrix model N=64 (GUE H0, V), f=cos t, T=2pi, M=100",
    "adjoint1024": "adjoint: random-matrix model N=1024, piecewise-constant f_j ~ U(-1,1), M=256, "
                   "loss 1-|Tr(W^dagger U)|^2/N^2 with Haar W, checkpoint every 16 steps; "
                   "step = forward build + gradient",
    "dimer10000": "Bose-Hubbard dimer, 9999 bosons (N=10^4, tridiagonal), params as dimer1000, M=500",
    "gue10000": "random-matrix model N=10^4 (GUE H0, V), f=cos t, T=2pi, M=200",
    "gue4096m6": "random-matrix model N=4096 as gue4096 with the paper's sixth-order Magnus "
                 "scheme (Eq. (14), three Gauss-Legendre nodes), M=50 steps",
    "adjointdimer10000": "adjoint: Bose-Hubbard dimer, 9999 bosons (N=10^4, tridiagonal, J=1, "
                         "U=0.01), piecewise-constant f_j ~ U(-1,1) on V = n1 - n2, T=2pi, M=256, "
                         "loss 1-|Tr(W^dagger U)|^2/N^2 with W = U_T of the drive f_j + 0.02 u_j, "
                         "checkpoint every 16 steps; step = forward build + gradient",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gue4096", choices=sorted(WORKLOAD_TEXT),
                    help="gue4096 (default), dimer1000, gue64, adjoint1024 (build + gradient), "
                         "dimer10000, gue10000 (minutes per build), gue4096m6 (sixth-order scheme)")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the dense Chebyshev products (default: bf16x3, fp64 for "
                         "gue64; the tridiagonal path is FP64)")
    ap.add_argument("--no-small-chain", action="store_true",
                    help="N <= 64: time the launch-per-product form instead of the one-launch chain")
    ap.add_argument("--no-fp64-ref", action="store_true",
                    help="skip the FP64 reference build of a mixed-precision run")
    ap.add_argument("--no-eig", action="store_true", help="skip the host eigenphase comparison")
    ap.add_argument("--eig", action="store_true",
                    help="also time the host eigenphases of U_T when there is no FP64 reference "
                         "build to compare with (FP64 and tridiagonal runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scheme", choices=["magnus4", "magnus6", "cf4"], default=None,
                    help="step operator (default: the workload's)")
    ap.add_argument("--M", type=int, default=0, help="steps per period (default: the workload's)")
    ap.add_argument("--time-error-ref", default="", metavar="SCHEME:M",
                    help="also build an FP64 reference with this scheme and step count and report "
                         "the time-discretisation error e_col of the timed result against it")
    ap.add_argument("--second-round", action="store_true",
                    help="after the timed builds, diagonalise U_T on the host and time the second "
                         "propagation round (period-averaged energies of all Floquet states)")
    ap.add_argument("--fd-check", type=float, default=0.0, metavar="EPS",
                    help="gradient workloads: also compare the gradient along a seeded direction "
                         "with a central difference of step EPS (two more builds)")
    ap.add_argument("--shard", type=int, default=0, metavar="P",
                    help="also time one GPU's share of a P-GPU column split: the first N/P "
                         "columns of the identity propagated over the period (Sec. 5), against "
                         "1/P of the full build")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run one device-to-device copy of BYTES bytes (the reference "
                         "kernel for scaling HBM traffic counters) and exit")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--oracle-cols", type=int, default=-1, metavar="C",
                    help="columns on which the FP64 oracle follows all M steps as the reference "
                         "of errors.vs_oracle (default 4 for N <= 4096, 0 = off above)")
    ap.add_argument("--mixed-tol", type=float, default=0.0,
                    help="split-BF16: error target from which each term's product format is "
                         "chosen (0 = the library's default)")
    ap.add_argument("--fp64-builds", type=int, default=3,
                    help="timed FP64 reference builds (after one warm-up); their median is reported")
    return ap.parse_args()


def cpu_baseline(wl, f_nodes, target_s: float):
    """The FP64 oracle on a bounded sample of the same workload, scaled to one
    full build: columns are independent and every step costs the same, so the
    cost is linear in both (the paper extrapolates in M the same way)."""
    import numpy as np

    import oracle as orc
    t_cpu0 = time.time()
    h = wl.T / wl.M
    a, b = orc.magnus4_weights(f_nodes, h)
    # Untimed setup, as on the GPU side: the fixed operators and the coefficients.
    if wl.layout == "dense":
        ncols = 64
        H0, V = wl.arrays["h0"], wl.arrays["v"]
        K = orc.commutator(H0, V)
        lo, hi = -4.5, 4.5       # any cover of the spectrum; the cost does not depend on it
        heff = lambda k: orc.magnus4_heff(H0, V, K, a[k], b[k])  # noqa: E731
    else:
        ncols = 8
        d, e, v = wl.arrays["h0_diag"], wl.arrays["h0_off"], wl.arrays["v_diag"]
        H0, V, K = orc.tridiag_matrices(d, e, v)
        lo, hi = orc.tridiag_cover(d, e, v, a, b)
        heff = lambda k: (H0 + a[k] * V + b[k] * K).tocsr()  # noqa: E731
    beta, dE, R = orc.rescale(lo, hi, h)
    coef = orc.bessel_coefficients(R, orc.choose_L(R, 1e-12))
    X = np.eye(wl.n, dtype=np.complex128)[:, :ncols]
    # Timed: per step, the operator build (independent of the number of columns)
    # and the Chebyshev step on ncols columns (linear in the number of columns).
    t_op = t_step = 0.0
    steps = 0
    while steps < wl.M and (steps < 1 or t_op + t_step < target_s):
        t0 = time.perf_counter()
        Hk = heff(steps)
        t1 = time.perf_counter()
        X = orc.chebyshev_step(Hk, beta, dE, h, coef, X)
        t2 = time.perf_counter()
        t_op += t1 - t0
        t_step += t2 - t1
        steps += 1
    scaled = wl.M * (t_op / steps + (t_step / steps) * (wl.n / ncols))
    dt = t_op + t_step
    sample = (f"{steps} of {wl.M} steps on {ncols} of {wl.n} columns; per-step operator time "
              f"x M plus per-step Chebyshev time x M x N/{ncols}")
    cores = _blas_threads()
    return {"value": scaled, "unit": "s/build", "cores": cores, "kind": "oracle",
            "sample": sample, "sample_seconds": round(dt, 3),
            "wall_seconds": round(time.time() - t_cpu0, 1)}


def oracle_columns(wl, kw, f_nodes, info, ncols: int):
    """The FP64 oracle (Chebyshev route, the build's interval and order) on
    `ncols` seeded columns of the identity over all M steps: the reference
    for the error of each GPU result on those columns."""
    import numpy as np

    import oracle as orc
    rng = np.random.default_rng(1508 + 99)
    cols = np.sort(rng.choice(wl.n, ncols, replace=False))
    X0 = np.eye(wl.n, dtype=np.complex128)[:, cols]
    common = dict(route="cheb", e_min=info["e_min"], e_max=info["e_max"], L=info["L"], X0=X0,
                  scheme=wl.scheme)
    t0 = time.perf_counter()
    if wl.layout == "dense":
        Xref = orc.build_ut(kw["h0"], kw["hmod"], f_nodes, wl.T, wl.M, **common)
    else:
        Xref = orc.build_ut_tridiag(kw["h0_diag"], kw["h0_off"], kw["hmod_diag"], f_nodes, wl.T,
                                    wl.M, **common)
    return cols, Xref, time.perf_counter() - t0


def _log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _blas_threads() -> int:
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        n = [i.get("num_threads") for i in info if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return len(os.sched_getaffinity(0))


#: MFMA operations issued per algorithmic real flop of a complex product
#: (algorithmic: four real products, 8 N^3 flop): FP32 runs the four real
#: products once; FP64 on 128 x 128 tiles runs three (Gauss), 3 / 4, and four on
#: 64 x 64 tiles; BF16x3 runs three real products (Gauss) for each of six piece
#: pairs, 18 / 4 = 4.5.
MFMA_FLOPS_PER_FLOP = {"fp64": 0.75, "fp32": 1.0, "bf16x3": 4.5}

#: products of at least this many output elements use 128 x 128 tiles
BIG_TILE_ELEMS = 256 * 128 * 128


def mfma_flops_per_flop(precision: str, n: int, rows: int = 0) -> float:
    """MFMA flops per algorithmic flop of a product with (rows or n) x n outputs."""
    if precision == "fp64" and (rows or n) * n < BIG_TILE_ELEMS:
        return 1.0
    return MFMA_FLOPS_PER_FLOP[precision]
PEAKS = {"fp64": PEAK_FP64_MFMA_TFLOPS, "fp32": PEAK_FP32_MFMA_TFLOPS,
         "bf16x3": PEAK_BF16_MFMA_TFLOPS}
KERNEL_NAMES = {"fp64": "zgemm_nt_f64_kernel<128,128,8,2,4,Gauss,EpiCheb<MID>> (FP64 MFMA 16x16x4, "
                        "3 real products)",
                "fp32": "cheb_f32_kernel<128,128,32,2,4,EpiMix<MID>> (FP32 MFMA 16x16x4)",
                "bf16x3": "cheb_bf3_kernel<128,128,2,4,MID> (BF16 MFMA 32x32x16, 3 real products "
                          "x 6 piece pairs)"}

def kernel_name(precision: str, n: int) -> str:
    """The middle product's kernel: 128 x 128 tiles, or 64 x 64 below BIG_TILE_ELEMS outputs."""
    if n * n >= BIG_TILE_ELEMS:
        return KERNEL_NAMES[precision]
    return {"fp64": "zgemm_nt_f64_kernel<64,64,16,2,2,EpiCheb<MID>> (FP64 MFMA 16x16x4)",
            "fp32": "cheb_f32_kernel<64,64,32,2,2,EpiMix<MID>> (FP32 MFMA 16x16x4)",
            "bf16x3": "cheb_bf3_kernel<64,64,2,2,MID> (BF16 MFMA 32x32x16, 3 real products "
                      "x 6 piece pairs)"}[precision]


#: Kernel sources behind each roofline entry; HBM traffic recorded under
#: profiles/ is reported only while these files are unchanged.
TRAFFIC_SOURCES = {
    "fp64": ["kernels_dense.hip", "formats.h", "internal.h"],
    "fp32": ["kernels_mixed.hip", "formats.h", "internal.h"],
    "bf16x3": ["kernels_mixed.hip", "formats.h", "internal.h"],
    "bf16x3_f64acc": ["kernels_mixed.hip", "formats.h", "internal.h"],
    "bf16x2": ["kernels_mixed.hip", "formats.h", "internal.h"],
    "bf16x1": ["kernels_mixed.hip", "formats.h", "internal.h"],
    "tridiag": ["kernels_tridiag.hip", "internal.h"],
}
TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "hbm_traffic.md")


def source_digest(key: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES[key]:
        with open(os.path.join(ROOT, "paper_1508_07621_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(key: str, workload: str):
    """HBM bytes per launch of the dominant kernel from the rocprofv3 counter
    table (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration), or None
    when there is no row for this kernel and workload or its sources changed."""
    try:
        lines = open(TRAFFIC_TABLE).read().splitlines()
    except OSError:
        return None
    digest = source_digest(key)
    for line in lines:
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == key and cells[1] == workload and cells[2] == digest:
            fetch, write = float(cells[3]), float(cells[4])
            return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
                    "source_digest": digest}
    return None


def time_builds(ctx, U, warmup: int, steps: int, tag: str, walls=None):
    """W untimed builds, then K builds timed between device synchronisations
    (every build returns after its stream has drained: the unitarity check
    reads its result on the host). `walls` (a list) receives each build's wall
    time."""
    import torch
    for i in range(warmup):
        ctx.build_ut(out=U)
        _log(f"{tag} warmup build {i + 1}/{warmup}: {ctx.last_report['ms_build']:.1f} ms")
    torch.cuda.synchronize()
    reports = []
    t0 = time.perf_counter()
    for i in range(steps):
        t1 = time.perf_counter()
        ctx.build_ut(out=U)
        if walls is not None:
            walls.append(time.perf_counter() - t1)
        reports.append(ctx.last_report)
        _log(f"{tag} timed build {i + 1}/{steps}: {reports[-1]['ms_build']:.1f} ms")
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, reports


def time_build_grad(ctx, U, W, warmup: int, steps: int):
    """Forward build with the gradient tape, then the reverse sweep for the loss
    1 - |Tr(W^dagger U)|^2 / N^2 (U_bar formed on the device); K timed pairs."""
    import torch
    n = U.shape[0]

    def one():
        ctx.build_ut(out=U)
        tau = torch.sum(torch.conj(W) * U)
        ubar = (-2.0 / n ** 2) * tau * W
        t0 = time.perf_counter()
        g = ctx.grad(ubar)
        return time.perf_counter() - t0, g, tau.item()

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    reports, grad_reports, gsum = [], [], 0.0
    t0 = time.perf_counter()
    for i in range(steps):
        dt, g, tau = one()
        gsum += dt
        reports.append(ctx.last_report)
        grad_reports.append(ctx.report)
        _log(f"build+grad {i + 1}/{steps}: build {reports[-1]['ms_build']:.1f} ms, "
             f"gradient {1e3 * dt:.1f} ms")
    torch.cuda.synchronize()
    return ((time.perf_counter() - t0) / steps, reports, 1e3 * gsum / steps, grad_reports, g,
            1.0 - abs(tau) ** 2 / n ** 2)


def fd_direction(wl, kw, f, g, W, eps: float):
    """Directional check of the gradient: (L(f + eps d) - L(f - eps d)) / (2 eps)
    against g . d for a seeded unit direction d over the amplitudes, with two
    more builds of the library."""
    import numpy as np
    import torch
    from paper_1508_07621_amd import floquet as fl
    n = W.shape[0]
    d = np.random.default_rng(1508 + 77).standard_normal(f.size)
    d /= np.linalg.norm(d)
    vals = []
    for sgn in (+1, -1):
        ff = f + sgn * eps * d
        c = fl.FloquetContext(T=wl.T, M=wl.M, f_nodes=np.stack([ff, ff], 1), device=W.device, **kw)
        Uf = c.build_ut()
        tau = torch.sum(torch.conj(W) * Uf).item()
        vals.append(1.0 - abs(tau) ** 2 / n ** 2)
        del c, Uf
    fd = (vals[0] - vals[1]) / (2 * eps)
    ad = float(np.dot(g, d))
    return {"direction": "seeded unit vector over the amplitudes", "eps": eps, "adjoint": ad,
            "finite_difference": fd, "rel_diff": abs(ad - fd) / max(abs(fd), 1e-300)}


ALGO_NOTE = ("algorithmic flops: 8 N^3 per complex N x N x N product (four real products); the "
             "FP64 kernel on 128 x 128 tiles forms each complex product from Gauss's three real "
             "products (6 N^3 MFMA flops), so its algorithmic rate can exceed the FP64 MFMA peak; "
             "split-BF16 issues three real products per kept piece pair")


def dense_roofline(reports, n: int, precision: str, workload: str):
    """The middle Chebyshev product: achieved = algorithmic flops (8 N^3) per
    launch over the launch time, against the MFMA peak of the precision the
    product runs in; the MFMA flops actually issued are reported beside it."""
    from paper_1508_07621_amd._abi import K_MID
    n_launch = sum(r["n_kernel"][K_MID] for r in reports)
    ms_launch = sum(r["ms_kernel"][K_MID] for r in reports) / max(n_launch, 1)
    flops = 8.0 * n ** 3                                   # one complex N x N x N product
    mfma_flops = flops * mfma_flops_per_flop(precision, n)
    achieved = flops / (ms_launch * 1e-3) / 1e12
    issued = mfma_flops / (ms_launch * 1e-3) / 1e12
    peak = PEAKS[precision]
    tr = recorded_traffic(precision, workload)
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": tr["bytes"] if tr else None,
            "traffic_detail": tr, "kernel": kernel_name(precision, n),
            "avg_launch_ms": round(ms_launch, 4), "launches_timed": n_launch,
            "algorithmic_flops_per_launch": flops, "note": ALGO_NOTE,
            "issued_mfma": {"flops_per_launch": mfma_flops, "achieved": round(issued, 3),
                            "frac": round(issued / peak, 4)}}


#: split-BF16 builds: profile kinds of the products by term format
TERM_KINDS = {8: "fp64", 9: "bf16x3_f64acc", 10: "bf16x3", 11: "bf16x2", 12: "bf16x1"}
#: MFMA flops issued per algorithmic flop (8 N^3 per complex product) of each format:
#: FP64 Gauss (3 of 4 real products); FP64-accumulating split-BF16: four real products
#: x six piece pairs / 4; split-BF16 with FP32 sums: Gauss x 6, 3 or 1 piece pairs / 4
#: (64 x 64 output tiles; on 128 x 128 tiles the one- and two-piece products run the
#: four real products, TERM_MFMA_X4)
TERM_MFMA = {"fp64": 0.75, "bf16x3_f64acc": 6.0, "bf16x3": 4.5, "bf16x2": 2.25, "bf16x1": 0.75}
TERM_MFMA_X4 = {"bf16x2": 3.0, "bf16x1": 1.0}
TERM_KERNEL_X4 = {
    "bf16x2": "cheb_x4_kernel<KIND,P,2> (BF16 MFMA 32x32x16 on 64 x 64 wave tiles, 4 real "
              "products x 3 piece pairs)",
    "bf16x1": "cheb_x4_kernel<KIND,P,1> (BF16 MFMA 32x32x16 on 64 x 64 wave tiles, 4 real "
              "products x 1 piece pair)",
}


def x4_tiles(n: int) -> bool:
    """Whether the split-BF16 products of an n-state build run on 128 x 128 output
    tiles (states padded to 128 from n = 1024 on, to 64 below), where the one- and
    two-piece products use cheb_x4_kernel."""
    t = 128 if n >= 1024 else 64
    npad = (n + t - 1) // t * t
    return npad % 128 == 0 and npad * npad >= BIG_TILE_ELEMS


def term_mfma(name: str, n: int) -> float:
    if name == "fp64":
        return mfma_flops_per_flop("fp64", n)
    if name in TERM_MFMA_X4 and x4_tiles(n):
        return TERM_MFMA_X4[name]
    return TERM_MFMA[name]


def term_kernel(name: str, n: int) -> str:
    if name in TERM_KERNEL_X4 and x4_tiles(n):
        return TERM_KERNEL_X4[name]
    return TERM_KERNEL[name]


TERM_KERNEL = {
    "fp64": "zgemm_nt_f64_kernel<128,128,8,2,4,Gauss,EpiCheb> (FP64 MFMA 16x16x4)",
    "bf16x3_f64acc": "cheb_acc_kernel<128> (BF16 MFMA 32x32x16, 4 real products x 6 piece "
                     "pairs, FP64 sums per 64-column block)",
    "bf16x3": "cheb_bf3_kernel<128,128,2,4,KIND,P,3> (BF16 MFMA 32x32x16, 3 real products x 6 "
              "piece pairs)",
    "bf16x2": "cheb_bf3_kernel<128,128,2,4,KIND,P,2> (3 real products x 3 piece pairs)",
    "bf16x1": "cheb_bf3_kernel<128,128,2,4,KIND,P,1> (3 real products x 1 piece pair)",
}


def term_schedule(reports, n: int, workload: str):
    """Per term format of a split-BF16 build: launches per build, average
    launch time, share of the build, algorithmic and issued MFMA rates; and
    the roofline entry of the format that takes the most time."""
    rows = {}
    for k, name in TERM_KINDS.items():
        cnt = sum(r["n_kernel"][k] for r in reports)
        if not cnt:
            continue
        ms = sum(r["ms_kernel"][k] for r in reports)
        avg = ms / cnt
        flops = 8.0 * n ** 3
        peak = PEAK_FP64_MFMA_TFLOPS if name == "fp64" else PEAK_BF16_MFMA_TFLOPS
        mf = flops * term_mfma(name, n)
        rows[name] = {"launches_per_build": cnt / len(reports), "avg_launch_ms": round(avg, 4),
                      "ms_per_build": round(ms / len(reports), 2),
                      "algorithmic_tflops": round(flops / (avg * 1e-3) / 1e12, 2),
                      "frac": round(flops / (avg * 1e-3) / 1e12 / peak, 4),
                      "issued_mfma_frac": round(mf / (avg * 1e-3) / 1e12 / peak, 4)}
    if not rows:
        return None, None
    dom = max(rows, key=lambda k: rows[k]["ms_per_build"])
    r = rows[dom]
    flops = 8.0 * n ** 3
    peak = PEAK_FP64_MFMA_TFLOPS if dom == "fp64" else PEAK_BF16_MFMA_TFLOPS
    mf = flops * term_mfma(dom, n)
    avg = r["avg_launch_ms"]
    tr = recorded_traffic(dom, workload)
    roof = {"bound": "mfma", "achieved": r["algorithmic_tflops"], "peak": peak,
            "unit": "TFLOP/s", "frac": r["frac"], "traffic": tr["bytes"] if tr else None,
            "traffic_detail": tr, "kernel": term_kernel(dom, n),
            "term_format": dom, "avg_launch_ms": avg,
            "launches_timed": int(round(r["launches_per_build"] * len(reports))),
            "algorithmic_flops_per_launch": flops, "note": ALGO_NOTE,
            "issued_mfma": {"flops_per_launch": mf, "achieved": round(mf / (avg * 1e-3) / 1e12, 3),
                            "frac": round(mf / (avg * 1e-3) / 1e12 / peak, 4)}}
    return rows, roof


def chain_roofline(reports, n: int, M: int, terms_per_step: int):
    """The one-launch chain of N <= 64 FP64 builds: every step's products in
    one kernel on N/16 workgroups (one per 16 states), so the launch's
    algorithmic work is M x (terms per step) x 8 N^3 over the chain's time; it
    uses N/16 of the 256 compute units, so its fraction of the FP64 peak is
    bounded by (N/16)/256 by construction."""
    from paper_1508_07621_amd._abi import K_CHAIN
    cnt = sum(r["n_kernel"][K_CHAIN] for r in reports)
    ms = sum(r["ms_kernel"][K_CHAIN] for r in reports) / cnt
    flops = float(M) * terms_per_step * 8.0 * n ** 3
    ach = flops / (ms * 1e-3) / 1e12
    cus = max(n // 16, 1)
    return {"bound": "mfma", "achieved": round(ach, 4), "peak": PEAK_FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_MFMA_TFLOPS, 5), "traffic": None,
            "traffic_detail": None,
            "kernel": "small_chain_kernel (whole build in one launch, 16 states per workgroup, "
                      "FP64 MFMA 16x16x4)",
            "avg_launch_ms": round(ms, 4), "launches_timed": cnt,
            "algorithmic_flops_per_launch": flops,
            "compute_units_used": cus,
            "frac_of_used_units": round(ach / (PEAK_FP64_MFMA_TFLOPS * cus / 256), 4)}


def dense_reverse_roofline(grad_reports, n: int, L: int, M: int, precision: str = "fp64"):
    """The dense gradient's reverse-sweep products (FP64, or FP32 matrix cores
    for FP32 contexts): per step, L launches of Ht times the stacked
    [P_l; Pbar_{l+1}] (2n rows) for l >= 2 and of Ht times Pbar (n rows) for
    l = 1, 0."""
    from paper_1508_07621_amd._abi import K_ADJ_REV
    n_rev = sum(r["n_kernel"][K_ADJ_REV] for r in grad_reports)
    if not n_rev:
        return None
    ms = sum(r["ms_kernel"][K_ADJ_REV] for r in grad_reports) / n_rev
    rows = (2 * max(L - 2, 0) + (1 if L >= 2 else 0) + 1) * n   # rows per step, all launches
    flops = 8.0 * rows * n * n * M * len(grad_reports) / n_rev  # per launch, averaged
    f32 = precision == "fp32"
    mf = flops * (1.0 if f32 else mfma_flops_per_flop("fp64", n, 2 * n))
    peak = PEAK_FP32_MFMA_TFLOPS if f32 else PEAK_FP64_MFMA_TFLOPS
    ach = flops / (ms * 1e-3) / 1e12
    issued = mf / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": None,
            "traffic_detail": None,
            "kernel": ("cheb_f32_kernel<..., EpiAdjStep> (FP32 MFMA 16x16x4" if f32 else
                       "zgemm_nt_f64_kernel + EpiAdjStep (FP64 MFMA 16x16x4") +
                      "; reverse sweep: Ht times [P_l; Pbar_{l+1}])",
            "avg_launch_ms": round(ms, 4), "launches_timed": n_rev,
            "algorithmic_flops_per_launch": flops, "note": ALGO_NOTE,
            "issued_mfma": {"flops_per_launch": mf, "achieved": round(issued, 3),
                            "frac": round(issued / peak, 4)}}


def time_error(U, wl, kw, spec: str):
    """e_col of U against an FP64 build of the same problem with another scheme
    and step count (a converged reference isolates the time discretisation)."""
    import torch
    from paper_1508_07621_amd import floquet as fl
    from workloads import drive_cos
    scheme, m = spec.split(":")
    m = int(m)
    eps0, eps1 = (0.5, 1.5) if wl.layout == "tridiag" else (0.0, 1.0)
    f = drive_cos(fl.node_times(wl.T, m, scheme=scheme), eps0, eps1, 1.0)
    _log(f"time-discretisation reference: {scheme}, M = {m}, FP64")
    ref = fl.FloquetContext(T=wl.T, M=m, f_nodes=f, tol=1e-12, precision="fp64", scheme=scheme,
                            device=U.device, **kw)
    R = ref.build_ut()
    return {"reference": f"FP64 {scheme} build with M = {m}",
            "e_col": torch.linalg.vector_norm(U - R, dim=0).max().item()}


def second_round(ctx, U, wl, kw):
    """The paper's post-processing of a build: host eigenvectors of U_T, then one
    more period of propagation of all N Floquet states on the device with their
    period-averaged energies (timed), sorted by mean energy. Full-size check:
    the mean energies of a complete orthonormal set sum to the grid mean of
    Tr H(t_k) = Tr H0 + f(t_k) Tr Hmod."""
    import numpy as np
    import torch
    eps0, eps1 = (0.5, 1.5) if wl.layout == "tridiag" else (0.0, 1.0)
    fg = eps0 + eps1 * np.cos(np.arange(wl.M) * wl.T / wl.M)
    _log("second round: host eigendecomposition and device period averages")
    t0 = time.perf_counter()
    lam, phi = np.linalg.eig(U.cpu().numpy())
    eig_s = time.perf_counter() - t0
    phi = phi / np.linalg.norm(phi, axis=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_mean = ctx.period_average(phi, fg)
    torch.cuda.synchronize()
    round_s = time.perf_counter() - t0
    if wl.layout == "dense":
        tr0, trv = np.trace(kw["h0"]).real, np.trace(kw["hmod"]).real
    else:
        tr0, trv = float(np.sum(kw["h0_diag"])), float(np.sum(kw["hmod_diag"]))
    expect = tr0 + float(np.mean(fg)) * trv
    # the paper's per-state accuracy (Sec. 7, Eq. (error)): every Floquet state
    # of U_T(h) against the best-matching one of a companion build at h/2
    from paper_1508_07621_amd import analysis
    from paper_1508_07621_amd import floquet as fl
    from workloads import drive_cos
    _log("second round: companion build at h/2 and per-state errors")
    f2 = drive_cos(fl.node_times(wl.T, 2 * wl.M, scheme=wl.scheme), eps0, eps1, 1.0)
    ctx2 = fl.FloquetContext(T=wl.T, M=2 * wl.M, f_nodes=f2, tol=1e-12,
                             precision=ctx.precision, scheme=wl.scheme, device=U.device, **kw)
    t0 = time.perf_counter()
    U2 = ctx2.build_ut()
    torch.cuda.synchronize()
    half_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    sigma, dq, _ = analysis.state_errors_of_builds(U, U2, wl.T)
    err_s = time.perf_counter() - t0
    del ctx2, U2
    return {"s_period_average": round(round_s, 4), "host_eig_vectors_s": round(eig_s, 1),
            "states": int(phi.shape[1]), "mean_energy_range": [float(e_mean.min()),
                                                                float(e_mean.max())],
            "trace_check": {"sum_mean_energies": float(e_mean.sum()), "expected": expect,
                            "abs_diff": abs(float(e_mean.sum()) - expect)},
            "state_errors": {"reference": "companion build at h/2 (M = %d), host eigenvectors of "
                                          "both, best-matching state" % (2 * wl.M),
                             "overlap_deficiency_max": float(sigma.max()),
                             "overlap_deficiency_median": float(np.median(sigma)),
                             "quasienergy_diff_max": float(dq.max()),
                             "quasienergy_diff_median": float(np.median(dq)),
                             "s_half_step_build": round(half_s, 3),
                             "host_s": round(err_s, 1)}}


def shard_share(ctx, U, wl, P: int, warmup: int, steps: int, s_full: float, precision: str):
    """One GPU's share of the column split over P GPUs (Sec. 5, Fig. 2): the
    first N/P identity columns propagated over the whole period with the same
    context, timed like the builds. Each GPU of the split would run exactly
    this (its own columns, no communication inside the period); the result must
    equal those columns of the full build."""
    import torch
    from paper_1508_07621_amd._abi import K_MID, K_TRIDIAG
    n = U.shape[0]
    if P < 2 or n % P:
        raise SystemExit(f"--shard {P}: P must be >= 2 and divide N = {n}")
    cols = n // P
    X0 = torch.eye(n, dtype=U.dtype, device=U.device)[:, :cols].contiguous()
    out = torch.empty_like(X0)
    for _ in range(warmup):
        ctx.propagate(X0, 0, wl.M, out=out)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.propagate(X0, 0, wl.M, out=out)
        reps.append(ctx.report)
        _log(f"shard 1/{P} timed propagation {i + 1}/{steps}")
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    kind = K_MID if wl.layout == "dense" else K_TRIDIAG
    n_launch = sum(r["n_kernel"][kind] for r in reps)
    ms_launch = sum(r["ms_kernel"][kind] for r in reps) / max(n_launch, 1)
    res = {"P": P, "columns": cols, "s_per_share": round(t, 6),
           "ideal_s": round(s_full / P, 6), "efficiency_vs_full_build": round(s_full / P / t, 4),
           "max_abs_vs_full_build": (out - U[:, :cols]).abs().max().item(),
           "dominant_kernel_avg_ms": round(ms_launch, 4)}
    if wl.layout == "dense":
        flops = 8.0 * n * n * cols
        mf = flops * mfma_flops_per_flop(precision, n, cols)
        res["dominant_kernel_mfma_frac"] = round(mf / (ms_launch * 1e-3) / 1e12 / PEAKS[precision], 4)
    return res


def host_eigenphases(U):
    """Host FP64 eigenphases: LAPACK zgeev through NumPy (the paper's routine)
    up to N = 4096, the Hermitian Cayley route above (zgeev takes minutes at
    N = 10^4). Returns (phases, method)."""
    from paper_1508_07621_amd.analysis import eigenphases, eigenphases_unitary
    if U.shape[0] <= 4096:
        return eigenphases(U), "zgeev"
    return eigenphases_unitary(U), "zheevd of the Cayley transform"


def eigen_errors(U, Uref, T: float):
    """Host FP64 eigenphases of both results and the largest quasienergy
    difference (symmetric circular matching)."""
    import numpy as np
    t0 = time.perf_counter()
    th, _ = host_eigenphases(U)
    _log("host eigenphases of the first result done")
    th_ref, _ = host_eigenphases(Uref)

    def one_way(x, y):
        ext = np.concatenate([y - 2 * math.pi, y, y + 2 * math.pi])
        idx = np.searchsorted(ext, x)
        lo = np.clip(idx - 1, 0, len(ext) - 1)
        hi = np.clip(idx, 0, len(ext) - 1)
        return float(np.max(np.minimum(np.abs(x - ext[lo]), np.abs(x - ext[hi]))))

    d = max(one_way(th, th_ref), one_way(th_ref, th)) / T
    return d, time.perf_counter() - t0


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: measures one GPU only (got --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); the column-sharded multi-GPU layout is a design note, "
              "not an implemented path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1508_07621_amd import floquet as fl
    from paper_1508_07621_amd._abi import K_TRIDIAG
    from workloads import drive_cos, workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy}), flush=True)
        return
    wl = workload(args.workload, M=args.M or None)
    if args.scheme:
        wl.scheme = args.scheme
    if args.precision is None:  # the 64-state configuration is the plain FP64 build
        args.precision = "fp64" if args.workload == "gue64" else "bf16x3"
    if args.no_small_chain:
        os.environ["FQ_SMALL_CHAIN"] = "0"
    precision = args.precision if wl.layout == "dense" else "fp64"
    grad_mode = wl.amplitudes is not None
    if grad_mode:
        f_nodes = np.stack([wl.amplitudes, wl.amplitudes], 1)
        if (wl.layout == "dense" and args.precision == "bf16x3"
                and "--precision" not in sys.argv):
            precision = "fp32"  # the configuration's complex64 forward
    elif wl.layout == "tridiag":
        f_nodes = drive_cos(fl.node_times(wl.T, wl.M, scheme=wl.scheme), 0.5, 1.5, 1.0)
    else:
        f_nodes = drive_cos(fl.node_times(wl.T, wl.M, scheme=wl.scheme), 0.0, 1.0, 1.0)
    if wl.layout == "dense":
        kw = dict(h0=wl.arrays["h0"], hmod=wl.arrays["v"])
    else:
        kw = dict(h0_diag=wl.arrays["h0_diag"], h0_off=wl.arrays["h0_off"],
                  hmod_diag=wl.arrays["v_diag"])

    t_setup = time.perf_counter()
    c64_grad = grad_mode and wl.layout == "dense"   # the dense adjoint configuration's complex64
    interval = {}
    if grad_mode and args.fd_check > 0:
        # room around the library's interval for the perturbed drives of the
        # check, which then use the same interval and order (the gradient holds
        # beta, dE and L fixed)
        probe = fl.FloquetContext(T=wl.T, M=wl.M, f_nodes=f_nodes, tol=1e-12, device=dev,
                                  scheme=wl.scheme, **kw).report
        margin = 1.0 + 1e-3 * (probe["e_max"] - probe["e_min"])
        interval = dict(e_min=probe["e_min"] - margin, e_max=probe["e_max"] + margin)
    ctx = fl.FloquetContext(T=wl.T, M=wl.M, f_nodes=f_nodes, tol=1e-12, precision=precision,
                            mixed_tol=args.mixed_tol if precision != "fp64" else 0.0,
                            profile=True, device=dev, checkpoint_every=16 if grad_mode else 0,
                            dtype="complex64" if c64_grad else "complex128",
                            grad_pair_sums=grad_mode,   # gradient w.r.t. step amplitudes
                            scheme=wl.scheme, **interval, **kw)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    info = ctx.report
    _log(f"setup {setup_s:.2f} s: L={info['L']} R={info['R']:.4f} "
         f"interval=[{info['e_min']:.6g}, {info['e_max']:.6g}]")
    n = wl.n
    U = torch.empty((n, n), dtype=ctx.state_dtype, device=dev)
    if grad_mode:
        if "w" in wl.arrays:
            W = torch.from_numpy(wl.arrays["w"]).to(device=dev, dtype=ctx.state_dtype)
        else:  # the target gate: U_T of the nearby drive (untimed)
            ft = wl.arrays["f_target"]
            _log("target U_T of the nearby drive")
            tctx = fl.FloquetContext(T=wl.T, M=wl.M, f_nodes=np.stack([ft, ft], 1), tol=1e-12,
                                     device=dev, **kw)
            W = tctx.build_ut()
            del tctx
        s_per_build, reports, grad_ms, grad_reports, g_last, loss = time_build_grad(
            ctx, U, W, args.warmup, args.steps)
    else:
        s_per_build, reports = time_builds(ctx, U, args.warmup, args.steps, precision)
    last = reports[-1]
    errors = {"unitarity_max": last["unitarity_max"], "unitarity_fro": last["unitarity_fro"]}
    Uref = None

    extra = {}
    if grad_mode:
        extra["gradient"] = {"ms_per_grad": round(grad_ms, 3),
                             "ms_per_build": round(1e3 * s_per_build - grad_ms, 3),
                             "loss": loss, "max_abs_grad": float(np.max(np.abs(g_last))),
                             "note": ("value = forward build (FP32 products, tape every 16 steps) "
                                      "+ reverse sweep for the 256 amplitudes (segments "
                                      "recomputed in FP64, reverse products on FP32 matrix "
                                      "cores); U_T and U_bar stored in complex64; "
                                      "node-pair sums only (the commutator contraction, "
                                      "which cancels in them, skipped)")
                                     if wl.layout == "dense" else
                                     ("value = forward build (streamed passes, checkpoints every "
                                      "16 steps) + streamed FP64 reverse sweep for the 256 "
                                      "amplitudes (node-pair sums only)")}
        if args.fd_check > 0:
            _log("directional finite-difference check of the gradient")
            fkw = {k: v for k, v in kw.items()}
            fkw.update(e_min=info["e_min"], e_max=info["e_max"], L=info["L"])
            extra["gradient"]["fd_direction"] = fd_direction(wl, fkw, wl.amplitudes,
                                                             g_last.sum(axis=1), W, args.fd_check)
    if wl.layout == "dense":
        from paper_1508_07621_amd._abi import K_CHAIN
        if sum(r["n_kernel"][K_CHAIN] for r in reports):
            roof = chain_roofline(reports, n, wl.M, info["L"] * (2 if wl.scheme == "cf4" else 1))
        elif precision == "bf16x3":
            rows, roof = term_schedule(reports, n, args.workload)
            from paper_1508_07621_amd._abi import TERM_FORMAT_NAMES
            extra["schedule"] = {
                "term_formats": [TERM_FORMAT_NAMES[f] for f in last["term_format"] if f >= 0],
                "mixed_err_est": last["mixed_err_est"], "per_format": rows}
        else:
            roof = dense_roofline(reports, n, precision, args.workload)
        build_tflops = info["L"] * wl.M * 8.0 * n ** 3 / s_per_build / 1e12
        if grad_mode:
            rev = dense_reverse_roofline(grad_reports, n, info["L"], wl.M, precision)
            if rev:  # build + gradient: the FP64 reverse-sweep products dominate
                extra["build_roofline"] = roof
                roof = rev
        if precision != "fp64" and not args.no_fp64_ref and not grad_mode:
            # The FP64 build of the same workload: reference result and timing.
            ref = fl.FloquetContext(T=wl.T, M=wl.M, f_nodes=f_nodes, tol=1e-12, precision="fp64",
                                    e_min=info["e_min"], e_max=info["e_max"], L=info["L"],
                                    profile=True, device=dev, scheme=wl.scheme, **kw)
            Uref = torch.empty_like(U)
            walls = []
            _, rep_ref = time_builds(ref, Uref, 1, max(args.fp64_builds, 1), "fp64", walls)
            s_ref = float(np.median(walls))
            D = U - Uref
            errors.update({
                "reference": "FP64 build of the same workload on the GPU (same interval and L)",
                "e_col": torch.linalg.vector_norm(D, dim=0).max().item(),
                "fro_over_sqrtN": torch.linalg.vector_norm(D).item() / math.sqrt(n),
                "max_abs": D.abs().max().item(),
                "ref_unitarity_max": rep_ref[-1]["unitarity_max"],
            })
            if not args.no_eig:
                _log("host FP64 eigenphases of both results")
                dq, eig_s = eigen_errors(U.cpu().numpy(), Uref.cpu().numpy(), wl.T)
                errors["max_quasienergy_error"] = dq
                extra["eig_seconds_host"] = round(eig_s, 1)
                extra["eig_method"] = ("zgeev" if n <= 4096 else
                                       "zheevd of the Cayley transform")
            extra["fp64"] = {"s_per_build": round(s_ref, 4),
                             "timing": f"median of {len(walls)} builds after one warm-up",
                             "s_per_build_each": [round(w, 4) for w in walls],
                             "build_tflops_algorithmic": round(
                                 info["L"] * wl.M * 8.0 * n ** 3 / s_ref / 1e12, 3),
                             "build_tflops_note": ALGO_NOTE,
                             "roofline": dense_roofline(rep_ref, n, "fp64", args.workload)}
            extra["speedup_vs_fp64"] = round(s_ref / s_per_build, 3)
            del ref
    else:
        n_launch = sum(r["n_kernel"][K_TRIDIAG] for r in reports)
        ms_launch = sum(r["ms_kernel"][K_TRIDIAG] for r in reports) / max(n_launch, 1)
        per_build = max(n_launch // max(len(reports), 1), 1)  # launches per build
        # algorithmic work of one launch: the build's total over its launches
        flops = float(TRIDIAG_FLOPS_PER_ELEMENT_TERM) * n * n * wl.M * info["L"] / per_build
        achieved = flops / (ms_launch * 1e-3) / 1e12
        tr = recorded_traffic("tridiag", args.workload)
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4),
                "traffic": tr["bytes"] if tr else None, "traffic_detail": tr,
                "kernel": ("tridiag_gauge_kernel<16,512> (whole chain per state column, real gauge form)"
                           if n <= TRIDIAG_RESIDENT_MAX_N else
                           "tridiag_stream_kernel<16,1> (128-term passes; 768 owned + 2 x 128 ghost "
                           "rows per workgroup, real gauge form)"),
                "avg_launch_ms": round(ms_launch, 4), "launches_timed": n_launch,
                "algorithmic_flops_per_launch": flops}
        build_tflops = flops * per_build / s_per_build / 1e12
        if grad_mode:
            # build + gradient: the streamed reverse pass dominates
            from paper_1508_07621_amd._abi import K_ADJ_FWD, K_ADJ_REV
            n_rev = sum(r["n_kernel"][K_ADJ_REV] for r in grad_reports)
            ms_rev = sum(r["ms_kernel"][K_ADJ_REV] for r in grad_reports) / max(n_rev, 1)
            n_fwd = sum(r["n_kernel"][K_ADJ_FWD] for r in grad_reports)
            ms_fwd = sum(r["ms_kernel"][K_ADJ_FWD] for r in grad_reports) / max(n_fwd, 1)
            if n_rev:
                per_grad = n_rev / len(grad_reports)
                flops_rev = (float(TRIDIAG_ADJ_REV_FLOPS_PER_ELEMENT_TERM) * n * n * wl.M
                             * info["L"] / per_grad)
                ach = flops_rev / (ms_rev * 1e-3) / 1e12
                extra["build_roofline"] = roof
                roof = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_VECTOR_TFLOPS, 4),
                        "traffic": None, "traffic_detail": None,
                        "kernel": (("tridiag_adj_persist_kernel<HI_ODD> (persistent reverse "
                                    "passes of up to 128 terms, two workgroups per CU walking "
                                    "the (window, column) items, the next item's state loaded "
                                    "into LDS during the terms; " if ctx.grad_pair_sums else
                                    "tridiag_adj_stream_kernel<true, HI_ODD> (reverse passes of "
                                    "up to 128 terms with the K contraction; ")
                                   + "768 owned + 2 x 128 ghost rows per item, one wave per real "
                                   "or imaginary part, real gauge frame)"),
                        "avg_launch_ms": round(ms_rev, 4), "launches_timed": n_rev,
                        "algorithmic_flops_per_launch": flops_rev}
                extra["gradient"]["segment_recompute_pass"] = {
                    "kernel": "tridiag_stream_kernel<16,1> (the forward pass, saving each step's "
                              "last two terms)", "avg_launch_ms": round(ms_fwd, 4),
                    "launches_timed": n_fwd}

    ocols = args.oracle_cols if args.oracle_cols >= 0 else (4 if n <= 4096 else 0)
    if ocols > 0 and not grad_mode:
        _log(f"FP64 oracle on {ocols} columns over all {wl.M} steps")
        cols, Xref, o_s = oracle_columns(wl, kw, f_nodes, info, ocols)

        def ecol(Ud):
            return float(np.max(np.linalg.norm(Ud[:, cols].cpu().numpy() - Xref, axis=0)))

        vs = {"reference": "FP64 oracle, Chebyshev route with the build's interval and L, on "
                           "seeded columns of the identity over all M steps",
              "columns": cols.tolist(), "oracle_s": round(o_s, 1), "e_col": ecol(U)}
        if Uref is not None:
            vs["fp64_e_col"] = ecol(Uref)
        errors["vs_oracle"] = vs
    del Uref
    if args.eig and not grad_mode and "eig_seconds_host" not in extra:
        # the paper's routine diagonalisation of U_T (Sec. 3, Sec. 5), timed on the host
        _log("host FP64 eigenphases of U_T")
        t0 = time.perf_counter()
        th, method = host_eigenphases(U.cpu().numpy())
        extra["eigenphases"] = {"host_s": round(time.perf_counter() - t0, 1), "method": method,
                                "quasienergy_range": [float(th.min() / wl.T),
                                                      float(th.max() / wl.T)],
                                "count": int(th.size)}
    if args.shard and not grad_mode:
        extra["shard"] = shard_share(ctx, U, wl, args.shard, args.warmup, args.steps,
                                     s_per_build, precision)
    if args.second_round and not grad_mode:
        extra["second_round"] = second_round(ctx, U, wl, kw)
    if args.time_error_ref and not grad_mode:
        extra["time_discretisation"] = time_error(U, wl, kw, args.time_error_ref)

    out = {
        "metric": "s per U_T build + TFLOP/s (% MFMA/HBM peak), mixed vs FP64 at stated error",
        "value": round(s_per_build, 6),
        "unit": "s/build",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * s_per_build, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[precision],
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "name": args.workload, "n": n,
                   "M": wl.M, "L": info["L"], "R": round(info["R"], 6),
                   "interval": [info["e_min"], info["e_max"]], "precision": precision,
                   "scheme": wl.scheme, "parallelism": "1 GPU"},
        "build_tflops_algorithmic": round(build_tflops, 3),
        "build_tflops_note": ALGO_NOTE if wl.layout == "dense" else
                             "algorithmic flops per element and term of the tridiagonal pass",
        "errors": errors,
        "setup_s": round(setup_s, 3),
        "roofline": roof,
    }
    out.update(extra)
    if (not args.no_cpu_baseline and not grad_mode and wl.n <= 10000
            and wl.scheme == "magnus4"):
        _log("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(wl, f_nodes, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
