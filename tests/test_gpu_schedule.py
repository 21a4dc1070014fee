"""Split-BF16 builds with every per-term product format, and mixes of them,
against the FP64 oracle (same interval and order).

Each term l of a step can run in its own format (FP64, three BF16 pieces with
FP64 accumulation, three / two / one BF16 pieces with FP32 accumulation); its
rounding error enters the step's sum with weight |c_l| = 2|J_l(R)|. The bar of
each case is ten times the worst-case (linear in the steps) sum of
|c_l| eps(format_l) over terms and steps, with eps the format's relative
precision: a kernel that mishandles a tile, a piece or a buffer is off by O(1).
The leading FP64 run exercises the step's buffer hand-over from FP64 planes to
the BF16 format at every position."""
import math

import numpy as np
import pytest

import oracle as orc
from workloads import drive_cos, gue

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi
U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def fl(require_gpu):
    from paper_1508_07621_amd import floquet
    floquet.node_times(1.0, 1)          # loads the library or raises
    return floquet


def _say(*a):
    print("[case]", *a, flush=True)


def _eps(fmt, nk):
    return {"fp64": 1e-15, "bf16x3_f64acc": 4 * U24, "bf16x3": (2 + math.sqrt(nk)) * U24,
            "bf16x2": 2.0 ** -15, "bf16x1": 2.0 ** -7}[fmt]


def _case(n, M, seed, T=TWO_PI):
    rng = np.random.default_rng(seed)
    H0, V = gue(n, rng), gue(n, rng)
    f = drive_cos(orc.node_times(T, M), 0.0, 1.0, 1.0)
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = orc.weyl_cover(H0, V, orc.commutator(H0, V), a, b)
    return H0, V, f, lo, hi


SCHEDULES = [
    ["fp64"],
    ["bf16x3_f64acc"],
    ["bf16x3"],
    ["bf16x2"],
    ["bf16x1"],
    ["fp64", "bf16x3"],
    ["fp64", "fp64", "bf16x3"],
    ["fp64", "fp64", "fp64", "bf16x2"],
    ["fp64", "fp64", "fp64", "fp64", "bf16x3_f64acc"],
    ["bf16x3_f64acc", "bf16x3", "bf16x2", "bf16x1"],
    ["fp64", "bf16x3_f64acc", "bf16x1"],
]


@pytest.mark.parametrize("n", [96, 1030])
@pytest.mark.parametrize("L", [1, 2, 3, 5])
@pytest.mark.parametrize("sched", SCHEDULES, ids=["-".join(s) for s in SCHEDULES])
def test_forced_schedule_matches_oracle(fl, n, L, sched):
    M = 4 if n > 500 else 6
    T = 0.3 * L       # keeps the truncation of order L moderate
    _say("schedule", sched, "n", n, "L", L)
    H0, V, f, lo, hi = _case(n, M, 100 + L, T)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            precision="bf16x3", term_formats=sched)
    U = ctx.build_ut().cpu().numpy()
    rep = ctx.last_report
    full = [sched[min(l, len(sched)) - 1] for l in range(1, L + 1)]
    from paper_1508_07621_amd._abi import TERM_FORMATS
    assert rep["term_format"][:L] == [TERM_FORMATS[x] for x in full]
    cols = list(range(n)) if n <= 300 else [0, 517, n - 1]
    X0 = np.eye(n, dtype=complex)[:, cols]
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0)
    _, _, R = orc.rescale(lo, hi, T / M)
    w = np.abs(orc.bessel_coefficients(R, L))
    nk = (n + 63) // 64 * 4 if n < 1024 else (n + 127) // 128 * 8
    bound = 10.0 * M * sum(w[l] * _eps(full[l - 1], nk) for l in range(1, L + 1)) + 1e-11
    err = orc.column_error(U[:, cols], Uref)
    _say("e_col", err, "bound", bound)
    assert err < bound


def test_auto_schedule_orders_formats_by_weight(fl):
    """The library's choice: terms with larger Bessel weight never get a
    cheaper format than terms with smaller weight, the estimate it reports is
    within the target, and a looser target never chooses costlier formats."""
    n, M = 512, 40
    H0, V, f, lo, hi = _case(n, M, 5)
    reps = {}
    for tol in (1e-9, 1e-7, 1e-5):
        ctx = fl.FloquetContext(h0=H0, hmod=V, T=TWO_PI, M=M, f_nodes=f, e_min=lo, e_max=hi,
                                tol=1e-12, precision="bf16x3", mixed_tol=tol)
        rep = ctx.report
        L = rep["L"]
        tf = rep["term_format"][:L]
        _say("mixed_tol", tol, "L", L, "formats", tf, "estimate", rep["mixed_err_est"])
        w = np.abs(orc.bessel_coefficients(rep["R"], L))[1:]
        order = np.argsort(-w)
        # cost rank: fp64 0 > acc 1 > x3 2 > x2 3 > x1 4 (larger value = cheaper)
        assert all(tf[order[i]] <= tf[order[i + 1]] or w[order[i]] == w[order[i + 1]]
                   for i in range(L - 1))
        assert rep["mixed_err_est"] <= tol
        reps[tol] = tf
    assert all(a <= b for a, b in zip(reps[1e-9], reps[1e-7]))
    assert all(a <= b for a, b in zip(reps[1e-7], reps[1e-5]))


LARGE_SCHEDULES = [["bf16x1"], ["bf16x2"], ["bf16x3_f64acc", "bf16x2", "bf16x1"],
                   ["fp64", "bf16x1"]]


@pytest.mark.parametrize("L", [1, 2, 3, 5])
@pytest.mark.parametrize("sched", LARGE_SCHEDULES, ids=["-".join(s) for s in LARGE_SCHEDULES])
def test_forced_schedule_large_tiles(fl, L, sched):
    """n = 2049 (17 x 17 tiles of 128): the split-BF16 products take their
    128 x 128 tiles, the FP64-sum product its 128-row tiles."""
    test_forced_schedule_matches_oracle(fl, 2049, L, sched)
