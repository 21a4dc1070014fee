"""Parity of the sixth-order Magnus scheme (the paper's Eq. (14)) on the GPU with
the FP64 oracle, through the C ABI.

The oracle forms each step's Omega by dense matrix arithmetic exactly as the
equation is written; the library expands it once into nine nested commutators
with per-step real weights. Both sides get the same drive samples, spectral
interval and Chebyshev order, so their difference is rounding only.
"""
import math

import numpy as np
import pytest

import oracle as orc
from workloads import drive_cos, gue

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi
FP64_TOL = 1e-10
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def fl(require_gpu):
    from paper_1508_07621_amd import floquet
    floquet.node_times(1.0, 1)          # loads the library or raises
    return floquet


def _say(*a):
    print("[case]", *a, flush=True)


def _case(n, seed):
    rng = np.random.default_rng(seed)
    return gue(n, rng), gue(n, rng)


def _nodes6(T, M, eps0=0.0, eps1=1.0):
    return drive_cos(orc.node_times6(T, M), eps0, eps1, 1.0)


def _oracle_interval(H0, V, f, T, M, tol=1e-12):
    h = T / M
    lo, hi = orc.exact_cover([orc.magnus6_heff(H0, V, f[k], h) for k in range(M)])
    return lo, hi, orc.choose_L(orc.rescale(lo, hi, h)[2], tol)


@pytest.mark.parametrize("n,M,seed", [(64, 40, 1508), (100, 12, 2), (200, 6, 3), (1030, 2, 4),
                                      (1, 3, 7), (65, 1, 10), (2049, 1, 11)])
def test_magnus6_fp64_matches_oracle(fl, n, M, seed):
    """Partial tiles (1, 65), ragged multi-tile sizes (100, 200, 1030) and a size
    on 128-row tiles (2049); M = 1 is a single step."""
    _say("magnus6 fp64", n, M, seed)
    H0, V = _case(n, seed)
    T = TWO_PI
    f = _nodes6(T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            scheme="magnus6")
    U = ctx.build_ut().cpu().numpy()
    rep = ctx.last_report
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, scheme="magnus6")
    err = orc.column_error(U, Uref)
    _say("e_col", err, "L", rep["L"], "unitarity", rep["unitarity_max"])
    assert rep["L"] == L
    assert err < FP64_TOL


@pytest.mark.parametrize("precision", ["bf16x3", "fp32"])
@pytest.mark.parametrize("n,M,T,seed", [(200, 20, TWO_PI, 3), (2049, 1, 0.5, 5)])
def test_magnus6_mixed_matches_oracle(fl, precision, n, M, T, seed):
    """Steps with R = h dE of order one, where the mixed path's budget holds
    (its error grows with the number of low-precision terms)."""
    _say("magnus6", precision, n, M, T, seed)
    H0, V = _case(n, seed)
    f = _nodes6(T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            scheme="magnus6", precision=precision)
    U = ctx.build_ut().cpu().numpy()
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, scheme="magnus6")
    err = orc.column_error(U, Uref)
    _say("e_col", err)
    assert err < MIXED_TOL


def test_magnus6_library_cover_contains_every_step(fl):
    """The library's own interval contains every step's exact spectrum, and a
    too narrow given interval is rejected."""
    from paper_1508_07621_amd._abi import FQ_ERR_SPECTRUM, FloquetError
    n, M = 96, 10
    H0, V = _case(n, 11)
    T = 1.5                                  # long steps: the commutator terms matter
    f = _nodes6(T, M, 0.3, 1.2)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, scheme="magnus6")
    rep = ctx.report
    lo, hi, _ = _oracle_interval(H0, V, f, T, M)
    _say("cover", rep["e_min"], rep["e_max"], "exact", lo, hi)
    assert rep["e_min"] <= lo and rep["e_max"] >= hi
    with pytest.raises(FloquetError) as ei:
        fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo + 0.05, e_max=hi,
                          scheme="magnus6")
    assert ei.value.status == FQ_ERR_SPECTRUM


def test_magnus6_propagate_range_and_columns(fl):
    n, M = 150, 12
    H0, V = _case(n, 21)
    T = TWO_PI
    f = _nodes6(T, M, 0.2, 0.9)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            scheme="magnus6")
    rng = np.random.default_rng(5)
    X0 = rng.normal(size=(n, 5)) + 1j * rng.normal(size=(n, 5))
    import torch
    X = ctx.propagate(torch.from_numpy(X0).cuda(), 3, 9).cpu().numpy()
    Xref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0,
                        k_range=(3, 9), scheme="magnus6")
    err = orc.column_error(X, Xref) / max(1.0, np.linalg.norm(X0, axis=0).max())
    _say("propagate e_col", err)
    assert err < FP64_TOL


def test_magnus6_sixth_order_against_a_fine_build(fl):
    """A property at any size: against a build with 16x finer steps, the error
    falls 64x per halving of h (order six), while the library's fourth-order
    scheme on the same drive falls 16x."""
    n = 48
    H0, V = _case(n, 3)
    T = TWO_PI

    def build(M, scheme):
        f = drive_cos(orc.node_times6(T, M) if scheme == "magnus6" else orc.node_times(T, M),
                      0.0, 1.0, 1.0)
        ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, tol=1e-15, scheme=scheme)
        return ctx.build_ut().cpu().numpy()

    ref = build(512, "magnus6")
    e6 = [orc.column_error(build(M, "magnus6"), ref) for M in (16, 32)]
    e4 = [orc.column_error(build(M, "magnus4"), ref) for M in (16, 32)]
    r6, r4 = e6[0] / e6[1], e4[0] / e4[1]
    _say("errors m6", e6, "m4", e4, "ratios", r6, r4)
    assert 50.0 < r6 < 75.0
    assert 13.0 < r4 < 19.0
    assert e6[1] < 1e-2 * e4[1]
