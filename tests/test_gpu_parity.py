"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every comparison runs the library and the oracle on the same seeded inputs with
the same spectral interval and Chebyshev order, so their difference is pure
rounding; the bar for the FP64 path is 1e-10 in the worst column 2-norm.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as orc
from workloads import dimer_tridiag, drive_cos, gue, haar_unitary, workload

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi
FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def fl(require_gpu):
    from paper_1508_07621_amd import floquet
    floquet.node_times(1.0, 1)          # loads the library or raises
    return floquet


def _say(*a):
    print("[case]", *a, flush=True)


def _cos_nodes(fl, T, M, eps0=0.0, eps1=1.0):
    return drive_cos(orc.node_times(T, M), eps0, eps1, 1.0)


def _dense_case(n, seed):
    rng = np.random.default_rng(seed)
    return gue(n, rng), gue(n, rng)


def _oracle_interval(H0, V, f, T, M, tol=1e-12):
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = orc.weyl_cover(H0, V, orc.commutator(H0, V), a, b)
    _, _, R = orc.rescale(lo, hi, T / M)
    return lo, hi, orc.choose_L(R, tol)


# ---- dense FP64 ----------------------------------------------------------------------------------

@pytest.mark.parametrize("n,M,seed", [(64, 100, 1508), (100, 12, 2), (200, 6, 3), (1030, 2, 4),
                                      (1, 5, 7), (2, 1, 8), (3, 3, 9), (65, 1, 10), (2049, 1, 11)])
def test_dense_fp64_matches_oracle(fl, n, M, seed):
    """Sizes span one partial tile (n = 1, 2, 3), a tile plus one row (65), several
    tiles with ragged tails (100, 200, 1030) and a size that takes 128-row tiles in
    row-major order (2049 -> 17 x 17 tiles; the padded XCD order of larger grids
    is covered by the 10^4-state test); M = 1 is a single step."""
    _say("dense fp64", n, M, seed)
    H0, V = _dense_case(n, seed)
    T = TWO_PI
    f = _cos_nodes(fl, T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L)
    U = ctx.build_ut().cpu().numpy()
    rep = ctx.last_report
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L)
    err = orc.column_error(U, Uref)
    _say("e_col", err, "L", rep["L"], "unitarity", rep["unitarity_max"])
    assert rep["L"] == L
    assert err < FP64_TOL
    mx, fro = orc.unitarity_error(U)
    assert abs(rep["unitarity_max"] - mx) < 1e-13 + 1e-6 * mx
    assert abs(rep["unitarity_fro"] - fro) < 1e-13 + 1e-6 * fro


def test_dense_library_cover_contains_every_step(fl):
    n, M = 96, 40
    _say("dense cover", n, M)
    H0, V = _dense_case(n, 11)
    T = TWO_PI
    f = _cos_nodes(fl, T, M, 0.3, 1.2)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, tol=1e-12)
    rep = ctx.report
    a, b = orc.magnus4_weights(f, T / M)
    K = orc.commutator(H0, V)
    for k in range(M):
        ev = np.linalg.eigvalsh(H0 + a[k] * V + b[k] * K)
        assert rep["e_min"] <= ev[0] and ev[-1] <= rep["e_max"]
    U = ctx.build_ut().cpu().numpy()
    Ue = orc.build_ut(H0, V, f, T, M, route="exact")
    assert orc.column_error(U, Ue) < M * 1e-12 + 1e-10


@pytest.mark.parametrize("L", [1, 2, 3])
def test_dense_low_orders(fl, L):
    """L = 1 and L = 2 take the special buffer paths of the step."""
    n, M = 64, 5
    _say("dense low order", L)
    H0, V = _dense_case(n, 21)
    T = 0.05
    f = _cos_nodes(fl, T, M)
    lo, hi, _ = _oracle_interval(H0, V, f, T, M)
    U = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L).build_ut()
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L)
    assert orc.column_error(U.cpu().numpy(), Uref) < 1e-12


def test_dense_static_closed_form(fl):
    n, M, c = 256, 16, 0.7
    _say("dense static", n)
    H0, V = _dense_case(n, 5)
    T = 1.3
    f = np.full((M, 2), c)
    U = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, tol=1e-13).build_ut().cpu().numpy()
    ref = scipy.linalg.expm(-1j * T * (H0 + c * V))
    assert orc.column_error(U, ref) < 1e-10


def test_dense_propagate_ranges_and_columns(fl):
    n, M = 150, 10
    _say("dense propagate", n, M)
    H0, V = _dense_case(n, 6)
    T = TWO_PI
    f = _cos_nodes(fl, T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L)
    X0 = haar_unitary(n, np.random.default_rng(9))[:, :7]
    X = ctx.propagate(X0, 3, 8).cpu().numpy()
    Xref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0, k_range=(3, 8))
    assert orc.column_error(X, Xref) < FP64_TOL
    # empty step range is the identity map
    X = ctx.propagate(X0, 4, 4).cpu().numpy()
    assert np.max(np.abs(X - X0)) == 0.0
    # column subset of the full build equals propagating those columns
    U = ctx.build_ut().cpu().numpy()
    E = np.eye(n, dtype=complex)[:, [0, 77, 149]]
    Xc = ctx.propagate(E).cpu().numpy()
    assert np.max(np.abs(Xc - U[:, [0, 77, 149]])) < 1e-13


def test_dense_rejects_too_narrow_interval(fl):
    from paper_1508_07621_amd._abi import FQ_ERR_SPECTRUM, FloquetError
    H0, V = _dense_case(64, 7)
    f = _cos_nodes(fl, TWO_PI, 10)
    with pytest.raises(FloquetError) as ei:
        fl.FloquetContext(h0=H0, hmod=V, T=TWO_PI, M=10, f_nodes=f, e_min=-1.0, e_max=1.0)
    assert ei.value.status == FQ_ERR_SPECTRUM


def test_dense_full_size_sampled_columns(fl):
    """The 4096-state random-matrix model in the benchmark's launch shape
    (few steps so that the oracle can follow three columns)."""
    wl = workload("gue4096")
    H0, V = wl.arrays["h0"], wl.arrays["v"]
    M = 4
    T = wl.T
    _say("dense full size", wl.n, M)
    f = _cos_nodes(fl, T, M)
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = -4.2, 4.2
    _, _, R = orc.rescale(lo, hi, T / M)
    L = orc.choose_L(R, 1e-12)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L)
    U = ctx.build_ut()
    rep = ctx.last_report
    cols = [0, 1234, 4095]
    Uc = U[:, cols].cpu().numpy()
    X0 = np.eye(wl.n, dtype=complex)[:, cols]
    Xref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0)
    err = orc.column_error(Uc, Xref)
    _say("e_col", err, "unitarity", rep["unitarity_max"], "ms", rep["ms_build"])
    assert err < FP64_TOL
    assert rep["unitarity_max"] < 1e-11


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("bf16x3", 1e-6)])
def test_dense_n10000_full_launch_sampled_columns(fl, precision, tol):
    """The 10^4-state random-matrix model at its real shape: the whole identity
    block (79 x 79 tiles of 128) through the first two of its 200 steps (same
    step size, interval and order as the full build), four columns checked
    against the oracle."""
    wl = workload("gue10000")
    H0, V = wl.arrays["h0"], wl.arrays["v"]
    T, M, n = wl.T, wl.M, wl.n
    f = _cos_nodes(fl, T, M)
    lo, hi = -4.5, 4.5
    _, _, R = orc.rescale(lo, hi, T / M)
    L = orc.choose_L(R, 1e-12)
    _say("dense n=10^4", precision, "L", L)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            precision=precision)
    X = ctx.propagate(np.eye(n, dtype=complex), 0, 2)
    cols = [0, 4321, 8191, n - 1]
    Xc = X[:, cols].cpu().numpy()
    del X
    Xref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L,
                        X0=np.eye(n, dtype=complex)[:, cols], k_range=(0, 2))
    err = orc.column_error(Xc, Xref)
    _say("e_col", err)
    assert err < tol


# ---- dense mixed precision --------------------------------------------------------------------------

MIXED_TOL = 1e-6


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,M,seed,tol", [(64, 100, 1508, MIXED_TOL), (200, 20, 3, MIXED_TOL),
                                          (1030, 20, 4, MIXED_TOL), (300, 3, 8, MIXED_TOL)])
def test_dense_mixed_matches_oracle(fl, precision, n, M, seed, tol):
    """Bar 1e-6 in the worst column. The first cases have step sizes like the
    workloads' (R <= 1.3); the last takes three steps of R ~ 8 (27 products per
    step), where many terms carry Bessel weights |c_l| ~ 0.1-0.6: the library's
    per-term schedule gives those the accurate formats."""
    _say("dense", precision, n, M, seed)
    H0, V = _dense_case(n, seed)
    T = TWO_PI
    f = _cos_nodes(fl, T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            precision=precision)
    U = ctx.build_ut().cpu().numpy()
    rep = ctx.last_report
    cols = list(range(n)) if n <= 300 else [0, 511, n - 1]
    X0 = np.eye(n, dtype=complex)[:, cols]
    Xref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0)
    err = orc.column_error(U[:, cols], Xref)
    _say("e_col", err, "L", L, "unitarity", rep["unitarity_max"])
    assert err < tol
    assert rep["unitarity_max"] < tol


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_dense_mixed_low_orders_and_propagate(fl, precision):
    n, M = 96, 6
    H0, V = _dense_case(n, 31)
    T = 0.3
    f = _cos_nodes(fl, T, M)
    lo, hi, _ = _oracle_interval(H0, V, f, T, M)
    for L in (1, 2, 3):
        _say("dense", precision, "L", L)
        U = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                              precision=precision).build_ut().cpu().numpy()
        Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L)
        assert orc.column_error(U, Uref) < MIXED_TOL
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=5,
                            precision=precision)
    X0 = haar_unitary(n, np.random.default_rng(2))[:, :9]
    X = ctx.propagate(X0, 1, 5).cpu().numpy()
    Xref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=5, X0=X0, k_range=(1, 5))
    assert orc.column_error(X, Xref) < MIXED_TOL


# ---- optional re-orthonormalisation ------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("bf16x3", 1e-6)])
def test_dense_reorthonormalized_matches_oracle_polar_factor(fl, precision, tol):
    """Two FP64 Newton-Schulz steps after the build: against the polar factor
    of the oracle's U_T; the report keeps the build's own unitarity."""
    n, M = 200, 20
    H0, V = _dense_case(n, 13)
    T = TWO_PI
    f = _cos_nodes(fl, T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    kw = dict(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L, precision=precision)
    plain = fl.FloquetContext(**kw)
    U0 = plain.build_ut().cpu().numpy()
    ctx = fl.FloquetContext(reorthonormalize=True, **kw)
    U = ctx.build_ut().cpu().numpy()
    rep = ctx.last_report
    Uref = orc.nearest_unitary(orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L))
    err = orc.column_error(U, Uref)
    _say("reortho", precision, "e_col", err, "before", rep["unitarity_max"], "after",
         rep["unitarity_max_after"])
    assert err < tol
    assert rep["unitarity_max_after"] < 1e-14
    assert rep["unitarity_max"] == plain.last_report["unitarity_max"]
    assert orc.unitarity_error(U)[0] < 1e-14
    assert orc.column_error(U, U0) < 10 * max(rep["unitarity_max"], 1e-15) + 1e-13


def test_tridiag_reorthonormalized_matches_oracle_polar_factor(fl):
    ctx, (d, e, v, f, T, lo, hi, L) = _dimer_ctx(fl, 128, 0.01, 20)
    ctx2 = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=20, f_nodes=f, e_min=lo,
                             e_max=hi, L=L, reorthonormalize=True)
    U = ctx2.build_ut().cpu().numpy()
    Uref = orc.nearest_unitary(orc.build_ut_tridiag(d, e, v, f, T, 20, route="cheb", e_min=lo,
                                                    e_max=hi, L=L))
    err = orc.column_error(U, Uref)
    _say("tridiag reortho e_col", err, "after", ctx2.last_report["unitarity_max_after"])
    assert err < FP64_TOL
    assert ctx2.last_report["unitarity_max_after"] < 1e-14


# ---- propagation with snapshots ----------------------------------------------------------------------

def test_dense_propagate_snapshots(fl):
    """States after steps k0 + j s (the second round over a period): every
    snapshot against the oracle's propagation over the same steps."""
    n, M = 100, 12
    H0, V = _dense_case(n, 21)
    T = TWO_PI
    f = _cos_nodes(fl, T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L)
    X0 = haar_unitary(n, np.random.default_rng(5))[:, :7]
    X, snaps = ctx.propagate(X0, 2, 11, snap_every=3)
    assert snaps.shape == (3, n, 7)
    for j, k in enumerate((5, 8, 11)):
        ref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0,
                           k_range=(2, k))
        assert orc.column_error(snaps[j].cpu().numpy(), ref) < FP64_TOL
    assert np.array_equal(snaps[2].cpu().numpy(), X.cpu().numpy())


@pytest.mark.parametrize("nb,M,steps,every", [(150, 12, (1, 9), 2), (4499, 300, (0, 3), 1)])
def test_tridiag_propagate_snapshots(fl, nb, M, steps, every):
    ctx, (d, e, v, f, T, lo, hi, L) = _dimer_ctx(fl, nb, 0.05, M)
    n = nb + 1
    X0 = np.eye(n, dtype=complex)[:, [0, n // 2, n - 1]]
    X, snaps = ctx.propagate(X0, *steps, snap_every=every)
    ks = list(range(steps[0] + every, steps[1] + 1, every))
    assert snaps.shape[0] == len(ks)
    for j, k in enumerate(ks):
        ref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0,
                                   k_range=(steps[0], k))
        err = orc.column_error(snaps[j].cpu().numpy(), ref)
        _say("snapshot", n, k, err)
        assert err < FP64_TOL


# ---- complex64 storage of the state blocks ----------------------------------------------------------

def test_complex64_storage_dense_and_tridiag(fl):
    """dtype complex64: U_T, X and snapshots are stored in complex64 (the
    propagation itself keeps its working precision): errors at the complex64
    rounding level against the oracle, unitarity still measured in FP64."""
    import torch
    n, M = 96, 8
    H0, V = _dense_case(n, 41)
    T = TWO_PI
    f = _cos_nodes(fl, T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            dtype="complex64")
    U = ctx.build_ut()
    assert U.dtype == torch.complex64
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L)
    err = orc.column_error(U.cpu().numpy().astype(complex), Uref)
    _say("c64 dense e_col", err, "unitarity", ctx.last_report["unitarity_max"])
    assert err < 2e-6
    assert ctx.last_report["unitarity_max"] < 2e-6
    X0 = haar_unitary(n, np.random.default_rng(3))[:, :5].astype(np.complex64)
    X, snaps = ctx.propagate(X0, 1, 7, snap_every=3)
    assert X.dtype == torch.complex64 and snaps.dtype == torch.complex64
    ref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L,
                       X0=X0.astype(complex), k_range=(1, 4))
    assert orc.column_error(snaps[0].cpu().numpy().astype(complex), ref) < 2e-6

    ctx2, (d, e, v, f2, T2, lo2, hi2, L2) = _dimer_ctx(fl, 128, 0.01, 20)
    ctx3 = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T2, M=20, f_nodes=f2, e_min=lo2,
                             e_max=hi2, L=L2, dtype="complex64")
    U3 = ctx3.build_ut()
    assert U3.dtype == torch.complex64
    Uref3 = orc.build_ut_tridiag(d, e, v, f2, T2, 20, route="cheb", e_min=lo2, e_max=hi2, L=L2)
    err3 = orc.column_error(U3.cpu().numpy().astype(complex), Uref3)
    _say("c64 tridiag e_col", err3)
    assert err3 < 2e-6


# ---- tridiagonal (dimer) FP64 ---------------------------------------------------------------------

def _dimer_ctx(fl, nb, U_int, M, eps0=0.5, eps1=1.5, L=None, tol=1e-12):
    d, e, v = dimer_tridiag(nb, 1.0, U_int)
    T = TWO_PI
    f = _cos_nodes(fl, T, M, eps0, eps1)
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = orc.tridiag_cover(d, e, v, a, b)
    if hi - lo < 1e-12 * max(1.0, abs(lo)):      # constant H (one level): any width is exact
        lo, hi = lo - 1e-8, hi + 1e-8
    _, _, R = orc.rescale(lo, hi, T / M)
    L = orc.choose_L(R, tol) if L is None else L
    ctx = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f,
                            e_min=lo, e_max=hi, L=L)
    return ctx, (d, e, v, f, T, lo, hi, L)


@pytest.mark.parametrize("nb,U_int,M", [(0, 0.01, 10), (1, 0.0, 40), (9, 0.01, 50),
                                         (128, 0.01, 20), (200, 0.3, 20), (520, 0.01, 10),
                                         (1499, 0.01, 4)])
def test_tridiag_matches_oracle(fl, nb, U_int, M):
    _say("tridiag", nb, U_int, M)
    ctx, (d, e, v, f, T, lo, hi, L) = _dimer_ctx(fl, nb, U_int, M)
    U = ctx.build_ut().cpu().numpy()
    n = nb + 1
    cols = sorted({0, n // 3, n - 1})
    X0 = np.eye(n, dtype=complex)[:, cols]
    Xref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0)
    err = orc.column_error(U[:, cols], Xref)
    _say("e_col", err, "L", L)
    assert err < FP64_TOL
    assert ctx.last_report["unitarity_max"] < 1e-11


def test_tridiag_library_cover_is_exact(fl):
    d, e, v = dimer_tridiag(300, 1.0, 0.01)
    M = 25
    f = _cos_nodes(fl, TWO_PI, M, 0.5, 1.5)
    ctx = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=TWO_PI, M=M, f_nodes=f)
    rep = ctx.report
    lo, hi = orc.tridiag_cover(d, e, v, *orc.magnus4_weights(f, TWO_PI / M))
    assert abs(rep["e_min"] - lo) < 1e-9 * abs(lo) + 1e-9
    assert abs(rep["e_max"] - hi) < 1e-9 * abs(hi) + 1e-9


def test_tridiag_dimer1000_full_config(fl):
    """Dimer with 999 bosons, M = 500: sampled columns against the oracle and
    the time-reversal symmetry U = U^T of the whole matrix."""
    wl = workload("dimer1000")
    d, e, v = wl.arrays["h0_diag"], wl.arrays["h0_off"], wl.arrays["v_diag"]
    M, T = wl.M, wl.T
    _say("tridiag dimer1000", wl.n, M)
    f = drive_cos(orc.node_times(T, M), 0.5, 1.5, 1.0)
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = orc.tridiag_cover(d, e, v, a, b)
    _, _, R = orc.rescale(lo, hi, T / M)
    L = orc.choose_L(R, 1e-12)
    ctx = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f,
                            e_min=lo, e_max=hi, L=L)
    U = ctx.build_ut().cpu().numpy()
    rep = ctx.last_report
    cols = [0, 499, 999]
    X0 = np.eye(wl.n, dtype=complex)[:, cols]
    Xref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0)
    err = orc.column_error(U[:, cols], Xref)
    _say("e_col", err, "L", L, "R", R, "unitarity", rep["unitarity_max"], "ms", rep["ms_build"])
    assert L == rep["L"]
    assert err < FP64_TOL
    assert np.max(np.abs(U - U.T)) < 1e-10
    assert rep["unitarity_max"] < 1e-10


@pytest.mark.parametrize("nb,M,steps,cols", [(4499, 300, (0, 3), [0, 1, 3839, 3840, 4499]),
                                           (5000, 2000, (7, 9), [17, 2500, 5000])])
def test_tridiag_streamed_long_columns(fl, nb, M, steps, cols):
    """Columns longer than one workgroup holds (n > 4096) run in passes of at
    most 128 terms over blocks with ghost rows. M = 300 gives L ~ 400 (four
    passes per step); the second case has L small enough for one pass per
    step. Columns straddle the block cut at row 3840."""
    ctx, (d, e, v, f, T, lo, hi, L) = _dimer_ctx(fl, nb, 0.01, M)
    n = nb + 1
    _say("tridiag streamed", n, "M", M, "L", L, "steps", steps)
    X0 = np.eye(n, dtype=complex)[:, cols]
    X = ctx.propagate(X0, *steps).cpu().numpy()
    Xref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0,
                                k_range=steps)
    err = orc.column_error(X, Xref)
    _say("e_col", err)
    assert err < FP64_TOL


def test_tridiag_dimer10000_sampled_columns(fl):
    """The 9999-boson dimer (n = 10^4, M = 500, L = 1870: 15 passes per step) in
    its full launch shape for the first two steps: every column of the identity,
    four of them checked against the oracle, and unitarity of the block."""
    wl = workload("dimer10000")
    d, e, v = wl.arrays["h0_diag"], wl.arrays["h0_off"], wl.arrays["v_diag"]
    M, T, n = wl.M, wl.T, wl.n
    f = drive_cos(orc.node_times(T, M), 0.5, 1.5, 1.0)
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = orc.tridiag_cover(d, e, v, a, b)
    _, _, R = orc.rescale(lo, hi, T / M)
    L = orc.choose_L(R, 1e-12)
    _say("tridiag dimer10000", n, "M", M, "L", L)
    ctx = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f,
                            e_min=lo, e_max=hi, L=L)
    X = ctx.propagate(np.eye(n, dtype=complex), 0, 2)
    cols = [0, 3840, 7679, n - 1]
    Xc = X[:, cols].cpu().numpy()
    G = (X.conj().T @ X).cpu()
    del X
    uerr = float((G - np.eye(n)).abs().max())
    Xref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L,
                                X0=np.eye(n, dtype=complex)[:, cols], k_range=(0, 2))
    err = orc.column_error(Xc, Xref)
    _say("e_col", err, "unitarity", uerr)
    assert err < FP64_TOL
    assert uerr < 1e-10


def test_tridiag_propagate(fl):
    ctx, (d, e, v, f, T, lo, hi, L) = _dimer_ctx(fl, 150, 0.05, 12)
    n = 151
    X0 = haar_unitary(n, np.random.default_rng(4))[:, :5]
    X = ctx.propagate(X0, 2, 9).cpu().numpy()
    Xref = orc.build_ut_tridiag(d, e, v, f, T, 12, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0,
                                k_range=(2, 9))
    assert orc.column_error(X, Xref) < FP64_TOL


def _random_tridiag(n, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n), rng.standard_normal(n - 1) + 1j * rng.standard_normal(n - 1),
            rng.standard_normal(n))


@pytest.mark.parametrize("layout,n", [("dense", 70), ("tridiag", 150), ("tridiag", 4500)])
def test_propagate_empty_range_returns_x0(fl, layout, n):
    """k0 == k1 applies no step: X_out = X0, also at k0 = M (no step's gauge
    factors exist there) and in place."""
    _say("empty range", layout, n)
    T, M = TWO_PI, 6
    f = _cos_nodes(fl, T, M, 0.2, 0.9)
    if layout == "dense":
        H0, V = _dense_case(n, 31)
        ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f)
    else:
        d, e, v = _random_tridiag(n, 32)
        ctx = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f)
    rng = np.random.default_rng(33)
    X0 = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    for k in (0, 3, M):
        X = ctx.propagate(X0, k, k).cpu().numpy()
        assert np.array_equal(X, X0)
    import torch
    Xd = torch.from_numpy(X0).cuda()
    ctx.propagate(Xd, M, M, out=Xd)
    assert np.array_equal(Xd.cpu().numpy(), X0)


def test_tridiag_streamed_in_place(fl):
    """Columns longer than one workgroup holds (4500 rows) propagated in place:
    one step whose terms fit one 128-term pass (that pass reads X0 with ghost
    rows and writes X_out), and three steps."""
    import torch
    n, M, T = 4500, 10, TWO_PI
    d, e, v = _random_tridiag(n, 34)
    f = _cos_nodes(fl, T, M, 0.2, 0.9)
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = orc.tridiag_cover(d, e, v, a, b)
    L = orc.choose_L(orc.rescale(lo, hi, T / M)[2], 1e-12)
    _say("streamed in place", n, M, "L", L)
    assert L + 1 <= 128
    ctx = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f, e_min=lo,
                            e_max=hi, L=L)
    X0 = haar_unitary(n, np.random.default_rng(35))[:, :4]
    for k0, k1 in ((3, 4), (3, 6)):
        Xd = torch.from_numpy(X0).cuda()
        ctx.propagate(Xd, k0, k1, out=Xd)
        Xref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L,
                                    X0=X0, k_range=(k0, k1))
        err = orc.column_error(Xd.cpu().numpy(), Xref)
        _say("steps", k0, k1, "e_col", err)
        assert err < FP64_TOL


def test_tridiag_complex_offdiagonal(fl):
    """A general Hermitian tridiagonal H0 (complex couplings) with a diagonal Hmod."""
    rng = np.random.default_rng(12)
    n, M = 300, 8
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1) + 1j * rng.standard_normal(n - 1)
    v = rng.standard_normal(n)
    T = 2.0
    f = _cos_nodes(fl, T, M, 0.2, 0.9)
    a, b = orc.magnus4_weights(f, T / M)
    lo, hi = orc.tridiag_cover(d, e, v, a, b)
    _, _, R = orc.rescale(lo, hi, T / M)
    L = orc.choose_L(R, 1e-12)
    U = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f,
                          e_min=lo, e_max=hi, L=L).build_ut().cpu().numpy()
    Uref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L)
    assert orc.column_error(U, Uref) < FP64_TOL


# ---- streams -----------------------------------------------------------------------------------------

def test_context_on_side_stream_matches_default_stream(fl):
    """Every setup copy and fill of fq_create runs on the context's stream: a
    context created and built on a non-blocking side stream, with its operators
    uploaded on that stream just before, gives bit for bit the result of the
    default stream (tridiagonal: host copies of the diagonals and the gauge
    table; dense eigenbasis layout: the eigenvalue copy and the Lanczos cover)."""
    import torch
    T, M = TWO_PI, 30
    d, e, v = dimer_tridiag(200, 1.0, 0.01)
    f = _cos_nodes(fl, T, M, 0.5, 1.5)
    rng = np.random.default_rng(44)
    E = np.sort(rng.standard_normal(150))
    V = gue(150, rng)
    fd = _cos_nodes(fl, T, M)

    def builds():
        tri = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f)
        den = fl.FloquetContext(h0_eigenvalues=E, hmod=V, T=T, M=M, f_nodes=fd)
        return tri.build_ut(), den.build_ut(), tri.report, den.report

    _say("side stream: default-stream builds")
    ref = builds()
    side = torch.cuda.Stream()
    _say("side stream: builds on a non-blocking stream")
    with torch.cuda.stream(side):
        got = builds()
    side.synchronize()
    for r, g in zip(ref[:2], got[:2]):
        assert torch.equal(r, g)
    for r, g in zip(ref[2:], got[2:]):
        assert (r["e_min"], r["e_max"], r["L"]) == (g["e_min"], g["e_max"], g["L"])


# ---- full-length workload against the oracle --------------------------------------------------------

def test_dense_n4096_full_period_sampled_columns(fl):
    """The 4096-state random-matrix workload exactly as the benchmark builds it
    (library interval and order, all M = 200 steps): three columns of the FP64
    and of the split-BF16 build against the oracle followed over the whole
    period on those columns."""
    import torch
    wl = workload("gue4096")
    H0, V = wl.arrays["h0"], wl.arrays["v"]
    T, M, n = wl.T, wl.M, wl.n
    f = _cos_nodes(fl, T, M)
    cols = [7, 2048, 4095]
    ref = None
    for precision, tol in (("fp64", FP64_TOL), ("bf16x3", MIXED_TOL)):
        _say("gue4096 full period", precision)
        ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, tol=1e-12,
                                precision=precision)
        rep = ctx.report
        U = ctx.build_ut()
        Uc = U[:, cols].cpu().numpy()
        del U, ctx
        torch.cuda.empty_cache()
        if ref is None:
            _say("oracle: 3 columns over", M, "steps, L", rep["L"])
            ref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=rep["e_min"],
                               e_max=rep["e_max"], L=rep["L"],
                               X0=np.eye(n, dtype=complex)[:, cols])
        err = orc.column_error(Uc, ref)
        _say("e_col", precision, err)
        assert err < tol


def test_divergence_flag(fl):
    """The report flags a build whose result is far from unitary: with a
    Chebyshev order far below what the step needs (R ~ 8 with L = 2) the series
    does not converge and ||U^dagger U - 1|| is of order one; the properly
    ordered build of the same problem is not flagged."""
    H0, V = _dense_case(64, 5)
    T, M = TWO_PI, 3
    f = _cos_nodes(fl, T, M)
    lo, hi, L = _oracle_interval(H0, V, f, T, M)
    for order, flag in ((L, 0), (2, 1)):
        ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=order)
        ctx.build_ut()
        rep = ctx.last_report
        _say("L", order, "unitarity", rep["unitarity_max"], "diverged", rep["diverged"])
        assert rep["diverged"] == flag


@pytest.mark.parametrize("case", ["magnus4", "cf4", "eigen", "propagate"])
def test_small_chain_matches_launch_per_product_form(fl, case, monkeypatch):
    """N <= 64 in FP64 runs every step of a build in one launch (16 states per
    workgroup, Ht formed in LDS per step); the launch-per-product form
    (FQ_SMALL_CHAIN=0) and the oracle must agree with it."""
    import torch
    n, M = 64 if case != "propagate" else 50, 100
    T = TWO_PI
    H0, V = _dense_case(n, 1508)
    scheme = "cf4" if case == "cf4" else "magnus4"
    f = _cos_nodes(fl, T, M)
    kw = dict(T=T, M=M, f_nodes=f, scheme=scheme)
    if case == "eigen":
        E, Q = np.linalg.eigh(H0)
        kw.update(h0_eigenvalues=E, hmod=Q.conj().T @ V @ Q)
    else:
        kw.update(h0=H0, hmod=V)
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("FQ_SMALL_CHAIN", flag)
        ctx = fl.FloquetContext(profile=True, **kw)
        if case == "propagate":
            X0 = haar_unitary(n, np.random.default_rng(3))[:, :7]
            outs.append(ctx.propagate(X0, 13, 71).cpu().numpy())
        else:
            outs.append(ctx.build_ut().cpu().numpy())
            from paper_1508_07621_amd._abi import K_CHAIN
            launches = ctx.last_report["n_kernel"][K_CHAIN]
            assert launches == (1 if flag == "1" else 0)
        rep = ctx.report
    _say(case, "chain vs per-product", np.abs(outs[0] - outs[1]).max())
    assert np.abs(outs[0] - outs[1]).max() < 1e-13
    if case == "magnus4":
        Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=rep["e_min"], e_max=rep["e_max"],
                            L=rep["L"])
        assert orc.column_error(outs[0], Uref) < FP64_TOL
