"""The commutator-free fourth-order scheme (two half-step exponentials of
linear combinations of H at the Gauss-Legendre nodes) on the GPU against the
FP64 oracle: dense and tridiagonal builds, propagation ranges and snapshots,
the gradient, and its order.
"""
import math

import numpy as np
import pytest

import oracle as orc
from workloads import dimer_tridiag, drive_cos, gue, haar_unitary

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


def _case(n, seed):
    rng = np.random.default_rng(seed)
    return gue(n, rng), gue(n, rng)


def _dense_interval(H0, V, f, T, M, tol=1e-12):
    lo, hi = orc.exact_cover(orc.cf4_exponents(H0, V, f))
    return lo, hi, orc.choose_L(orc.rescale(lo, hi, T / (2 * M))[2], tol)


def _tridiag_interval(d, e, v, f, T, M, tol=1e-12):
    ff = np.asarray(f).reshape(-1, 2)
    a = np.stack([2 * (orc.CF4_A1 * ff[:, 0] + orc.CF4_A2 * ff[:, 1]),
                  2 * (orc.CF4_A2 * ff[:, 0] + orc.CF4_A1 * ff[:, 1])], 1).ravel()
    lo, hi = orc.tridiag_cover(d, e, v, a, np.zeros_like(a))
    return lo, hi, orc.choose_L(orc.rescale(lo, hi, T / (2 * M))[2], tol)


@pytest.mark.parametrize("n,M,seed,precision,tol", [
    (64, 20, 1508, "fp64", FP64_TOL), (200, 6, 3, "fp64", FP64_TOL), (1030, 2, 4, "fp64", FP64_TOL),
    (1, 3, 7, "fp64", FP64_TOL), (200, 20, 5, "bf16x3", 1e-6), (200, 20, 5, "fp32", 1e-6)])
def test_cf4_dense_matches_oracle(fl, n, M, seed, precision, tol):
    _say("cf4 dense", n, M, seed, precision)
    H0, V = _case(n, seed)
    T = TWO_PI
    f = drive_cos(orc.node_times(T, M), 0.0, 1.0, 1.0)
    lo, hi, L = _dense_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            scheme="cf4", precision=precision)
    U = ctx.build_ut().cpu().numpy()
    rep = ctx.last_report
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, scheme="cf4")
    err = orc.column_error(U, Uref)
    _say("e_col", err, "L", rep["L"], "M", rep["M"])
    assert rep["L"] == L and rep["M"] == M
    assert err < tol


@pytest.mark.parametrize("nb,M", [(150, 12), (4499, 4)])
def test_cf4_tridiag_matches_oracle(fl, nb, M):
    """Resident columns (151 rows) and streamed passes (4500 rows)."""
    _say("cf4 tridiag", nb, M)
    d, e, v = dimer_tridiag(nb, 1.0, 0.01)
    T = TWO_PI if nb < 1000 else 0.02
    f = drive_cos(orc.node_times(T, M), 0.5, 1.5, 1.0)
    lo, hi, L = _tridiag_interval(d, e, v, f, T, M)
    ctx = fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f, e_min=lo,
                            e_max=hi, L=L, scheme="cf4")
    n = nb + 1
    cols = [0, n // 3, n - 1]
    X0 = np.zeros((n, len(cols)), dtype=np.complex128)
    X0[cols, np.arange(len(cols))] = 1.0
    X = ctx.propagate(X0).cpu().numpy()
    Xref = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0,
                                scheme="cf4")
    err = orc.column_error(X, Xref)
    _say("e_col", err, "L", L)
    assert err < FP64_TOL


def test_cf4_propagate_ranges_and_snapshots(fl):
    """Step indices of the caller count whole steps (two half-steps each)."""
    n, M = 120, 10
    H0, V = _case(n, 9)
    T = TWO_PI
    f = drive_cos(orc.node_times(T, M), 0.3, 0.8, 1.0)
    lo, hi, L = _dense_interval(H0, V, f, T, M)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            scheme="cf4")
    X0 = haar_unitary(n, np.random.default_rng(10))[:, :4]
    X, snaps = ctx.propagate(X0, 2, 8, snap_every=3)
    snaps = snaps.cpu().numpy()
    assert snaps.shape == (2, n, 4)
    for j, k1 in enumerate((5, 8)):
        ref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, X0=X0,
                           k_range=(2, k1), scheme="cf4")
        assert orc.column_error(snaps[j], ref) < FP64_TOL
    assert orc.column_error(X.cpu().numpy(), snaps[-1]) == 0.0


def _trace_loss_and_bar(U, W):
    N = U.shape[0]
    tau = np.trace(W.conj().T @ U)
    loss = 1.0 - abs(tau) ** 2 / N ** 2
    return loss, -2.0 * tau * W / N ** 2


@pytest.mark.parametrize("layout", ["dense", "tridiag"])
def test_cf4_gradient_matches_oracle_differences(fl, layout):
    """Every node derivative of a trace-fidelity loss against central
    differences of the oracle's build."""
    M, T = 8, TWO_PI
    f = drive_cos(orc.node_times(T, M), 0.4, 1.2, 1.0)
    if layout == "dense":
        n = 24
        H0, V = _case(n, 77)
        lo, hi = -5.0, 5.0
        L = 30
        kw = dict(h0=H0, hmod=V)

        def build(ff):
            return orc.build_ut(H0, V, ff, T, M, route="cheb", e_min=lo, e_max=hi, L=L,
                                scheme="cf4")
    else:
        nb = 23
        n = nb + 1
        d, e, v = dimer_tridiag(nb, 1.0, 0.3)
        lo, hi, _ = _tridiag_interval(d, e, v, f, T, M)
        lo, hi = lo - 1.0, hi + 1.0   # room for the perturbed drives
        L = orc.choose_L(orc.rescale(lo, hi, T / (2 * M))[2], 1e-14)
        kw = dict(h0_diag=d, h0_off=e, hmod_diag=v)

        def build(ff):
            return orc.build_ut_tridiag(d, e, v, ff, T, M, route="cheb", e_min=lo, e_max=hi, L=L,
                                        scheme="cf4")
    W = haar_unitary(n, np.random.default_rng(78))
    ctx = fl.FloquetContext(T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L, checkpoint_every=3,
                            scheme="cf4", **kw)
    U = ctx.build_ut().cpu().numpy()
    _, Ubar = _trace_loss_and_bar(U, W)
    g = ctx.grad(Ubar)
    eps = 1e-5
    fd = np.zeros_like(f)
    for k in range(M):
        for i in range(2):
            fp, fm = f.copy(), f.copy()
            fp[k, i] += eps
            fm[k, i] -= eps
            fd[k, i] = (_trace_loss_and_bar(build(fp), W)[0] -
                        _trace_loss_and_bar(build(fm), W)[0]) / (2 * eps)
    err = np.max(np.abs(g - fd)) / np.max(np.abs(fd))
    _say(layout, "cf4 gradient rel err", err)
    assert err < 1e-6
    assert np.max(np.abs(g[:, 0] - g[:, 1])) > 1e-6 * np.max(np.abs(g))


def test_cf4_fourth_order_against_a_fine_build(fl):
    """Error ratio 16 per halving of h against a build with 16x finer steps."""
    n = 48
    H0, V = _case(n, 3)
    T = TWO_PI

    def build(M):
        f = drive_cos(orc.node_times(T, M), 0.0, 1.0, 1.0)
        ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, tol=1e-15, scheme="cf4")
        return ctx.build_ut().cpu().numpy()

    ref = build(512)
    e = [orc.column_error(build(M), ref) for M in (16, 32)]
    _say("cf4 errors", e, "ratio", e[0] / e[1])
    assert 13.0 < e[0] / e[1] < 19.0
