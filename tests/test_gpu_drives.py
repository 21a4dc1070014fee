"""Several drive terms, H(t) = H0 + sum_s f_s(t) Hmod_s, on the GPU against the
FP64 oracle: builds for the Magnus-4 (with the commutators [H0, Hmod_s] and
[Hmod_s, Hmod_t]) and commutator-free schemes, both dense layouts, mixed
precision, the gradient with respect to every drive sample, and the period
average.
"""
import math

import numpy as np
import pytest

import oracle as orc
from workloads import gue, haar_unitary

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


def _problem(n, S, seed):
    rng = np.random.default_rng(seed)
    return gue(n, rng), [gue(n, rng) for _ in range(S)]


def _drive(T, M, S):
    """f_s(t) = cos((s + 1) t + s / 2) / (s + 1) at the two nodes: (M, 2, S)."""
    t = orc.node_times(T, M)
    return np.stack([np.cos((s + 1) * t + 0.5 * s) / (s + 1) for s in range(S)], -1)


def _interval(H0, Vs, f, T, M, scheme, tol=1e-12):
    h = T / M
    if scheme == "cf4":
        ops = orc.cf4_exponents(H0, Vs, f)
        h = h / 2
    else:
        ops = [orc.magnus4_heff_drives(H0, Vs, f[k, 0], f[k, 1], T / M) for k in range(M)]
    lo, hi = orc.exact_cover(ops)
    return lo, hi, orc.choose_L(orc.rescale(lo, hi, h)[2], tol)


@pytest.mark.parametrize("n,M,S,scheme,precision,tol", [
    (64, 12, 2, "magnus4", "fp64", FP64_TOL), (200, 6, 3, "magnus4", "fp64", FP64_TOL),
    (1030, 2, 4, "magnus4", "fp64", FP64_TOL), (90, 8, 3, "cf4", "fp64", FP64_TOL),
    (200, 16, 2, "magnus4", "bf16x3", 1e-6), (200, 16, 2, "cf4", "fp32", 1e-6)])
def test_drives_build_matches_oracle(fl, n, M, S, scheme, precision, tol):
    _say("drives", n, M, S, scheme, precision)
    H0, Vs = _problem(n, S, 100 + n + S)
    T = TWO_PI
    f = _drive(T, M, S)
    lo, hi, L = _interval(H0, Vs, f, T, M, scheme)
    ctx = fl.FloquetContext(h0=H0, hmod=Vs, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            scheme=scheme, precision=precision)
    U = ctx.build_ut().cpu().numpy()
    Uref = orc.build_ut(H0, Vs, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, scheme=scheme)
    err = orc.column_error(U, Uref)
    _say("e_col", err, "L", L)
    assert err < tol


def test_drives_eigenbasis_and_library_cover(fl):
    """Two drive terms with H0 given by its eigenvalues; the library's own
    interval contains every step's exact spectrum."""
    n, M, S, T = 120, 10, 2, TWO_PI
    rng = np.random.default_rng(110)
    E = np.sort(rng.normal(size=n))
    Vs = [gue(n, rng) for _ in range(S)]
    H0 = np.diag(E).astype(np.complex128)
    f = _drive(T, M, S)
    lo, hi, L = _interval(H0, Vs, f, T, M, "magnus4")
    ctx = fl.FloquetContext(h0_eigenvalues=E, hmod=Vs, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi,
                            L=L)
    U = ctx.build_ut().cpu().numpy()
    Uref = orc.build_ut(H0, Vs, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L)
    assert orc.column_error(U, Uref) < FP64_TOL
    own = fl.FloquetContext(h0_eigenvalues=E, hmod=Vs, T=T, M=M, f_nodes=f).report
    _say("own cover", own["e_min"], own["e_max"], "exact", lo, hi)
    assert own["e_min"] <= lo and own["e_max"] >= hi


def _trace_loss_and_bar(U, W):
    N = U.shape[0]
    tau = np.trace(W.conj().T @ U)
    return 1.0 - abs(tau) ** 2 / N ** 2, -2.0 * tau * W / N ** 2


@pytest.mark.parametrize("scheme", ["magnus4", "cf4"])
def test_drives_gradient_matches_oracle_differences(fl, scheme):
    """Every derivative d loss / d f_s(node) for two drive terms against central
    differences of the oracle (the [V1, V2] term is bilinear in the samples)."""
    n, M, S, T = 24, 6, 2, TWO_PI
    H0, Vs = _problem(n, S, 120)
    W = haar_unitary(n, np.random.default_rng(121))
    f = _drive(T, M, S)
    lo, hi, _ = _interval(H0, Vs, f, T, M, scheme)
    lo, hi = lo - 1.0, hi + 1.0
    h = T / M / (2 if scheme == "cf4" else 1)
    L = orc.choose_L(orc.rescale(lo, hi, h)[2], 1e-14)
    ctx = fl.FloquetContext(h0=H0, hmod=Vs, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L,
                            checkpoint_every=2, scheme=scheme)
    U = ctx.build_ut().cpu().numpy()
    g = ctx.grad(_trace_loss_and_bar(U, W)[1])
    assert g.shape == (M, 2, S)

    def loss(ff):
        Uo = orc.build_ut(H0, Vs, ff, T, M, route="cheb", e_min=lo, e_max=hi, L=L, scheme=scheme)
        return _trace_loss_and_bar(Uo, W)[0]

    eps = 1e-5
    fd = np.zeros_like(f)
    for idx in np.ndindex(*f.shape):
        fp, fm = f.copy(), f.copy()
        fp[idx] += eps
        fm[idx] -= eps
        fd[idx] = (loss(fp) - loss(fm)) / (2 * eps)
    err = np.max(np.abs(g - fd)) / np.max(np.abs(fd))
    _say(scheme, "drives gradient rel err", err)
    assert err < 1e-6


def test_drives_period_average_matches_oracle(fl):
    n, M, S, T = 100, 8, 3, TWO_PI
    H0, Vs = _problem(n, S, 130)
    f = _drive(T, M, S)
    tg = np.arange(M) * T / M
    fg = np.stack([np.cos((s + 1) * tg + 0.5 * s) / (s + 1) for s in range(S)], -1)
    lo, hi, L = _interval(H0, Vs, f, T, M, "magnus4")
    X0 = haar_unitary(n, np.random.default_rng(131))[:, :6]
    ctx = fl.FloquetContext(h0=H0, hmod=Vs, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi, L=L)
    got = ctx.period_average(X0, fg)
    ref = orc.period_average(H0, Vs, f, fg, T, M, X0, route="cheb", e_min=lo, e_max=hi, L=L)
    err = np.abs(got - ref).max()
    _say("drives period average", err)
    assert err < 1e-12
