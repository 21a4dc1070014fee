"""The dense model in the eigenbasis of H0 (the paper's working basis,
Eq. (Ham2)): H0 = diag(E_i) given by its eigenvalues, commutators with H0 taken
elementwise. Checked against the FP64 oracle (which receives diag(E) as a
dense matrix) and against the library's input-basis build after the change of
basis.
"""
import math

import numpy as np
import pytest

import oracle as orc
from workloads import drive_cos, gue

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


def _nodes(T, M, scheme):
    return drive_cos(orc.node_times6(T, M) if scheme == "magnus6" else orc.node_times(T, M),
                     0.2, 0.9, 1.0)


def _interval(H0, V, f, T, M, scheme):
    h = T / M
    if scheme == "magnus6":
        lo, hi = orc.exact_cover([orc.magnus6_heff(H0, V, f[k], h) for k in range(M)])
    elif scheme == "cf4":
        lo, hi = orc.exact_cover(orc.cf4_exponents(H0, V, f))
        h = h / 2
    else:
        a, b = orc.magnus4_weights(f, h)
        lo, hi = orc.weyl_cover(H0, V, orc.commutator(H0, V), a, b)
    return lo, hi, orc.choose_L(orc.rescale(lo, hi, h)[2], 1e-12)


@pytest.mark.parametrize("n,M,scheme,precision,tol", [
    (100, 12, "magnus4", "fp64", FP64_TOL), (130, 6, "magnus6", "fp64", FP64_TOL),
    (1030, 2, "magnus6", "fp64", FP64_TOL), (90, 8, "cf4", "fp64", FP64_TOL),
    (200, 20, "magnus4", "bf16x3", 1e-6)])
def test_eigenbasis_layout_matches_oracle(fl, n, M, scheme, precision, tol):
    _say("eigenbasis", n, M, scheme, precision)
    rng = np.random.default_rng(90 + n)
    E = np.sort(rng.normal(size=n))
    V = gue(n, rng)
    H0 = np.diag(E).astype(np.complex128)
    T = TWO_PI
    f = _nodes(T, M, scheme)
    lo, hi, L = _interval(H0, V, f, T, M, scheme)
    ctx = fl.FloquetContext(h0_eigenvalues=E, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi,
                            L=L, scheme=scheme, precision=precision)
    U = ctx.build_ut().cpu().numpy()
    Uref = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi, L=L, scheme=scheme)
    err = orc.column_error(U, Uref)
    _say("e_col", err)
    assert err < tol


def test_eigenbasis_build_is_the_input_basis_build_transformed(fl):
    """With H0 = Q diag(E) Q^dagger, the build in the eigenbasis with
    Hmod' = Q^dagger Hmod Q is Q^dagger U_T Q (same interval and order); the
    library's own covers contain every step's spectrum in both forms."""
    n, M, T = 160, 10, TWO_PI
    rng = np.random.default_rng(91)
    H0, V = gue(n, rng), gue(n, rng)
    E, Q = np.linalg.eigh(H0)
    Ve = Q.conj().T @ V @ Q
    Ve = 0.5 * (Ve + Ve.conj().T)
    f = _nodes(T, M, "magnus4")
    lo, hi, L = _interval(H0, V, f, T, M, "magnus4")
    U = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi,
                          L=L).build_ut().cpu().numpy()
    ctx = fl.FloquetContext(h0_eigenvalues=E, hmod=Ve, T=T, M=M, f_nodes=f, e_min=lo, e_max=hi,
                            L=L)
    Ue = ctx.build_ut().cpu().numpy()
    err = orc.column_error(Ue, Q.conj().T @ U @ Q)
    _say("basis change e_col", err)
    assert err < FP64_TOL
    own = fl.FloquetContext(h0_eigenvalues=E, hmod=Ve, T=T, M=M, f_nodes=f).report
    a, b = orc.magnus4_weights(f, T / M)
    K = orc.commutator(H0, V)
    xlo, xhi = orc.exact_cover([orc.magnus4_heff(H0, V, K, a[k], b[k]) for k in range(M)])
    _say("own cover", own["e_min"], own["e_max"], "exact", xlo, xhi)
    assert own["e_min"] <= xlo and own["e_max"] >= xhi
