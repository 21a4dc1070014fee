"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test checks the oracle against a closed form, an independent integrator,
group theory, a published table or a mathematical identity, chosen so that a
plausible slip (a dropped term, a flipped sign, a transposed product, a wrong
index) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg
import scipy.special

import oracle as orc
from workloads import dimer_dense, dimer_tridiag, drive_cos, gue, haar_unitary

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TWO_PI = 2.0 * math.pi


def _rm(n, seed):
    rng = np.random.default_rng(seed)
    return gue(n, rng), gue(n, rng)


def _nodes_cos(T, M, eps0=0.0, eps1=1.0, omega=1.0):
    return drive_cos(orc.node_times(T, M), eps0, eps1, omega)


def _brute_force(H_of_t, n, T, rtol=1e-13, atol=1e-13):
    """U(T) from i dU/dt = H(t) U, U(0) = 1, by an adaptive 8th-order
    Runge-Kutta (DOP853) on the real and imaginary parts."""
    def rhs(t, y):
        U = (y[: n * n] + 1j * y[n * n:]).reshape(n, n)
        dU = -1j * (H_of_t(t) @ U)
        return np.concatenate([dU.real.ravel(), dU.imag.ravel()])

    y0 = np.concatenate([np.eye(n).ravel(), np.zeros(n * n)])
    sol = scipy.integrate.solve_ivp(rhs, (0.0, T), y0, method="DOP853", rtol=rtol, atol=atol)
    y = sol.y[:, -1]
    return (y[: n * n] + 1j * y[n * n:]).reshape(n, n)


def _spin_matrices(S2):
    """Spin-S matrices (S = S2/2) in the basis m = -S, ..., S (ascending)."""
    S = S2 / 2.0
    m = np.arange(S2 + 1) - S
    Sz = np.diag(m).astype(np.complex128)
    Sp = np.zeros((S2 + 1, S2 + 1), dtype=np.complex128)
    for i in range(S2):
        Sp[i + 1, i] = math.sqrt(S * (S + 1) - m[i] * (m[i] + 1))
    Sx = (Sp + Sp.conj().T) / 2
    Sy = (Sp - Sp.conj().T) / 2j
    return Sx, Sy, Sz


# --- Bessel weights and the scalar expansion -------------------------------------------------

def test_bessel_against_published_table():
    rows = np.loadtxt(os.path.join(GOLDEN, "bessel_table.txt"))
    for n, x, ref in rows:
        a = orc.bessel_coefficients(x, int(n))
        val = a[int(n)] / (1.0 if n == 0 else 2.0)
        assert abs(val - ref) <= 5e-10 * max(1.0, abs(ref)) + 1e-19, (n, x, val, ref)


@pytest.mark.parametrize("R", [0.126, 0.251, 3.0, 37.03, 250.0])
def test_jacobi_anger(R):
    """sum_l a_l (-i)^l T_l(x) = exp(-i R x) on [-1, 1] to the chosen tolerance,
    and J_0 + 2 sum_k J_2k = 1."""
    tol = 1e-13
    L = orc.choose_L(R, tol)
    a = orc.bessel_coefficients(R, L)
    x = np.linspace(-1.0, 1.0, 2001)
    p, _ = orc.chebyshev_polynomial_values(x, a, 0.0, 1.0)
    assert np.max(np.abs(p - np.exp(-1j * R * x))) < 50 * tol
    big = orc.bessel_coefficients(R, L + 40)
    assert abs(big[0] + np.sum(big[2::2]) - 1.0) < 1e-12


def test_choose_L_is_minimal():
    for R in [0.05, 0.126, 1.0, 10.0, 37.03, 300.0]:
        tol = 1e-12
        L = orc.choose_L(R, tol)
        j = np.abs(scipy.special.jv(np.arange(L + 400), R))
        assert 2 * j[L + 1:].sum() <= tol
        if L > 1:
            assert 2 * j[L:].sum() > tol


def test_chebyshev_polynomial_derivative():
    a = orc.bessel_coefficients(2.0, 30)
    x = np.linspace(-0.9, 0.9, 7)
    _, dp = orc.chebyshev_polynomial_values(x, a, 0.3, 0.1)
    e = 1e-6
    pp, _ = orc.chebyshev_polynomial_values(x + e, a, 0.3, 0.1)
    pm, _ = orc.chebyshev_polynomial_values(x - e, a, 0.3, 0.1)
    assert np.max(np.abs((pp - pm) / (2 * e) - dp)) < 1e-7


def test_chebyshev_step_on_known_spectrum():
    """Matrix recurrence on H = Q diag(lam) Q^dagger with Q and lam chosen, not
    computed: must equal Q diag(exp(-i h lam)) Q^dagger X."""
    rng = np.random.default_rng(7)
    n = 12
    Q = haar_unitary(n, rng)
    lam = rng.uniform(-3.0, 5.0, n)
    H = (Q * lam) @ Q.conj().T
    X = haar_unitary(n, rng)[:, :5]
    h = 0.37
    beta, dE, R = orc.rescale(-3.0, 5.0, h)
    a = orc.bessel_coefficients(R, orc.choose_L(R, 1e-14))
    got = orc.chebyshev_step(H, beta, dE, h, a, X)
    ref = (Q * np.exp(-1j * h * lam)) @ (Q.conj().T @ X)
    assert np.max(np.abs(got - ref)) < 1e-12


# --- Gauss-Legendre nodes and the Magnus-4 step -----------------------------------------------

def test_node_times_integrate_cubics_exactly():
    T, M = 2.0, 7
    t = orc.node_times(T, M)
    h = T / M
    for deg in range(4):
        quad = h / 2 * np.sum(t[:, 0] ** deg + t[:, 1] ** deg)
        assert abs(quad - T ** (deg + 1) / (deg + 1)) < 1e-12
    quad4 = h / 2 * np.sum(t[:, 0] ** 4 + t[:, 1] ** 4)
    assert abs(quad4 - T ** 5 / 5) > 1e-6        # degree 4 is not exact


def test_static_hamiltonian_closed_form():
    """f = const: no commutator term, U_T = exp(-i T (H0 + c V)) exactly."""
    H0, V = _rm(8, 11)
    T, M, c = 1.7, 20, 0.6
    f = np.full((M, 2), c)
    ref = scipy.linalg.expm(-1j * T * (H0 + c * V))
    Ue = orc.build_ut(H0, V, f, T, M, route="exact")
    Uc = orc.build_ut(H0, V, f, T, M, route="cheb", tol=1e-14)
    assert orc.column_error(Ue, ref) < 1e-12
    assert orc.column_error(Uc, ref) < 1e-11


def test_zero_h0_closed_form():
    """H0 = 0: all steps commute and the Gauss-Legendre sum of cos over a
    period vanishes, so U_T = exp(-i eps0 T V)."""
    _, V = _rm(6, 12)
    T, M = TWO_PI, 30
    f = _nodes_cos(T, M, eps0=0.4, eps1=1.3)
    U = orc.build_ut(np.zeros_like(V), V, f, T, M, route="cheb", tol=1e-14)
    ref = scipy.linalg.expm(-1j * 0.4 * T * V)
    assert orc.column_error(U, ref) < 1e-11


def _gue_drive(n, seed):
    H0, V = _rm(n, seed)
    return H0, V, (lambda t: H0 + math.cos(t) * V)


def test_brute_force_tiny():
    H0, V, Ht = _gue_drive(4, 21)
    T, M = TWO_PI, 200
    ref = _brute_force(Ht, 4, T)
    U = orc.build_ut(H0, V, _nodes_cos(T, M), T, M, route="cheb")
    assert orc.column_error(U, ref) < 2e-7


def test_fourth_order_convergence_and_commutator_sign():
    """e(M) / e(2M) -> 16 for the scheme; swapping the two nodes flips the sign
    of the commutator term and must drop the order to 2 (ratio 4)."""
    H0, V, Ht = _gue_drive(6, 3)
    T = TWO_PI
    ref = _brute_force(Ht, 6, T)
    errs, errs_flip = [], []
    for M in (25, 50, 100):
        f = _nodes_cos(T, M)
        errs.append(orc.column_error(orc.build_ut(H0, V, f, T, M, route="exact"), ref))
        errs_flip.append(orc.column_error(orc.build_ut(H0, V, f[:, ::-1], T, M, route="exact"), ref))
    r = [errs[i] / errs[i + 1] for i in range(2)]
    rf = [errs_flip[i] / errs_flip[i + 1] for i in range(2)]
    assert all(14.0 < x < 18.0 for x in r), r
    assert all(3.5 < x < 4.6 for x in rf), rf


def test_ordering_later_steps_on_the_left():
    """A non-commuting two-valued piecewise drive: the chain must equal
    E_2 E_1 (later on the left), not E_1 E_2."""
    H0, V = _rm(5, 4)
    T, M = 1.0, 2
    f = np.array([[0.3, 0.3], [-1.1, -1.1]])
    h = T / M
    E1 = scipy.linalg.expm(-1j * h * (H0 + 0.3 * V))
    E2 = scipy.linalg.expm(-1j * h * (H0 - 1.1 * V))
    U = orc.build_ut(H0, V, f, T, M, route="cheb", tol=1e-14)
    assert orc.column_error(U, E2 @ E1) < 1e-12
    assert orc.column_error(U, E1 @ E2) > 1e-3


def test_step_ranges_compose():
    """E_M..E_{k+1} (E_k..E_1 X) = E_M..E_1 X: resuming from any step."""
    H0, V = _rm(7, 14)
    T, M = TWO_PI, 12
    f = _nodes_cos(T, M)
    X0 = haar_unitary(7, np.random.default_rng(3))[:, :3]
    full = orc.build_ut(H0, V, f, T, M, route="exact", X0=X0)
    mid = orc.build_ut(H0, V, f, T, M, route="exact", X0=X0, k_range=(0, 5))
    rest = orc.build_ut(H0, V, f, T, M, route="exact", X0=mid, k_range=(5, 12))
    assert orc.column_error(rest, full) < 1e-13


def test_unitarity_of_chebyshev_route():
    H0, V = _rm(16, 5)
    T, M = TWO_PI, 50
    U = orc.build_ut(H0, V, _nodes_cos(T, M), T, M, route="cheb", tol=1e-13)
    mx, fro = orc.unitarity_error(U)
    assert mx < 1e-12 and fro < 1e-11


def test_route_c_matches_route_e_to_truncation():
    H0, V = _rm(10, 6)
    T, M = TWO_PI, 40
    f = _nodes_cos(T, M)
    Ue = orc.build_ut(H0, V, f, T, M, route="exact")
    for tol in (1e-8, 1e-12):
        Uc = orc.build_ut(H0, V, f, T, M, route="cheb", tol=tol)
        assert orc.column_error(Uc, Ue) <= M * tol + 1e-12


def test_cover_independence():
    """Widening the spectral interval changes the Chebyshev route only at
    truncation level."""
    H0, V = _rm(8, 8)
    T, M = TWO_PI, 30
    f = _nodes_cos(T, M)
    U1, info = orc.build_ut(H0, V, f, T, M, route="cheb", tol=1e-13, return_info=True)
    U2 = orc.build_ut(H0, V, f, T, M, route="cheb", tol=1e-13,
                      e_min=info["e_min"] - 3.0, e_max=info["e_max"] + 5.0)
    assert orc.column_error(U1, U2) < 1e-10


def test_weyl_cover_contains_every_step():
    H0, V = _rm(20, 9)
    T, M = TWO_PI, 25
    h = T / M
    a, b = orc.magnus4_weights(_nodes_cos(T, M), h)
    K = orc.commutator(H0, V)
    lo, hi = orc.weyl_cover(H0, V, K, a, b)
    for k in range(M):
        ev = np.linalg.eigvalsh(H0 + a[k] * V + b[k] * K)
        assert lo <= ev[0] and ev[-1] <= hi


# --- Bose-Hubbard dimer -----------------------------------------------------------------------

def test_dimer_noninteracting_is_spin_representation():
    """U = 0: H0 = -2 J S_x and V = 2 S_z of spin S = Nb/2 (Schwinger map). The
    Lie-algebra map preserves commutators, so the discrete scheme on Nb bosons
    equals the spin-S image of the same scheme on one boson (2 x 2)."""
    nb, J = 9, 1.0
    T, M = TWO_PI, 40
    f = _nodes_cos(T, M, eps0=0.5, eps1=1.5)
    d1, e1, v1 = dimer_tridiag(1, J, 0.0)
    u = orc.build_ut_tridiag(d1, e1, v1, f, T, M, route="exact")
    Sx1, Sy1, Sz1 = _spin_matrices(1)
    sig = [2 * Sx1, 2 * Sy1, 2 * Sz1]
    # u = cos|a| 1 - i sin|a| (a/|a|).sigma  (det u = 1 since H is traceless)
    c = np.real(np.trace(u)) / 2
    s_vec = np.array([np.real(1j * np.trace(u @ s) / 2) for s in sig])   # = sin|a| a/|a|
    ang = math.atan2(np.linalg.norm(s_vec), c)
    avec = s_vec / np.linalg.norm(s_vec) * ang
    SxN, SyN, SzN = _spin_matrices(nb)
    ref = scipy.linalg.expm(-1j * 2 * (avec[0] * SxN + avec[1] * SyN + avec[2] * SzN))
    dN, eN, vN = dimer_tridiag(nb, J, 0.0)
    for route in ("exact", "cheb"):
        U = orc.build_ut_tridiag(dN, eN, vN, f, T, M, route=route, tol=1e-14)
        assert orc.column_error(U, ref) < 1e-11, route
    # eigenphase ladder: eig(u) = exp(-/+ i phi) -> eig(U) = exp(-i 2 m phi)
    th_u = orc.eigenphases(u)
    phi = abs(th_u[0])
    ladder = -2 * (np.arange(nb + 1) - nb / 2) * phi
    ladder = np.angle(np.exp(-1j * ladder)) * -1.0
    assert orc.quasienergy_distance(orc.eigenphases(ref), ladder, T) < 1e-10


def test_two_level_dimer_brute_force():
    d1, e1, v1 = dimer_tridiag(1, 1.0, 0.0)
    H0, V = dimer_dense(1, 1.0, 0.0)
    T, M = TWO_PI, 200
    ref = _brute_force(lambda t: H0 + (0.5 + 1.5 * math.cos(t)) * V, 2, T)
    u = orc.build_ut_tridiag(d1, e1, v1, _nodes_cos(T, M, 0.5, 1.5), T, M, route="cheb")
    assert orc.column_error(u, ref) < 1e-7


def test_dimer_time_reversal_symmetry():
    """Real symmetric H0, V and f(T - t) = f(t): U_T equals its transpose."""
    d, e, v = dimer_tridiag(12, 1.0, 0.3)
    T, M = TWO_PI, 60
    U = orc.build_ut_tridiag(d, e, v, _nodes_cos(T, M, 0.5, 1.5), T, M, route="cheb")
    assert np.max(np.abs(U - U.T)) < 1e-12
    assert np.max(np.abs(U - np.eye(len(d)))) > 0.1


def test_tridiag_route_matches_dense_route():
    nb = 7
    d, e, v = dimer_tridiag(nb, 1.0, 0.2)
    H0, V = dimer_dense(nb, 1.0, 0.2)
    T, M = TWO_PI, 20
    f = _nodes_cos(T, M, 0.5, 1.5)
    lo, hi = orc.tridiag_cover(d, e, v, *orc.magnus4_weights(f, T / M))
    Ut = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", e_min=lo, e_max=hi)
    Ud = orc.build_ut(H0, V, f, T, M, route="cheb", e_min=lo, e_max=hi)
    assert orc.column_error(Ut, Ud) < 1e-12


def test_tridiag_cover_is_exact_extremes():
    d, e, v = dimer_tridiag(30, 1.0, 0.01)
    e = e * np.exp(1j * np.linspace(0, 2, len(e)))     # complex off-diagonal
    H0 = np.diag(d) + np.diag(e, 1) + np.diag(np.conj(e), -1)
    T, M = TWO_PI, 9
    a, b = orc.magnus4_weights(_nodes_cos(T, M, 0.5, 1.5), T / M)
    lo, hi = orc.tridiag_cover(d, e, v, a, b)
    K = orc.commutator(H0, np.diag(v).astype(complex))
    evs = [np.linalg.eigvalsh(H0 + a[k] * np.diag(v) + b[k] * K) for k in range(M)]
    assert abs(lo - min(x[0] for x in evs)) < 1e-9
    assert abs(hi - max(x[-1] for x in evs)) < 1e-9


# --- Metrics ----------------------------------------------------------------------------------

def test_quasienergy_distance_properties():
    rng = np.random.default_rng(1)
    th = np.sort(rng.uniform(-math.pi, math.pi, 50))
    T = 2.0
    assert orc.quasienergy_distance(th, th, T) == 0.0
    assert abs(orc.quasienergy_distance(th, th + 1e-7, T) - 1e-7 / T) < 1e-12
    a = np.array([math.pi - 1e-6])
    b = np.array([-math.pi + 1e-6])
    assert abs(orc.quasienergy_distance(a, b, 1.0) - 2e-6) < 1e-12


def test_eigenphases_of_known_unitary():
    rng = np.random.default_rng(2)
    Q = haar_unitary(9, rng)
    th = np.sort(rng.uniform(-3.0, 3.0, 9))
    U = (Q * np.exp(-1j * th)) @ Q.conj().T
    assert np.max(np.abs(orc.eigenphases(U) - th)) < 1e-12


# --- Gradient ---------------------------------------------------------------------------------

@pytest.mark.parametrize("route", ["exact", "cheb"])
def test_gradient_against_central_differences(route):
    rng = np.random.default_rng(33)
    n, M, T = 6, 10, 2.0
    H0, V = gue(n, rng), gue(n, rng)
    f = rng.uniform(-1, 1, M)
    W = haar_unitary(n, rng)
    lo, hi = -6.0, 6.0

    def loss(ff):
        U = orc.build_ut(H0, V, np.stack([ff, ff], 1), T, M, route=route,
                         e_min=lo, e_max=hi, L=20)
        return orc.trace_fidelity_loss(U, W)

    g = orc.grad_piecewise(H0, V, f, T, W, route=route, e_min=lo, e_max=hi, L=20)
    eps = 1e-5
    for k in range(M):
        fp, fm = f.copy(), f.copy()
        fp[k] += eps
        fm[k] -= eps
        fd = (loss(fp) - loss(fm)) / (2 * eps)
        assert abs(fd - g[k]) < 1e-8 + 1e-6 * abs(g[k]), (k, fd, g[k])


def test_gradient_routes_agree_to_truncation():
    rng = np.random.default_rng(34)
    n, M, T = 5, 8, 2.0
    H0, V = gue(n, rng), gue(n, rng)
    f = rng.uniform(-1, 1, M)
    W = haar_unitary(n, rng)
    ge = orc.grad_piecewise(H0, V, f, T, W, route="exact")
    gc = orc.grad_piecewise(H0, V, f, T, W, route="cheb", e_min=-6, e_max=6, tol=1e-14)
    assert np.max(np.abs(ge - gc)) < 1e-11


# --- Work model (Sec. 6, Table 2) -------------------------------------------------------------

def test_work_model_matches_paper_operation_counts():
    """The paper's profiler count, times 4 double-precision operations per
    packed instruction, equals M L complex N^3 products (8 N^3 real
    operations each) to within a few per cent: the hot path is M L zgemm's."""
    rows = np.loadtxt(os.path.join(GOLDEN, "paper_table2_opcounts.txt"))
    M, L = 100, 50
    for N, oc in rows:
        ratio = 4.0 * oc * 1e6 / (M * L * 8.0 * N ** 3)
        assert 1.0 <= ratio < 1.04, (N, ratio)


def test_nearest_unitary_is_the_polar_factor():
    """A = Q P with Q unitary and P Hermitian positive definite has the unique
    polar factor Q; a unitary input is its own polar factor."""
    rng = np.random.default_rng(11)
    n = 12
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(Z)
    S = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    P = scipy.linalg.expm(0.05 * (S + S.conj().T))          # Hermitian positive definite
    assert np.max(np.abs(orc.nearest_unitary(Q @ P) - Q)) < 1e-13
    assert np.max(np.abs(orc.nearest_unitary(Q) - Q)) < 1e-14
    W = orc.nearest_unitary(Q @ P)
    assert orc.unitarity_error(W)[0] < 1e-14


# --- The paper's sixth-order Magnus scheme (three Gauss-Legendre nodes) -----------------------


def _nodes6_cos(T, M):
    return drive_cos(orc.node_times6(T, M), 0.0, 1.0, 1.0)


def test_node_times6_integrate_quintics_exactly():
    """Weights 5/18, 8/18, 5/18 at the three nodes integrate t^5 over each step."""
    T, M = 1.7, 3
    h = T / M
    t = orc.node_times6(T, M)
    w = np.array([5.0, 8.0, 5.0]) / 18.0
    for k in range(M):
        exact = ((k + 1) ** 6 - k ** 6) * h ** 6 / 6.0
        assert abs(h * np.dot(w, t[k] ** 5) - exact) < 1e-13 * max(1.0, exact)


def test_magnus6_static_drive_is_the_plain_exponent():
    """A constant drive: every alpha_j but the first vanishes, H_eff = H0 + f V."""
    H0, V = _rm(5, 41)
    H = orc.magnus6_heff(H0, V, (0.7, 0.7, 0.7), 0.3)
    assert np.abs(H - (H0 + 0.7 * V)).max() < 1e-14


def test_magnus6_commuting_operators_reduce_to_gauss_legendre():
    """Diagonal H0 and V commute: Omega = -i (h H0 + V * integral of f over the
    step), and the three-node rule integrates a quintic drive exactly. A wrong
    alpha_1 or alpha_3 weight breaks this."""
    rng = np.random.default_rng(5)
    H0 = np.diag(rng.normal(size=4)).astype(np.complex128)
    V = np.diag(rng.normal(size=4)).astype(np.complex128)
    c = rng.normal(size=6)
    f = np.polynomial.Polynomial(c)
    t0, h = 0.4, 0.9
    f3 = f(t0 + np.asarray(orc.GL3_C) * h)
    F = f.integ()
    avg = (F(t0 + h) - F(t0)) / h
    H = orc.magnus6_heff(H0, V, f3, h)
    assert np.abs(H - (H0 + avg * V)).max() < 1e-12


def test_magnus6_sixth_order_convergence():
    """e(M) / e(2M) -> 64 against an independent integrator; dropping C_2 or the
    commutator bracket leaves order four (ratio 16), which this rejects."""
    H0, V, Ht = _gue_drive(6, 3)
    T = TWO_PI
    ref = _brute_force(Ht, 6, T)
    errs = []
    for M in (16, 32, 64):
        U = orc.build_ut(H0, V, _nodes6_cos(T, M), T, M, route="exact", scheme="magnus6")
        errs.append(orc.column_error(U, ref))
    r = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(55.0 < x < 70.0 for x in r), r


def test_magnus6_chebyshev_route_matches_exact_route():
    H0, V, _ = _gue_drive(7, 8)
    T, M = TWO_PI, 12
    f = _nodes6_cos(T, M)
    Ue = orc.build_ut(H0, V, f, T, M, route="exact", scheme="magnus6")
    Uc, info = orc.build_ut(H0, V, f, T, M, route="cheb", scheme="magnus6", tol=1e-14,
                            return_info=True)
    assert orc.column_error(Uc, Ue) < 1e-12
    # the exact cover is attained: some step's spectrum touches each end
    lo, hi = info["e_min"], info["e_max"]
    h = T / M
    evs = [np.linalg.eigvalsh(orc.magnus6_heff(H0, V, f[k], h)) for k in range(M)]
    assert min(e[0] for e in evs) == lo and max(e[-1] for e in evs) == hi


# --- Period averages (second propagation round) ----------------------------------------------


def test_period_average_of_stationary_states_is_their_energy():
    """A constant drive: eigenvectors of H0 + f V only gain phases, so their
    period-averaged energy is their eigenvalue."""
    H0, V = _rm(8, 51)
    T, M, fc = 2.0, 7, 0.4
    lam, Q = np.linalg.eigh(H0 + fc * V)
    f = np.full((M, 2), fc)
    avg = orc.period_average(H0, V, f, np.full(M, fc), T, M, Q, route="exact")
    assert np.abs(avg - lam).max() < 1e-12


def test_period_average_commuting_cosine_drive():
    """Diagonal H0, V and f = cos t over a full period: basis states keep their
    populations and the grid mean of cos vanishes, so <H>_T = H0_jj."""
    rng = np.random.default_rng(52)
    n, T, M = 5, TWO_PI, 9
    H0 = np.diag(rng.normal(size=n)).astype(np.complex128)
    V = np.diag(rng.normal(size=n)).astype(np.complex128)
    fg = np.cos(np.arange(M) * T / M)
    avg = orc.period_average(H0, V, _nodes_cos(T, M), fg, T, M, np.eye(n), route="exact")
    assert np.abs(avg - np.diag(H0).real).max() < 1e-12


def test_period_average_trace_over_a_unitary_basis():
    """For any orthonormal basis of states the averages sum to the grid mean of
    Tr H(t_k) = Tr H0 + f(t_k) Tr V (the chain is unitary)."""
    H0, V = _rm(9, 53)
    T, M = TWO_PI, 12
    fg = 0.3 + 0.8 * np.cos(np.arange(M) * T / M)
    W = haar_unitary(9, np.random.default_rng(54))
    avg = orc.period_average(H0, V, _nodes_cos(T, M, 0.3, 0.8), fg, T, M, W, route="exact")
    expect = np.trace(H0).real + np.mean(fg) * np.trace(V).real
    assert abs(avg.sum() - expect) < 1e-11


def test_period_average_matches_the_time_integral_for_a_floquet_state():
    """Floquet states from an independent integrator; their energy averaged over
    the period by integrating d/dt E = <phi|H|phi> along the same ODE, against
    the rectangle rule on a fine grid (spectral for a smooth periodic integrand)."""
    H0, V, Ht = _gue_drive(4, 55)
    T = TWO_PI
    U = _brute_force(Ht, 4, T)
    _, phi = np.linalg.eig(U)
    phi = phi / np.linalg.norm(phi, axis=0)

    def rhs(t, y):
        x = y[:4] + 1j * y[4:8]
        hx = Ht(t) @ x
        dx = -1j * hx
        return np.concatenate([dx.real, dx.imag, [np.real(np.vdot(x, hx))]])

    ref = []
    for j in range(4):
        y0 = np.concatenate([phi[:, j].real, phi[:, j].imag, [0.0]])
        sol = scipy.integrate.solve_ivp(rhs, (0.0, T), y0, method="DOP853", rtol=1e-12, atol=1e-12)
        ref.append(sol.y[-1, -1] / T)
    M = 400
    fg = np.cos(np.arange(M) * T / M)
    avg = orc.period_average(H0, V, _nodes_cos(T, M), fg, T, M, phi, route="exact")
    assert np.abs(avg - np.array(ref)).max() < 1e-7


def test_period_average_tridiag_matches_dense():
    d, e, v = dimer_tridiag(11, 1.0, 0.3)
    n, T, M = 12, TWO_PI, 10
    f = _nodes_cos(T, M, 0.5, 1.5)
    fg = 0.5 + 1.5 * np.cos(np.arange(M) * T / M)
    X0 = haar_unitary(n, np.random.default_rng(56))[:, :3]
    H0, V, _ = orc.tridiag_matrices(d, e, v)
    a = orc.period_average_tridiag(d, e, v, f, fg, T, M, X0, route="exact")
    b = orc.period_average(H0.toarray(), V.toarray(), f, fg, T, M, X0, route="exact")
    assert np.abs(a - b).max() < 1e-12


# --- Commutator-free fourth-order scheme ------------------------------------------------------


def test_cf4_fourth_order_and_factor_order():
    """e(M) / e(2M) -> 16 against an independent integrator; applying the two
    half-step exponentials in the other order flips the sign of the generated
    commutator term and leaves order two (ratio 4)."""
    H0, V, Ht = _gue_drive(6, 3)
    T = TWO_PI
    ref = _brute_force(Ht, 6, T)
    errs, errs_sw = [], []
    for M in (25, 50, 100):
        f = _nodes_cos(T, M)
        errs.append(orc.column_error(orc.build_ut(H0, V, f, T, M, route="exact", scheme="cf4"), ref))
        U = np.eye(6, dtype=np.complex128)
        h = T / M
        ops = orc.cf4_exponents(H0, V, f)
        for k in range(M):            # the two factors swapped
            for op in (ops[2 * k + 1], ops[2 * k]):
                U = orc.exact_step(op, h / 2, U)
        errs_sw.append(orc.column_error(U, ref))
    r = [errs[i] / errs[i + 1] for i in range(2)]
    rs = [errs_sw[i] / errs_sw[i + 1] for i in range(2)]
    assert all(14.0 < x < 18.0 for x in r), r
    assert all(3.5 < x < 4.6 for x in rs), rs


def test_cf4_commuting_operators_reduce_to_gauss_legendre():
    """Commuting H0, V: the product is exp(-i h (H0 + V (f1 + f2) / 2)), the
    two-node rule, exact for a cubic drive."""
    rng = np.random.default_rng(57)
    H0 = np.diag(rng.normal(size=4)).astype(np.complex128)
    V = np.diag(rng.normal(size=4)).astype(np.complex128)
    f = np.polynomial.Polynomial(rng.normal(size=4))
    T, M = 1.3, 3
    fn = f(orc.node_times(T, M))
    U = orc.build_ut(H0, V, fn, T, M, route="exact", scheme="cf4")
    F = f.integ()
    expect = np.diag(np.exp(-1j * (np.diag(H0) * T + np.diag(V) * (F(T) - F(0.0)))))
    assert np.abs(U - expect).max() < 1e-12


def test_cf4_tridiag_matches_dense_and_chebyshev_matches_exact():
    d, e, v = dimer_tridiag(11, 1.0, 0.3)
    T, M = TWO_PI, 10
    f = _nodes_cos(T, M, 0.5, 1.5)
    H0, V, _ = orc.tridiag_matrices(d, e, v)
    Ut = orc.build_ut_tridiag(d, e, v, f, T, M, route="cheb", tol=1e-14, scheme="cf4")
    Ud = orc.build_ut(H0.toarray(), V.toarray(), f, T, M, route="exact", scheme="cf4")
    assert orc.column_error(Ut, Ud) < 1e-11


# --- Several drive terms ----------------------------------------------------------------------


def _two_drives(seed):
    H0, V1 = _rm(6, seed)
    V2 = _rm(6, seed + 1)[0]
    return H0, V1, V2


@pytest.mark.parametrize("scheme", ["magnus4", "cf4"])
def test_two_drive_terms_fourth_order(scheme):
    """H0 + cos t V1 + sin 2t V2: ratio 16 per halving of h against DOP853. A
    wrong sign or weight of the [V1, V2] term leaves order two."""
    H0, V1, V2 = _two_drives(70)
    T = TWO_PI
    ref = _brute_force(lambda t: H0 + math.cos(t) * V1 + math.sin(2 * t) * V2, 6, T)
    errs = []
    for M in (25, 50, 100):
        t = orc.node_times(T, M)
        f = np.stack([np.cos(t), np.sin(2 * t)], -1)
        errs.append(orc.column_error(orc.build_ut(H0, [V1, V2], f, T, M, route="exact",
                                                  scheme=scheme), ref))
    r = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(14.0 < x < 18.0 for x in r), r


@pytest.mark.parametrize("scheme", ["magnus4", "cf4"])
def test_two_drive_terms_reduce_to_one(scheme):
    """V2 = V1 with f1 + f2 = f is the one-term model with f; V2 = 0 ignores f2."""
    H0, V1, _ = _two_drives(71)
    T, M = TWO_PI, 9
    t = orc.node_times(T, M)
    fa, fb = np.cos(t), 0.3 * np.sin(t)
    U1 = orc.build_ut(H0, V1, fa + fb, T, M, route="exact", scheme=scheme)
    U2 = orc.build_ut(H0, [V1, V1], np.stack([fa, fb], -1), T, M, route="exact", scheme=scheme)
    assert orc.column_error(U2, U1) < 1e-12
    Ua = orc.build_ut(H0, V1, fa, T, M, route="exact", scheme=scheme)
    U3 = orc.build_ut(H0, [V1, np.zeros_like(V1)], np.stack([fa, fb], -1), T, M, route="exact",
                      scheme=scheme)
    assert orc.column_error(U3, Ua) < 1e-12


# --- accuracy of individual Floquet states (Sec. 7, Eq. (error)) ----------------------------------

def _fold(q, T):
    """Quasienergies folded into (-pi/T, pi/T]."""
    period = 2.0 * math.pi / T
    return q - period * np.round(q / period + 1e-15)


def test_state_errors_vanish_for_commuting_operators_with_the_closed_form_quasienergies():
    """Diagonal H0, V and f = eps0 + eps1 cos t over a full period: every step
    commutes and the Gauss-Legendre sums of cos vanish, so U_T(h) = U_T(h/2) =
    diag(exp(-i (E_j + eps0 v_j) T)): the Floquet states are the basis states
    (sigma = 0, dq = 0) and the quasienergies are E_j + eps0 v_j modulo 2 pi / T."""
    rng = np.random.default_rng(71)
    n, T, M, eps0 = 6, TWO_PI, 10, 0.3
    E = np.sort(rng.uniform(-0.45, 0.45, n))
    v = rng.uniform(-0.2, 0.2, n)
    H0, V = np.diag(E).astype(complex), np.diag(v).astype(complex)
    U = orc.build_ut(H0, V, _nodes_cos(T, M, eps0), T, M, route="exact")
    U2 = orc.build_ut(H0, V, _nodes_cos(T, 2 * M, eps0), T, 2 * M, route="exact")
    sigma, dq, q = orc.floquet_state_errors(U, U2, T)
    assert sigma.max() < 1e-13 and dq.max() < 1e-13
    expect = np.sort(_fold(E + eps0 * v, T))
    assert np.abs(np.sort(_fold(q, T)) - expect).max() < 1e-13


def test_state_errors_against_an_independent_integrator():
    """Magnus-4 Floquet states of a random model: the error of each state of
    U_T(h) against the exact states (a DOP853 propagator) is estimated by its
    difference from U_T(h/2) as the paper does: with a fourth-order error C h^4,
    phi(h) - phi(h/2) = (15/16) C h^4, so the quasienergy estimate is 15/16 of the
    true error and the overlap deficiency, quadratic in the state error,
    (15/16)^2 of it. A state that is not matched to its partner, a missing
    normalisation or a wrong phase convention breaks both ratios."""
    H0, V = _rm(5, 72)
    T, M = TWO_PI, 24
    f = _nodes_cos(T, M)
    U = orc.build_ut(H0, V, f, T, M, route="exact")
    U2 = orc.build_ut(H0, V, _nodes_cos(T, 2 * M), T, 2 * M, route="exact")
    Uex = _brute_force(lambda t: H0 + math.cos(t) * V, 5, T)
    s_est, d_est, _ = orc.floquet_state_errors(U, U2, T)
    s_true, d_true, _ = orc.floquet_state_errors(U, Uex, T)
    assert d_true.min() > 1e-9 and s_true.min() > 1e-17   # errors resolved above round-off
    np.testing.assert_allclose(d_est / d_true, 15.0 / 16.0, rtol=0.03)
    np.testing.assert_allclose(s_est / s_true, (15.0 / 16.0) ** 2, rtol=0.06)


def test_state_errors_fall_with_the_fourth_power_of_the_step():
    """Halving h again: quasienergy differences fall by 16 (order four), overlap
    deficiencies by 256."""
    H0, V = _rm(5, 73)
    T = TWO_PI
    Us = [orc.build_ut(H0, V, _nodes_cos(T, m), T, m, route="exact") for m in (20, 40, 80)]
    s1, d1, _ = orc.floquet_state_errors(Us[0], Us[1], T)
    s2, d2, _ = orc.floquet_state_errors(Us[1], Us[2], T)
    assert 14.0 < np.median(d1 / d2) < 18.0
    assert 180.0 < np.median(s1 / s2) < 330.0
