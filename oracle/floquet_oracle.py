"""Plain FP64 CPU oracle of the Floquet-operator build (NumPy / SciPy).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package. It shares no
code with the HIP path (no kernels, headers, tables or helpers).

What it computes (Laptyeva et al., "Calculating Floquet states of large quantum
systems", arXiv:1508.07621):

* the Floquet operator U_T of H(t) = H0 + f(t) V (Sec. 3, Eq. (13)) as a chain
  of single-step exponentials, later steps acting from the left on column
  states (Sec. 2, Eq. (9); time grid t_k = k T / M);
* each step's Hamiltonian from the Magnus series (Sec. 2, Eq. (8)) truncated
  after its commutator term with two-point Gauss-Legendre quadrature (4th
  order), or by the paper's own sixth-order midpoint scheme (Sec. 3, Eq. (14)
  with its alpha_j and C_1, C_2), the alpha_j taken from three-point
  Gauss-Legendre quadrature;
* each exponential either exactly (Hermitian eigendecomposition, "route E") or
  by the paper's Chebyshev recurrence (Sec. 2, Eqs. (10)-(12), "route C"), on
  the spectrum rescaled into [-1, 1] (Eq. (11));
* quasienergies from the eigenvalues of U_T (Sec. 2, Eq. (4));
* the period average of the energy of propagated states (the second round of
  Sec. 3, Eq. (average) with A(t) = H(t)) by the rectangle rule on the step grid;
* the accuracy of individual Floquet states (Sec. 7, Eq. (error)): each state of
  U_T(h) against the best-matching state of U_T(h/2), as an overlap deficiency
  and a quasienergy difference (the printed overlap contains the eigenphase);
* the gradient of a trace-fidelity loss with respect to piecewise-constant drive
  amplitudes (not in the paper; exact Daleckii-Krein derivative of the chain).

Readings of the paper that this file takes (each pinned by a test):
* hbar = 1; the Magnus series is that of the generator A = -i H (the printed
  series omits the -i factors on its commutator terms);
* the rescaled operator of Eqs. (10)-(12) is (H_eff - beta) / dE with
  beta = (E_max + E_min)/2, dE = (E_max - E_min)/2, R = h dE, global phase
  exp(-i beta h);
* the spectral interval must contain the spectrum of every step's H_eff;
* in the sixth-order scheme the alpha_j are the three-point Gauss-Legendre
  combinations of A(t) = -i H(t) at the nodes 1/2 -/+ sqrt(15)/10 and 1/2:
  alpha_1 = h A_2, alpha_2 = (sqrt(15) h / 3)(A_3 - A_1),
  alpha_3 = (10 h / 3)(A_3 - 2 A_2 + A_1); these agree with the printed
  scaled midpoint derivatives to leading order, and with them the scheme has
  order six (with the exact derivatives it has order four).

Parity pins: every function here is pinned by a test in tests/test_oracle_pins.py
against closed forms, a brute-force ODE integration, group theory (spin
representation of the dimer) or the Jacobi-Anger identity; none is unpinned.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.special

__all__ = [
    "GL2_C1", "GL2_C2", "node_times", "commutator", "magnus4_weights", "magnus4_heff",
    "bessel_coefficients", "choose_L", "rescale", "weyl_cover", "tridiag_cover",
    "exact_step", "chebyshev_step", "build_ut", "build_ut_tridiag", "tridiag_matrices",
    "column_error", "unitarity_error", "nearest_unitary", "eigenphases",
    "quasienergy_distance",
    "trace_fidelity_loss", "grad_piecewise", "chebyshev_polynomial_values",
    "GL3_C", "node_times6", "magnus6_omega", "magnus6_heff", "exact_cover",
    "period_average", "period_average_tridiag", "CF4_A1", "CF4_A2", "cf4_exponents",
    "magnus4_heff_drives", "floquet_state_errors",
]

# ---------------------------------------------------------------------------
# Magnus-4 with two Gauss-Legendre nodes
# ---------------------------------------------------------------------------

#: Gauss-Legendre nodes on [0, 1]; c1 is the earlier one.
GL2_C1 = 0.5 - math.sqrt(3.0) / 6.0
GL2_C2 = 0.5 + math.sqrt(3.0) / 6.0


def node_times(T: float, M: int) -> np.ndarray:
    """Sampling times of the drive, shape (M, 2): t_{k-1} + c_{1,2} h, h = T/M.

    The step grid t_k = k T / M is the one of Sec. 2, Eq. (9).
    """
    h = T / M
    k = np.arange(M, dtype=np.float64)
    return np.stack([(k + GL2_C1) * h, (k + GL2_C2) * h], axis=1)


def commutator(H0: np.ndarray, V: np.ndarray) -> np.ndarray:
    """K = -i [H0, V], the time-independent commutator needed by the Magnus
    series of H0 + f(t) V (Sec. 3: only commutators of the fixed operators
    appear, computed once). K is Hermitian when H0 and V are."""
    return -1j * (H0 @ V - V @ H0)


def magnus4_weights(f_nodes: np.ndarray, h: float) -> Tuple[np.ndarray, np.ndarray]:
    """Per-step scalars (a_k, b_k) of H_eff,k = H0 + a_k V + b_k K.

    Derivation, for the generator A(t) = -i H(t) and one step of length h
    (Sec. 2, Eq. (8), first two terms): the integral term with Gauss-Legendre
    quadrature is (h/2)(A_1 + A_2); the double-integral commutator term,
    approximated consistently to the same order, is (sqrt(3) h^2 / 12)[A_2, A_1].
    With A_j = -i (H0 + f_j V), [A_2, A_1] = -(f_1 - f_2)[H0, V], so the step
    operator Omega_A = -i h H_eff with
        a_k = (f_1 + f_2) / 2,   b_k = sqrt(3) h (f_1 - f_2) / 12,
    f_1 being the drive at the earlier node.
    """
    f = np.asarray(f_nodes, dtype=np.float64).reshape(-1, 2)
    a = 0.5 * (f[:, 0] + f[:, 1])
    b = math.sqrt(3.0) * h * (f[:, 0] - f[:, 1]) / 12.0
    return a, b


def magnus4_heff(H0, V, K, a: float, b: float):
    """H_eff = H0 + a V + b K (dense or scipy.sparse operands)."""
    return H0 + a * V + b * K


def _drive(H0, Vs, fs):
    """H0 + sum_s f_s V_s (one or several drive terms)."""
    H = H0
    for f, V in zip(fs, Vs):
        H = H + f * V
    return H


def magnus4_heff_drives(H0, Vs, f1s, f2s, h: float) -> np.ndarray:
    """H_eff of one step for H(t) = H0 + sum_s f_s(t) V_s (the several-term form
    Sec. 3 mentions), from the same truncation as magnus4_weights written out with
    matrices: Omega = (h/2)(A_1 + A_2) + (sqrt(3) h^2 / 12)[A_2, A_1],
    A_j = -i H(node j), H_eff = i Omega / h. f1s, f2s: the drive terms at the
    earlier and the later node."""
    A1 = -1j * _drive(H0, Vs, f1s)
    A2 = -1j * _drive(H0, Vs, f2s)
    om = 0.5 * h * (A1 + A2) + (math.sqrt(3.0) * h * h / 12.0) * (A2 @ A1 - A1 @ A2)
    H = 1j * om / h
    return 0.5 * (H + H.conj().T)


# ---------------------------------------------------------------------------
# The paper's sixth-order Magnus scheme (Sec. 3, Eq. (14)), three-point
# Gauss-Legendre alpha_j
# ---------------------------------------------------------------------------

#: Nodes of the three-point Gauss-Legendre rule on [0, 1], in time order.
GL3_C = (0.5 - math.sqrt(15.0) / 10.0, 0.5, 0.5 + math.sqrt(15.0) / 10.0)


def node_times6(T: float, M: int) -> np.ndarray:
    """Sampling times of the drive for the sixth-order scheme, shape (M, 3):
    t_{k-1} + c_j h for the three Gauss-Legendre nodes, h = T / M."""
    h = T / M
    k = np.arange(M, dtype=np.float64)[:, None]
    return (k + np.asarray(GL3_C)[None, :]) * h


def magnus6_omega(H0: np.ndarray, V: np.ndarray, f3, h: float) -> np.ndarray:
    """Omega of one step of length h for the generator A(t) = -i (H0 + f(t) V),
    by the paper's scheme (Sec. 3, Eq. (14)):
        Omega = alpha_1 + alpha_3 / 12 + [-20 alpha_1 - alpha_3 + C_1, alpha_2 + C_2] / 240,
        C_1 = [alpha_1, alpha_2],  C_2 = -[alpha_1, 2 alpha_3 + C_1] / 60,
    with the alpha_j from the drive f3 = (f_1, f_2, f_3) at the three nodes
    (reading in the module header). Dense matrix arithmetic, as written."""
    f1, f2, f3_ = (float(x) for x in f3)
    A1 = -1j * (H0 + f1 * V)
    A2 = -1j * (H0 + f2 * V)
    A3 = -1j * (H0 + f3_ * V)
    al1 = h * A2
    al2 = (math.sqrt(15.0) * h / 3.0) * (A3 - A1)
    al3 = (10.0 * h / 3.0) * (A3 - 2.0 * A2 + A1)

    def comm(X, Y):
        return X @ Y - Y @ X

    C1 = comm(al1, al2)
    C2 = -comm(al1, 2.0 * al3 + C1) / 60.0
    return al1 + al3 / 12.0 + comm(-20.0 * al1 - al3 + C1, al2 + C2) / 240.0


def magnus6_heff(H0: np.ndarray, V: np.ndarray, f3, h: float) -> np.ndarray:
    """H_eff with exp(Omega) = exp(-i h H_eff): H_eff = i Omega / h, made exactly
    Hermitian by averaging with its adjoint (Omega is anti-Hermitian up to
    rounding)."""
    H = 1j * magnus6_omega(H0, V, f3, h) / h
    return 0.5 * (H + H.conj().T)


def exact_cover(Heffs) -> Tuple[float, float]:
    """min / max over the given Hermitian matrices of their exact extreme
    eigenvalues (LAPACK): the tightest interval containing every spectrum."""
    lo, hi = np.inf, -np.inf
    for H in Heffs:
        ev = np.linalg.eigvalsh(H)
        lo = min(lo, float(ev[0]))
        hi = max(hi, float(ev[-1]))
    return lo, hi


# ---------------------------------------------------------------------------
# Commutator-free fourth-order scheme (the variant Sec. 2 and Sec. 8 name)
# ---------------------------------------------------------------------------

#: Weights of the two-exponential commutator-free scheme on the two
#: Gauss-Legendre nodes: E = exp(-i h (A2 H1 + A1 H2)) exp(-i h (A1 H1 + A2 H2)).
CF4_A1 = 0.25 + math.sqrt(3.0) / 6.0
CF4_A2 = 0.25 - math.sqrt(3.0) / 6.0


def cf4_exponents(H0, V, f_nodes):
    """See _cf4_exponents; V may be a list of drive matrices, with f_nodes of shape
    (M, 2, S)."""
    if isinstance(V, (list, tuple)):
        f = np.asarray(f_nodes, dtype=np.float64).reshape(-1, 2, len(V))
        ops = []
        for k in range(f.shape[0]):
            H1 = _drive(H0, V, f[k, 0])
            H2 = _drive(H0, V, f[k, 1])
            ops.append(2.0 * (CF4_A1 * H1 + CF4_A2 * H2))   # acts first
            ops.append(2.0 * (CF4_A2 * H1 + CF4_A1 * H2))
        return ops
    return _cf4_exponents(H0, V, f_nodes)


def _cf4_exponents(H0, V, f_nodes):
    """The step's two exponents as a list of Hermitian operators, each to be
    exponentiated over half a step, in the order they act (earlier first):
    exp(-i h (a H1 + b H2)) = exp(-i (h/2) 2 (a H1 + b H2)) with a + b = 1/2 and
    H_j = H0 + f_j V at the step's two Gauss-Legendre nodes (f1 earlier).
    BCH of the product reproduces the Magnus-4 exponent (h/2)(A1 + A2) +
    (sqrt(3) h^2 / 12)[A2, A1] of A = -i H up to O(h^5)."""
    f = np.asarray(f_nodes, dtype=np.float64).reshape(-1, 2)
    ops = []
    for f1, f2 in f:
        H1 = H0 + f1 * V
        H2 = H0 + f2 * V
        ops.append(2.0 * (CF4_A1 * H1 + CF4_A2 * H2))   # acts first
        ops.append(2.0 * (CF4_A2 * H1 + CF4_A1 * H2))
    return ops


# ---------------------------------------------------------------------------
# Chebyshev expansion (Sec. 2, Eqs. (10)-(12))
# ---------------------------------------------------------------------------

def bessel_coefficients(R: float, L: int) -> np.ndarray:
    """Real expansion weights of Eq. (12): a_0 = J_0(R), a_l = 2 J_l(R), l = 1..L.

    Bessel values from scipy.special.jv (AMOS), independent of any recurrence.
    """
    l = np.arange(L + 1, dtype=np.float64)
    a = 2.0 * scipy.special.jv(l, R)
    a[0] *= 0.5
    return a


def choose_L(R: float, tol: float) -> int:
    """Smallest L with 2 * sum_{l > L} |J_l(R)| <= tol.

    Because |T_l(x)| <= 1 on [-1, 1], this bounds the truncation error of the
    series of Eq. (12) for any operator whose rescaled spectrum lies in [-1, 1].
    """
    lmax = int(R + 40.0 + 12.0 * max(R, 1.0) ** (1.0 / 3.0)) + 64
    j = np.abs(scipy.special.jv(np.arange(lmax + 1, dtype=np.float64), R))
    tail = 2.0 * np.cumsum(j[::-1])[::-1]          # tail[l] = 2 sum_{m >= l} |J_m|
    for L in range(0, lmax):
        if tail[L + 1] <= tol:
            return max(L, 1)
    raise ValueError("choose_L: R too large for the table")


def rescale(e_min: float, e_max: float, h: float):
    """beta, dE and R = h dE for the spectral interval [e_min, e_max] (Eq. (11))."""
    dE = 0.5 * (e_max - e_min)
    beta = 0.5 * (e_max + e_min)
    return beta, dE, h * dE


def chebyshev_step(Heff, beta: float, dE: float, h: float, a: np.ndarray, X: np.ndarray) -> np.ndarray:
    """One single-step propagation by the paper's recurrence (Eqs. (10)-(12)):
    phi_0 = X, phi_1 = -i Ht phi_0, phi_{l+1} = -2 i Ht phi_l + phi_{l-1},
    X_new = exp(-i beta h) sum_l a_l phi_l, with Ht = (Heff - beta) / dE.
    Heff may be dense or scipy.sparse.
    """
    L = len(a) - 1

    def apply(P):
        return (Heff @ P - beta * P) / dE

    phi_prev = X
    acc = a[0] * phi_prev
    phi = -1j * apply(phi_prev)
    acc = acc + a[1] * phi
    for l in range(1, L):
        phi_next = -2j * apply(phi) + phi_prev
        acc = acc + a[l + 1] * phi_next
        phi_prev, phi = phi, phi_next
    return np.exp(-1j * beta * h) * acc


def exact_step(Heff: np.ndarray, h: float, X: np.ndarray) -> np.ndarray:
    """exp(-i h Heff) X by the Hermitian eigendecomposition (route E)."""
    lam, Q = np.linalg.eigh(Heff)
    return Q @ (np.exp(-1j * h * lam)[:, None] * (Q.conj().T @ X))


def chebyshev_polynomial_values(x: np.ndarray, a: np.ndarray, beta: float, h: float):
    """Scalar p(x) = exp(-i beta h) sum_l a_l (-i)^l T_l(x) and p'(x), by the
    three-term recurrences of T_l and of U_l (T_l' = l U_{l-1})."""
    x = np.asarray(x, dtype=np.float64)
    L = len(a) - 1
    t_prev, t = np.ones_like(x), x.copy()
    u_prev, u = np.zeros_like(x), np.ones_like(x)      # U_{-1}, U_0
    p = a[0] * t_prev + 0j
    dp = np.zeros_like(x) + 0j
    if L >= 1:
        p = p + a[1] * (-1j) * t
        dp = dp + a[1] * (-1j) * u
    for l in range(1, L):
        t_prev, t = t, 2.0 * x * t - t_prev
        u_prev, u = u, 2.0 * x * u - u_prev
        p = p + a[l + 1] * (-1j) ** (l + 1) * t
        dp = dp + a[l + 1] * (-1j) ** (l + 1) * (l + 1) * u
    ph = np.exp(-1j * beta * h)
    return ph * p, ph * dp


# ---------------------------------------------------------------------------
# Spectral interval
# ---------------------------------------------------------------------------

def weyl_cover(H0, V, K, a, b) -> Tuple[float, float]:
    """An interval containing spec(H0 + a_k V + b_k K) for every k, from Weyl's
    inequalities and the extreme eigenvalues of H0, V and K."""
    l0 = np.linalg.eigvalsh(H0)
    lv = np.linalg.eigvalsh(V)
    nk = float(np.max(np.abs(np.linalg.eigvalsh(K))))
    a = np.asarray(a)
    b = np.asarray(b)
    lo = l0[0] + np.minimum(a * lv[0], a * lv[-1]) - np.abs(b) * nk
    hi = l0[-1] + np.maximum(a * lv[0], a * lv[-1]) + np.abs(b) * nk
    return float(lo.min()), float(hi.max())


def tridiag_matrices(h0_diag, h0_off, v_diag):
    """Sparse H0 (Hermitian tridiagonal), V (diagonal) and K = -i (H0 V - V H0)."""
    n = len(h0_diag)
    off = np.asarray(h0_off, dtype=np.complex128)
    H0 = scipy.sparse.diags([np.conj(off), np.asarray(h0_diag, np.complex128), off], [-1, 0, 1],
                            shape=(n, n), format="csr")
    V = scipy.sparse.diags([np.asarray(v_diag, np.complex128)], [0], shape=(n, n), format="csr")
    K = (-1j * (H0 @ V - V @ H0)).tocsr()
    return H0, V, K


def tridiag_cover(h0_diag, h0_off, v_diag, a, b) -> Tuple[float, float]:
    """Global min / max over steps of the exact extreme eigenvalues of the
    Hermitian tridiagonal H_eff,k (LAPACK on the real matrix with |offdiag|,
    which a diagonal unitary similarity relates to the complex one)."""
    H0, V, K = tridiag_matrices(h0_diag, h0_off, v_diag)
    lo, hi = np.inf, -np.inf
    for ak, bk in zip(np.atleast_1d(a), np.atleast_1d(b)):
        Hk = (H0 + ak * V + bk * K).tocsr()
        d = Hk.diagonal().real
        e = np.abs(Hk.diagonal(1))
        if len(d) == 1:
            ev = d
        else:
            ev = scipy.linalg.eigvalsh_tridiagonal(d, e, select="i", select_range=(0, 0))
            ev = np.concatenate([ev, scipy.linalg.eigvalsh_tridiagonal(
                d, e, select="i", select_range=(len(d) - 1, len(d) - 1))])
        lo = min(lo, float(ev.min()))
        hi = max(hi, float(ev.max()))
    return lo, hi


# ---------------------------------------------------------------------------
# The chain (Sec. 2, Eq. (9); Sec. 3, the algorithm)
# ---------------------------------------------------------------------------

def _chain(Hk_of, M: int, T: float, route: str, X0, e_min, e_max, L, tol, k_range=None):
    h = T / M
    info: Dict[str, float] = {}
    if route == "cheb":
        beta, dE, R = rescale(e_min, e_max, h)
        if L is None:
            L = choose_L(R, tol)
        a = bessel_coefficients(R, L)
        info.update(beta=beta, dE=dE, R=R, L=L)
    X = X0
    k0, k1 = (0, M) if k_range is None else k_range
    for k in range(k0, k1):
        Hk = Hk_of(k)
        if route == "exact":
            Hd = Hk.toarray() if scipy.sparse.issparse(Hk) else Hk
            X = exact_step(Hd, h, X)
        elif route == "cheb":
            X = chebyshev_step(Hk, beta, dE, h, a, X)
        else:
            raise ValueError(route)
    return X, info


def build_ut(H0: np.ndarray, V: np.ndarray, f_nodes: np.ndarray, T: float, M: int,
             route: str = "cheb", e_min: Optional[float] = None, e_max: Optional[float] = None,
             L: Optional[int] = None, tol: float = 1e-12, X0: Optional[np.ndarray] = None,
             return_info: bool = False, k_range: Optional[Tuple[int, int]] = None,
             scheme: str = "magnus4"):
    """U_T (or U_T X0) of the dense model H0 + f(t) V.

    scheme "magnus4": f_nodes has shape (M, 2), the drive at the two
    Gauss-Legendre nodes of each step (node_times); scheme "magnus6" (the
    paper's Eq. (14)): shape (M, 3) at the three nodes of node_times6; scheme
    "cf4": the commutator-free product of two half-step exponentials
    (cf4_exponents) on the nodes of node_times, run as 2M steps of h/2 (the
    Chebyshev route's R is that of h/2).
    route "exact" exponentiates each H_eff exactly; route "cheb" uses the
    Chebyshev recurrence with the interval [e_min, e_max] (default: the Weyl
    cover for magnus4, the exact cover for magnus6) and order L (default:
    choose_L(R, tol)). k_range = (k0, k1) applies only steps k0+1 .. k1 to X0:
    the propagator from t_k0 to t_k1, since single-step propagators compose
    (Sec. 2).
    """
    H0 = np.asarray(H0, np.complex128)
    n = H0.shape[0]
    h = T / M
    if isinstance(V, (list, tuple)):  # several drive terms, f_nodes (M, 2, S)
        Vs = [np.asarray(v, np.complex128) for v in V]
        X0 = np.eye(n, dtype=np.complex128) if X0 is None else np.asarray(X0, np.complex128)
        f = np.asarray(f_nodes, np.float64).reshape(M, 2, len(Vs))
        if scheme == "cf4":
            ops = cf4_exponents(H0, Vs, f)
            Mc, kr = 2 * M, None if k_range is None else (2 * k_range[0], 2 * k_range[1])
        elif scheme == "magnus4":
            ops = [magnus4_heff_drives(H0, Vs, f[k, 0], f[k, 1], h) for k in range(M)]
            Mc, kr = M, k_range
        else:
            raise ValueError(scheme)
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = exact_cover(ops)
        U, info = _chain(ops.__getitem__, Mc, T, route, X0, e_min, e_max, L, tol, kr)
        info.update(e_min=e_min, e_max=e_max)
        return (U, info) if return_info else U
    V = np.asarray(V, np.complex128)
    if scheme == "magnus6":
        f3 = np.asarray(f_nodes, np.float64).reshape(M, 3)
        Hs = [magnus6_heff(H0, V, f3[k], h) for k in range(M)]
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = exact_cover(Hs)
        Hk_of = Hs.__getitem__
    elif scheme == "magnus4":
        K = commutator(H0, V)
        a, b = magnus4_weights(f_nodes, h)
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = weyl_cover(H0, V, K, a, b)

        def Hk_of(k):
            return magnus4_heff(H0, V, K, a[k], b[k])
    elif scheme == "cf4":
        # 2M half-steps, each the exponential of one of cf4_exponents
        ops = cf4_exponents(H0, V, f_nodes)
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = exact_cover(ops)
        X0 = np.eye(n, dtype=np.complex128) if X0 is None else np.asarray(X0, np.complex128)
        kr = None if k_range is None else (2 * k_range[0], 2 * k_range[1])
        U, info = _chain(ops.__getitem__, 2 * M, T, route, X0, e_min, e_max, L, tol, kr)
        info.update(e_min=e_min, e_max=e_max)
        return (U, info) if return_info else U
    else:
        raise ValueError(scheme)
    X0 = np.eye(n, dtype=np.complex128) if X0 is None else np.asarray(X0, np.complex128)
    U, info = _chain(Hk_of, M, T, route, X0, e_min, e_max, L, tol, k_range)
    info.update(e_min=e_min, e_max=e_max)
    return (U, info) if return_info else U


def build_ut_tridiag(h0_diag, h0_off, v_diag, f_nodes, T: float, M: int, route: str = "cheb",
                     e_min: Optional[float] = None, e_max: Optional[float] = None,
                     L: Optional[int] = None, tol: float = 1e-12, X0: Optional[np.ndarray] = None,
                     return_info: bool = False, k_range: Optional[Tuple[int, int]] = None,
                     scheme: str = "magnus4"):
    """Same as build_ut for a Hermitian tridiagonal H0 and a diagonal V, with
    sparse products (default interval: tridiag_cover); schemes "magnus4" and
    "cf4"."""
    n = len(h0_diag)
    h = T / M
    H0, V, K = tridiag_matrices(h0_diag, h0_off, v_diag)
    if scheme == "cf4":
        ops = [op.tocsr() for op in cf4_exponents(H0, V, f_nodes)]
        if route == "cheb" and (e_min is None or e_max is None):
            # each half-step operator is H0 + a V with a = 2 (a1 f1 + a2 f2) or swapped
            f = np.asarray(f_nodes, np.float64).reshape(-1, 2)
            asub = np.stack([2 * (CF4_A1 * f[:, 0] + CF4_A2 * f[:, 1]),
                             2 * (CF4_A2 * f[:, 0] + CF4_A1 * f[:, 1])], 1).ravel()
            e_min, e_max = tridiag_cover(h0_diag, h0_off, v_diag, asub, np.zeros_like(asub))
        X0 = np.eye(n, dtype=np.complex128) if X0 is None else np.asarray(X0, np.complex128)
        kr = None if k_range is None else (2 * k_range[0], 2 * k_range[1])
        U, info = _chain(ops.__getitem__, 2 * M, T, route, X0, e_min, e_max, L, tol, kr)
        info.update(e_min=e_min, e_max=e_max)
        return (U, info) if return_info else U
    if scheme != "magnus4":
        raise ValueError(scheme)
    a, b = magnus4_weights(f_nodes, h)
    if route == "cheb" and (e_min is None or e_max is None):
        e_min, e_max = tridiag_cover(h0_diag, h0_off, v_diag, a, b)
    X0 = np.eye(n, dtype=np.complex128) if X0 is None else np.asarray(X0, np.complex128)
    U, info = _chain(lambda k: (H0 + a[k] * V + b[k] * K).tocsr(), M, T, route, X0,
                     e_min, e_max, L, tol, k_range)
    info.update(e_min=e_min, e_max=e_max)
    return (U, info) if return_info else U


# ---------------------------------------------------------------------------
# Second propagation round: period averages (Sec. 3, Eq. (average))
# ---------------------------------------------------------------------------

def _period_average(Hk_of, Hgrid_of, M, T, X0, route, e_min, e_max, L, tol, spp=1):
    """(1/M) sum_{k<M} <x_k|H(t_k)|x_k> / <x_k|x_k> per column, x_k the column
    after k steps: Eq. (average) with A(t) = H(t) by the rectangle rule on the
    step grid t_k = k h. A step is spp exponentials of Hk_of (h / spp each)."""
    X = np.asarray(X0, np.complex128)
    acc = np.zeros(X.shape[1])
    for k in range(M):
        HX = Hgrid_of(k) @ X
        acc += np.real(np.sum(X.conj() * HX, axis=0)) / np.sum(np.abs(X) ** 2, axis=0)
        X, _ = _chain(Hk_of, spp * M, T, route, X, e_min, e_max, L, tol,
                      (spp * k, spp * (k + 1)))
    return acc / M


def period_average(H0, V, f_nodes, f_grid, T: float, M: int, X0, scheme: str = "magnus4",
                   route: str = "cheb", e_min=None, e_max=None, L=None, tol: float = 1e-12):
    """Period-averaged energy of the columns of X0 for the dense model (Eq. (average)
    with A(t) = H0 + f(t) V); f_grid[k] = f(k h). The steps are those of build_ut
    with the same arguments (f_nodes at the scheme's nodes)."""
    H0 = np.asarray(H0, np.complex128)
    h = T / M
    if isinstance(V, (list, tuple)):  # several drive terms: f_nodes (M, 2, S), f_grid (M, S)
        Vs = [np.asarray(v, np.complex128) for v in V]
        f = np.asarray(f_nodes, np.float64).reshape(M, 2, len(Vs))
        if scheme == "cf4":
            ops, spp = cf4_exponents(H0, Vs, f), 2
        elif scheme == "magnus4":
            ops, spp = [magnus4_heff_drives(H0, Vs, f[k, 0], f[k, 1], h) for k in range(M)], 1
        else:
            raise ValueError(scheme)
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = exact_cover(ops)
        fg = np.asarray(f_grid, np.float64).reshape(M, len(Vs))
        return _period_average(ops.__getitem__, lambda k: _drive(H0, Vs, fg[k]), M, T, X0, route,
                               e_min, e_max, L, tol, spp)
    V = np.asarray(V, np.complex128)
    spp = 1
    if scheme == "magnus6":
        f3 = np.asarray(f_nodes, np.float64).reshape(M, 3)
        Hs = [magnus6_heff(H0, V, f3[k], h) for k in range(M)]
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = exact_cover(Hs)
        Hk_of = Hs.__getitem__
    elif scheme == "cf4":
        ops = cf4_exponents(H0, V, f_nodes)
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = exact_cover(ops)
        Hk_of = ops.__getitem__
        spp = 2
    else:
        K = commutator(H0, V)
        a, b = magnus4_weights(f_nodes, h)
        if route == "cheb" and (e_min is None or e_max is None):
            e_min, e_max = weyl_cover(H0, V, K, a, b)

        def Hk_of(k):
            return magnus4_heff(H0, V, K, a[k], b[k])
    fg = np.asarray(f_grid, np.float64)
    return _period_average(Hk_of, lambda k: H0 + fg[k] * V, M, T, X0, route, e_min, e_max, L, tol,
                           spp)


def period_average_tridiag(h0_diag, h0_off, v_diag, f_nodes, f_grid, T: float, M: int, X0,
                           route: str = "cheb", e_min=None, e_max=None, L=None,
                           tol: float = 1e-12):
    """period_average for a Hermitian tridiagonal H0 and a diagonal V (sparse)."""
    h = T / M
    H0, V, K = tridiag_matrices(h0_diag, h0_off, v_diag)
    a, b = magnus4_weights(f_nodes, h)
    if route == "cheb" and (e_min is None or e_max is None):
        e_min, e_max = tridiag_cover(h0_diag, h0_off, v_diag, a, b)
    fg = np.asarray(f_grid, np.float64)
    return _period_average(lambda k: (H0 + a[k] * V + b[k] * K).tocsr(),
                           lambda k: (H0 + fg[k] * V).tocsr(), M, T, X0, route, e_min, e_max,
                           L, tol)


# ---------------------------------------------------------------------------
# Metrics (Sec. 2, Eq. (4) for the eigenphases)
# ---------------------------------------------------------------------------

def column_error(U: np.ndarray, Uref: np.ndarray) -> float:
    """max_j || (U - Uref) e_j ||_2: the worst propagated basis state."""
    return float(np.max(np.linalg.norm(U - Uref, axis=0)))


def unitarity_error(U: np.ndarray) -> Tuple[float, float]:
    """(max-abs, Frobenius) norms of U^dagger U - 1."""
    G = U.conj().T @ U - np.eye(U.shape[0])
    return float(np.max(np.abs(G))), float(np.linalg.norm(G))


def nearest_unitary(U: np.ndarray) -> np.ndarray:
    """Polar factor U (U^dagger U)^(-1/2): the unitary matrix nearest to U in
    the Frobenius norm (the optional re-orthonormalisation of U_T; the paper
    only notes that the truncated expansion is unitary up to the truncation,
    Sec. 2). SciPy's polar decomposition."""
    return scipy.linalg.polar(np.asarray(U, np.complex128), side="right")[0]


def eigenphases(U: np.ndarray) -> np.ndarray:
    """theta_mu with U phi = exp(-i theta) phi, theta in (-pi, pi] (Eq. (4));
    general complex eigenvalues by LAPACK zgeev, as in the paper."""
    lam = np.linalg.eigvals(U)
    th = -np.angle(lam)
    th[th <= -math.pi] += 2.0 * math.pi
    return np.sort(th)


def floquet_state_errors(U: np.ndarray, U_half: np.ndarray, T: float):
    """Accuracy of each Floquet state of U = U_T(h) against U_half = U_T(h/2)
    (Sec. 7, Eq. (error) with the paper's companion run at half the time step).

    The Floquet states are the eigenvectors phi_mu of U (U phi_mu =
    exp(-i theta_mu) phi_mu, Sec. 2, Eq. (4)); the states of U_half are the
    references. The printed measure |1 - <phi_mu|U_T|phi~_mu>| keeps the
    eigenphase exp(-i theta_mu) inside the overlap, where it is not small;
    it is read here as its two parts. For every mu, taking the reference state
    nu with the largest |<phi~_nu|phi_mu>|:
        sigma[mu] = 1 - |<phi~_nu|phi_mu>|      (normalised states)
        dq[mu]    = circular distance between theta_mu / T and theta~_nu / T
                    (modulo 2 pi / T).
    Returns (sigma, dq, theta / T), indexed like the eigenvalues of U as
    LAPACK zgeev returns them."""
    n = U.shape[0]
    lam, phi = np.linalg.eig(np.asarray(U, np.complex128))
    lam_r, phi_r = np.linalg.eig(np.asarray(U_half, np.complex128))
    theta = -np.angle(lam)
    theta_r = -np.angle(lam_r)
    period = 2.0 * math.pi / T
    sigma = np.empty(n)
    dq = np.empty(n)
    for mu in range(n):
        v = phi[:, mu] / np.linalg.norm(phi[:, mu])
        best, nu = -1.0, -1
        for j in range(n):
            w = phi_r[:, j] / np.linalg.norm(phi_r[:, j])
            o = abs(np.vdot(w, v))
            if o > best:
                best, nu = o, j
        sigma[mu] = 1.0 - best
        d = abs(theta[mu] / T - theta_r[nu] / T) % period
        dq[mu] = min(d, period - d)
    return sigma, dq, theta / T


def quasienergy_distance(theta1: np.ndarray, theta2: np.ndarray, T: float) -> float:
    """Symmetric circular Hausdorff distance between two eigenphase sets, / T.

    Each phase is matched to the nearest phase of the other set on the circle,
    so no assignment is needed and near-degenerate pairs do not matter.
    """
    t1 = np.sort(np.asarray(theta1))
    t2 = np.sort(np.asarray(theta2))

    def one_way(x, y):
        ext = np.concatenate([y - 2 * math.pi, y, y + 2 * math.pi])
        idx = np.searchsorted(ext, x)
        lo = np.clip(idx - 1, 0, len(ext) - 1)
        hi = np.clip(idx, 0, len(ext) - 1)
        return np.max(np.minimum(np.abs(x - ext[lo]), np.abs(x - ext[hi])))

    return float(max(one_way(t1, t2), one_way(t2, t1)) / T)


# ---------------------------------------------------------------------------
# Gradient of a trace-fidelity loss (not in the paper)
# ---------------------------------------------------------------------------

def trace_fidelity_loss(U: np.ndarray, W: np.ndarray) -> float:
    """1 - |Tr(W^dagger U)|^2 / N^2."""
    n = U.shape[0]
    tau = np.vdot(W, U)                       # sum conj(W) * U = Tr(W^dagger U)
    return float(1.0 - abs(tau) ** 2 / n ** 2)


def grad_piecewise(H0: np.ndarray, V: np.ndarray, f: np.ndarray, T: float, W: np.ndarray,
                   route: str = "cheb", e_min: Optional[float] = None, e_max: Optional[float] = None,
                   L: Optional[int] = None, tol: float = 1e-12,
                   ks: Optional[Sequence[int]] = None) -> np.ndarray:
    """d loss / d f_k for a piecewise-constant drive H_k = H0 + f_k V on M = len(f)
    equal steps (Sec. 1 discusses such drives; each step is then a single
    exponential and the Magnus commutator term vanishes).

    Each step map is E_k = p(H_k) with p(x) = exp(-i h x) (route "exact") or the
    Chebyshev polynomial of the rescaled operator with fixed beta, dE, L (route
    "cheb"). Its derivative along V is the Daleckii-Krein formula
    Q [(Q^dagger V Q) o G] Q^dagger, G_ab = (p(l_a) - p(l_b)) / (l_a - l_b),
    G_aa = p'(l_a), from the eigendecomposition H_k = Q diag(l) Q^dagger.
    Then d tau / d f_k = Tr(W^dagger E_M .. E_{k+1} dE_k E_{k-1} .. E_1) and
    d loss / d f_k = -(2 / N^2) Re(conj(tau) d tau / d f_k).
    """
    H0 = np.asarray(H0, np.complex128)
    V = np.asarray(V, np.complex128)
    n = H0.shape[0]
    f = np.asarray(f, np.float64)
    M = len(f)
    h = T / M
    if route == "cheb":
        if e_min is None or e_max is None:
            K0 = np.zeros_like(H0)
            e_min, e_max = weyl_cover(H0, V, K0, f, np.zeros(M))
        beta, dE, R = rescale(e_min, e_max, h)
        if L is None:
            L = choose_L(R, tol)
        acoef = bessel_coefficients(R, L)

    def scalar_map(lam):
        if route == "exact":
            return np.exp(-1j * h * lam), -1j * h * np.exp(-1j * h * lam)
        x = (lam - beta) / dE
        p, dp = chebyshev_polynomial_values(x, acoef, beta, h)
        return p, dp / dE

    Es, dEs, Xs = [], [], []
    X = np.eye(n, dtype=np.complex128)
    want = set(range(M)) if ks is None else set(int(k) for k in ks)
    for k in range(M):
        lam, Q = np.linalg.eigh(H0 + f[k] * V)
        p, dp = scalar_map(lam)
        E = (Q * p[None, :]) @ Q.conj().T
        if k in want:
            dl = lam[:, None] - lam[None, :]
            same = np.abs(dl) < 1e-300
            G = np.where(same, dp[:, None] * np.ones((1, n)),
                         (p[:, None] - p[None, :]) / np.where(same, 1.0, dl))
            dE_k = Q @ ((Q.conj().T @ V @ Q) * G) @ Q.conj().T
        else:
            dE_k = None
        Es.append(E)
        dEs.append(dE_k)
        Xs.append(X)
        X = E @ X
    tau = np.vdot(W, X)
    B = W.conj().T                      # B_k = W^dagger E_M ... E_{k+1}
    out = np.zeros(M)
    for k in range(M - 1, -1, -1):
        if dEs[k] is not None:
            dtau = np.trace(B @ dEs[k] @ Xs[k])
            out[k] = -(2.0 / n ** 2) * float(np.real(np.conj(tau) * dtau))
        B = B @ Es[k]
    return out
