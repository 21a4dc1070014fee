"""Seeded generators for the synthetic workloads.

Models (Sec. 4 of the paper, with the parameters of the benchmark workloads):

* random-matrix model: H(t) = H0 + f(t) V with H0, V drawn from the Gaussian
  unitary ensemble, H = (A + A^dagger) / (2 sqrt(N)), Re A_ij, Im A_ij iid N(0, 1).
  The paper draws from the orthogonal ensemble (Sec. 4 and Sec. 6); the unitary
  ensemble is used here so that every product is genuinely complex.
* Bose-Hubbard dimer with Nb bosons, Fock basis |n1, Nb - n1>, index i = n1:
  H = -J (b1^+ b2 + h.c.) + (U/2) sum_s n_s (n_s - 1) + eps(t) (n1 - n2),
  so H0 is real tridiagonal and the drive operator V = diag(2 i - Nb) is diagonal
  (Sec. 4, Eq. (18) gives the paper's variant of this model).

Everything returned is a NumPy array on the host; callers move it where they
need it. Random streams: ``numpy.random.default_rng(seed)``, drawn in the order
H0, V, drive amplitudes, target unitary.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, Optional

import numpy as np


def gue(n: int, rng: np.random.Generator) -> np.ndarray:
    """One GUE(n) matrix: (A + A^dagger) / (2 sqrt(n)), A complex Gaussian.

    With Re/Im A_ij ~ N(0, 1) the off-diagonal second moment E|H_ij|^2 is 1/n
    and the eigenvalue density tends to the semicircle on [-2, 2].
    """
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    h = (a + a.conj().T) / (2.0 * math.sqrt(n))
    return np.ascontiguousarray(h, dtype=np.complex128)


def random_matrix_model(n: int, seed: int):
    """(H0, V) for the random-matrix model, drawn in that order from one stream."""
    rng = np.random.default_rng(seed)
    h0 = gue(n, rng)
    v = gue(n, rng)
    return h0, v, rng


def dimer_tridiag(nb: int, J: float = 1.0, U: float = 0.01):
    """Bose-Hubbard dimer with nb bosons as tridiagonal arrays (dimension nb + 1).

    Returns (h0_diag[n] float64, h0_off[n-1] complex128, v_diag[n] float64) where
    H0[i][i] = (U/2)(n1(n1-1) + n2(n2-1)), H0[i][i+1] = -J sqrt((i+1)(nb-i)),
    and V = n1 - n2 = diag(2i - nb).
    """
    i = np.arange(nb + 1, dtype=np.float64)
    n1 = i
    n2 = nb - i
    diag = 0.5 * U * (n1 * (n1 - 1.0) + n2 * (n2 - 1.0))
    off = -J * np.sqrt((i[:-1] + 1.0) * (nb - i[:-1]))
    vdiag = 2.0 * i - nb
    return diag.astype(np.float64), off.astype(np.complex128), vdiag.astype(np.float64)


def dimer_dense(nb: int, J: float = 1.0, U: float = 0.01):
    """The same dimer as dense complex matrices (H0, V), for small nb."""
    d, e, v = dimer_tridiag(nb, J, U)
    n = nb + 1
    h0 = np.zeros((n, n), dtype=np.complex128)
    h0[np.arange(n), np.arange(n)] = d
    h0[np.arange(n - 1), np.arange(1, n)] = e
    h0[np.arange(1, n), np.arange(n - 1)] = np.conj(e)
    vm = np.diag(v).astype(np.complex128)
    return h0, vm


def drive_cos(t, eps0: float = 0.0, eps1: float = 1.0, omega: float = 1.0):
    """Scalar drive eps0 + eps1 cos(omega t), evaluated at the given times."""
    t = np.asarray(t, dtype=np.float64)
    return eps0 + eps1 * np.cos(omega * t)


def piecewise_amplitudes(m: int, rng: np.random.Generator, lo: float = -1.0, hi: float = 1.0):
    """m drive amplitudes f_j ~ U(lo, hi) for a piecewise-constant drive."""
    return rng.uniform(lo, hi, size=m).astype(np.float64)


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex Ginibre matrix with the phases
    of R's diagonal moved into Q (Mezzadri, Notices AMS 54 (2007) 592)."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return np.ascontiguousarray(q * ph[None, :], dtype=np.complex128)


@dataclass
class Workload:
    """A named synthetic workload: model arrays plus the drive description."""

    name: str
    n: int
    layout: str                      # "dense" or "tridiag"
    T: float
    M: int
    drive: Callable                  # f(t) for smooth drives, or None
    amplitudes: Optional[np.ndarray] = None   # piecewise-constant f_j per step
    arrays: Dict[str, np.ndarray] = field(default_factory=dict)
    extra: Dict[str, object] = field(default_factory=dict)
    scheme: str = "magnus4"          # step operator: "magnus4" or "magnus6" (the paper's)


def _seed(index: int) -> int:
    return 1508 + index


def workload(name: str, n: Optional[int] = None, M: Optional[int] = None) -> Workload:
    """Build one of the named workloads; n and M may be shrunk for tests."""
    two_pi = 2.0 * math.pi
    if name == "gue64":
        n = n or 64
        h0, v, _ = random_matrix_model(n, _seed(0))
        return Workload(name, n, "dense", two_pi, M or 100,
                        lambda t: drive_cos(t, 0.0, 1.0, 1.0), arrays={"h0": h0, "v": v})
    if name == "dimer1000":
        nb = (n - 1) if n else 999
        d, e, vd = dimer_tridiag(nb, 1.0, 0.01)
        return Workload(name, nb + 1, "tridiag", two_pi, M or 500,
                        lambda t: drive_cos(t, 0.5, 1.5, 1.0),
                        arrays={"h0_diag": d, "h0_off": e, "v_diag": vd})
    if name == "gue4096":
        n = n or 4096
        h0, v, _ = random_matrix_model(n, _seed(2))
        return Workload(name, n, "dense", two_pi, M or 200,
                        lambda t: drive_cos(t, 0.0, 1.0, 1.0), arrays={"h0": h0, "v": v})
    if name == "gue4096m6":
        # the 4096-state model of gue4096 with the paper's sixth-order scheme
        # and four times longer steps
        n = n or 4096
        h0, v, _ = random_matrix_model(n, _seed(2))
        return Workload(name, n, "dense", two_pi, M or 50,
                        lambda t: drive_cos(t, 0.0, 1.0, 1.0), arrays={"h0": h0, "v": v},
                        scheme="magnus6")
    if name == "adjoint1024":
        n = n or 1024
        m = M or 256
        h0, v, rng = random_matrix_model(n, _seed(3))
        f = piecewise_amplitudes(m, rng)
        w = haar_unitary(n, rng)
        return Workload(name, n, "dense", two_pi, m, None, amplitudes=f,
                        arrays={"h0": h0, "v": v, "w": w})
    if name == "dimer10000":
        nb = (n - 1) if n else 9999
        d, e, vd = dimer_tridiag(nb, 1.0, 0.01)
        return Workload(name, nb + 1, "tridiag", two_pi, M or 500,
                        lambda t: drive_cos(t, 0.5, 1.5, 1.0),
                        arrays={"h0_diag": d, "h0_off": e, "v_diag": vd})
    if name == "adjointdimer10000":
        # the 9999-boson dimer of dimer10000 under a piecewise-constant drive of
        # m amplitudes f_j ~ U(-1, 1); the loss targets U_T of the nearby drive
        # f_j + 0.02 u_j (u_j ~ U(-1, 1)), a reachable target gate
        nb = (n - 1) if n else 9999
        m = M or 256
        d, e, vd = dimer_tridiag(nb, 1.0, 0.01)
        rng = np.random.default_rng(_seed(5))
        f = piecewise_amplitudes(m, rng)
        f_target = f + 0.02 * rng.uniform(-1.0, 1.0, m)
        return Workload(name, nb + 1, "tridiag", two_pi, m, None, amplitudes=f,
                        arrays={"h0_diag": d, "h0_off": e, "v_diag": vd, "f_target": f_target})
    if name == "gue10000":
        n = n or 10000
        h0, v, _ = random_matrix_model(n, _seed(4))
        return Workload(name, n, "dense", two_pi, M or 200,
                        lambda t: drive_cos(t, 0.0, 1.0, 1.0), arrays={"h0": h0, "v": v})
    raise KeyError(name)


WORKLOADS = ("gue64", "dimer1000", "gue4096", "adjoint1024", "dimer10000", "gue10000",
             "gue4096m6", "adjointdimer10000")
