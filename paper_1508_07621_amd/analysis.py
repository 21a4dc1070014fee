"""Host FP64 post-processing of a built U_T.

The diagonalisation of U_T is the routine, untimed host step after the
propagation (Sec. 3 and Sec. 5 of the paper, which used LAPACK zgeev); it runs
here through NumPy's LAPACK in float64 on a host copy.
"""
from __future__ import annotations

import math

import numpy as np


def eigenphases(U) -> np.ndarray:
    """Sorted theta_mu in (-pi, pi] with U phi_mu = exp(-i theta_mu) phi_mu
    (Sec. 2, Eq. (4)); quasienergies are theta / T."""
    try:
        import torch
        if isinstance(U, torch.Tensor):
            U = U.detach().cpu().numpy()
    except ImportError:
        pass
    lam = np.linalg.eigvals(np.asarray(U, dtype=np.complex128))
    th = -np.angle(lam)
    th[th <= -math.pi] += 2.0 * math.pi
    return np.sort(th)


def eigenphases_unitary(U) -> np.ndarray:
    """Sorted theta_mu in (-pi, pi] of a (nearly) unitary U through a Hermitian
    eigenproblem, for sizes where the general eigensolver (zgeev) is slow
    (N = 10^4 in minutes): for U' = exp(i phi) U the Cayley transform
    C = -i (1 - U')(1 + U')^(-1) has the eigenvalues tan(theta'_mu / 2),
    theta' = theta - phi, and is Hermitian when U is unitary; its Hermitian
    part is diagonalised (LAPACK zheevd, eigenvalues only) and
    theta = 2 atan(lambda) + phi. The departure of U from unitarity enters the
    phases at second order. phi is chosen so that no eigenvalue of U' is close
    to -1 (|C| bounded), trying a few phases."""
    try:
        import torch
        if isinstance(U, torch.Tensor):
            U = U.detach().cpu().numpy()
    except ImportError:
        pass
    U = np.asarray(U, dtype=np.complex128)
    n = U.shape[0]
    eye = np.eye(n, dtype=np.complex128)
    for phi in (0.0, 1.0, 2.0, 3.0, 0.5, 2.5):
        Up = np.exp(1j * phi) * U
        C = -1j * np.linalg.solve(eye + Up, eye - Up)
        if np.isfinite(C).all() and np.abs(C).max() < 1e8:
            break
    lam = np.linalg.eigvalsh(0.5 * (C + C.conj().T))
    th = 2.0 * np.arctan(lam) + phi
    th = np.mod(th + math.pi, 2.0 * math.pi) - math.pi
    th[th <= -math.pi] += 2.0 * math.pi
    return np.sort(th)


def floquet_states(ctx, U, f_grid):
    """The Floquet states of a built U_T ordered by mean energy (the paper's
    post-processing, Sec. 3 and Sec. 7): host eigendecomposition of U_T
    (LAPACK zgeev through NumPy), then the second propagation round on the
    device for the period-averaged energies (ctx.period_average). Returns
    (quasienergies theta/T, states as columns, mean energies), sorted by mean
    energy ascending. f_grid: the drive at t_k = k h, k = 0..M-1."""
    try:
        import torch
        if isinstance(U, torch.Tensor):
            U = U.detach().cpu().numpy()
    except ImportError:
        pass
    lam, phi = np.linalg.eig(np.asarray(U, dtype=np.complex128))
    th = -np.angle(lam)
    th[th <= -math.pi] += 2.0 * math.pi
    phi = phi / np.linalg.norm(phi, axis=0)
    e_mean = ctx.period_average(phi, f_grid)
    order = np.argsort(e_mean, kind="stable")
    return th[order] / ctx.T, phi[:, order], e_mean[order]


def state_errors(phi, eps, phi_ref, eps_ref, T):
    """State-specific accuracy of Floquet states against a reference set (e.g.
    from half the time step, as the paper's overlap phase error does): for each
    state mu, its best-overlapping reference state nu, the overlap deficiency
    1 - |<phi_mu|phi_ref_nu>| and the circular quasienergy difference
    |eps_mu - eps_ref_nu| (modulo 2 pi / T). The printed measure keeps the
    eigenphase inside the overlap, where it is not small; these two parts are
    the reading taken here."""
    ov = np.abs(np.asarray(phi_ref).conj().T @ np.asarray(phi))   # [nu, mu]
    nu = np.argmax(ov, axis=0)
    defic = 1.0 - ov[nu, np.arange(ov.shape[1])]
    period = 2.0 * math.pi / T
    d = np.abs(np.asarray(eps) - np.asarray(eps_ref)[nu]) % period
    return defic, np.minimum(d, period - d)


def state_errors_of_builds(U, U_half, T):
    """The accuracy of each Floquet state of U = U_T(h), estimated as the paper
    does (Sec. 7, Eq. (error)) from a companion build with half the time step,
    U_half = U_T(h/2): host eigendecompositions of both (LAPACK zgeev through
    NumPy), then state_errors of the first set against the second. Returns
    (sigma, dq, eps) per eigenvector of U: overlap deficiency with the
    best-matching state of U_half, quasienergy difference to it (modulo
    2 pi / T), and the quasienergy theta / T."""
    try:
        import torch
        if isinstance(U, torch.Tensor):
            U = U.detach().cpu().numpy()
        if isinstance(U_half, torch.Tensor):
            U_half = U_half.detach().cpu().numpy()
    except ImportError:
        pass
    out = []
    for W in (U, U_half):
        lam, phi = np.linalg.eig(np.asarray(W, dtype=np.complex128))
        th = -np.angle(lam)
        out.append((phi / np.linalg.norm(phi, axis=0), th / T))
    (phi, eps), (phi_r, eps_r) = out
    sigma, dq = state_errors(phi, eps, phi_r, eps_r, T)
    return sigma, dq, eps
