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
