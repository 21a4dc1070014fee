"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

Only model definitions and random draws live here (random-matrix Hamiltonians,
the Bose-Hubbard dimer in its Fock basis, drive functions evaluated at given
times, a Haar-random target unitary). None of the Floquet method's arithmetic
(Magnus nodes, commutators, Chebyshev expansion, spectral rescaling) is here:
each side implements that on its own.
"""
from .generators import (  # noqa: F401
    WORKLOADS,
    Workload,
    dimer_tridiag,
    dimer_dense,
    drive_cos,
    gue,
    haar_unitary,
    piecewise_amplitudes,
    random_matrix_model,
    workload,
)
