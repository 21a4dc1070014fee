"""MI355X-native Floquet-operator library (gfx950, hand-written HIP).

Builds the one-period propagator U_T of H(t) = H0 + f(t) Hmod by a chain of
Magnus-4 / Chebyshev single-step operators applied to all columns at once
(Laptyeva et al., arXiv:1508.07621). The compute path is libfloquet.so (C ABI
in include/floquet.h); this package is its ctypes binding.
"""
from .floquet import (  # noqa: F401
    FloquetContext,
    FloquetUT,
    bessel_weights,
    choose_order,
    floquet_build_UT,
    floquet_grad,
    floquet_propagate,
    node_times,
    tridiag_extremes,
)
from .analysis import eigenphases  # noqa: F401
