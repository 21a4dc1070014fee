"""One GPU's share of the column split over P GPUs (Sec. 5, Fig. 2).

Columns of U_T are independent propagations, so a GPU that propagates its N/P
identity columns over the whole period must get exactly those columns of the
full build: the same kernels run on fewer rows of the state block. Checked for
every share of a P-way split, dense (FP64 and split-BF16) and tridiagonal.
"""
import math

import numpy as np
import pytest
import torch

import oracle as orc
from workloads import dimer_tridiag, drive_cos, gue

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi


@pytest.fixture(scope="module")
def fl(require_gpu):
    from paper_1508_07621_amd import floquet
    floquet.node_times(1.0, 1)          # loads the library or raises
    return floquet


def _say(*a):
    print("[case]", *a, flush=True)


def _context(fl, layout, precision, n, M):
    T = TWO_PI
    if layout == "dense":
        rng = np.random.default_rng(70 + n)
        H0, V = gue(n, rng), gue(n, rng)
        f = drive_cos(orc.node_times(T, M), 0.0, 1.0, 1.0)
        return fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f, precision=precision)
    d, e, v = dimer_tridiag(n - 1, 1.0, 0.05)
    f = drive_cos(orc.node_times(T, M), 0.5, 1.5, 1.0)
    return fl.FloquetContext(h0_diag=d, h0_off=e, hmod_diag=v, T=T, M=M, f_nodes=f)


@pytest.mark.parametrize("layout,precision,n,P,tol", [
    ("dense", "fp64", 512, 4, 1e-13), ("dense", "bf16x3", 512, 4, 1e-9),
    ("dense", "fp64", 300, 3, 1e-13), ("tridiag", "fp64", 300, 3, 1e-14)])
def test_share_equals_columns_of_full_build(fl, layout, precision, n, P, tol):
    _say("share", layout, precision, n, P)
    M = 16
    ctx = _context(fl, layout, precision, n, M)
    U = ctx.build_ut()
    eye = torch.eye(n, dtype=U.dtype, device=U.device)
    c = n // P
    worst = 0.0
    for r in range(P):
        X0 = eye[:, r * c:(r + 1) * c].contiguous()
        X = ctx.propagate(X0, 0, M)
        worst = max(worst, (X - U[:, r * c:(r + 1) * c]).abs().max().item())
    _say("max |share - columns of U_T|", worst)
    assert worst <= tol
