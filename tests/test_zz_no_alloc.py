"""The allocation-free one-shot build (floquet_build_UT_static) against the
context build (fq_create + floquet_build_UT) on the same inputs: two calls in
a row on the library's static scratch, the second with a smaller problem, so
that what the first call left in the array must not leak into the second."""
import math

import numpy as np
import pytest

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


def _dense_kw(n, M, seed, precision):
    rng = np.random.default_rng(seed)
    H0, V = gue(n, rng), gue(n, rng)
    f = drive_cos(orc.node_times(TWO_PI, M), 0.0, 1.0, 1.0)
    return dict(h0=H0, hmod=V, T=TWO_PI, M=M, f_nodes=f, precision=precision)


def _tridiag_kw(nb, M):
    d, e, v = dimer_tridiag(nb, 1.0, 0.01)
    f = drive_cos(orc.node_times(TWO_PI, M), 0.5, 1.5, 1.0)
    return dict(h0_diag=d, h0_off=e, hmod_diag=v, T=TWO_PI, M=M, f_nodes=f)


def _check(fl, kw, tol):
    import torch
    ref = fl.FloquetContext(**kw)
    U_ref = ref.build_ut()
    U, rep = fl.floquet_build_UT_static(**kw)
    torch.cuda.synchronize()
    err = torch.linalg.vector_norm(U - U_ref, dim=0).max().item()
    _say("e_col vs context build", err, "unitarity", rep["unitarity_max"],
         ref.last_report["unitarity_max"])
    assert err <= tol
    assert rep["L"] == ref.last_report["L"] and rep["ms_build"] == 0.0
    assert rep["unitarity_max"] == pytest.approx(ref.last_report["unitarity_max"], rel=1e-6,
                                                 abs=1e-15)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("bf16x3", 1e-6)])
def test_static_dense_two_calls_second_smaller(fl, precision, tol):
    _say("static dense", precision, "n = 700 then n = 130")
    _check(fl, _dense_kw(700, 6, 21, precision), tol)
    _check(fl, _dense_kw(130, 9, 22, precision), tol)


def test_static_tridiag_two_calls_second_smaller(fl):
    _say("static tridiagonal", "n = 1000 then n = 201")
    _check(fl, _tridiag_kw(999, 40), 1e-10)
    _check(fl, _tridiag_kw(200, 25), 1e-10)


def test_static_rejects_oversized_problem(fl):
    from paper_1508_07621_amd._abi import FQ_ERR_ARG, FloquetError
    rng = np.random.default_rng(3)
    n = 1409
    kw = dict(h0=np.eye(n, dtype=complex), hmod=np.diag(rng.standard_normal(n)).astype(complex),
              T=1.0, M=2, f_nodes=np.zeros((2, 2)))
    with pytest.raises(FloquetError) as e:
        fl.floquet_build_UT_static(**kw)
    assert e.value.status == FQ_ERR_ARG
