"""fq_set_drive: a context's drive replaced in place (operators and workspace
kept) gives the same U_T, report and gradient as a context created with that
drive; a caller's fixed interval is checked against the new drive; the
autograd wrapper can reuse one context."""
import math

import numpy as np
import pytest

import oracle as orc
from workloads import dimer_tridiag, drive_cos, gue, haar_unitary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fl(require_gpu):
    from paper_1508_07621_amd import floquet
    floquet.node_times(1.0, 1)
    return floquet


from paper_1508_07621_amd._abi import (FQ_ERR_NONFINITE, FQ_ERR_SPECTRUM,  # noqa: E402
                                       FQ_ERR_STATE, FloquetError)


def _say(*a):
    print("[case]", *a, flush=True)


def _loss_bar(U, W):
    n = U.shape[0]
    tau = np.vdot(W, U)
    return 1.0 - abs(tau) ** 2 / n ** 2, -(2.0 / n ** 2) * tau * W


def _system(layout, rng):
    if layout == "dense":
        n = 40
        return n, dict(h0=gue(n, rng), hmod=gue(n, rng))
    d, e, v = dimer_tridiag(29, 1.0, 0.3)
    return 30, dict(h0_diag=d, h0_off=e, hmod_diag=v)


@pytest.mark.parametrize("layout,precision", [("dense", "fp64"), ("dense", "bf16x3"),
                                              ("tridiag", "fp64")])
def test_set_drive_equals_fresh_context(fl, layout, precision):
    rng = np.random.default_rng(31)
    n, sysk = _system(layout, rng)
    T, M = 2.0, 8
    f1 = drive_cos(orc.node_times(T, M), 0.1, 1.0, 1.0)
    f2 = drive_cos(orc.node_times(T, M), -0.3, 2.5, 2.0)   # a wider drive: new interval, R, L
    kw = dict(T=T, M=M, tol=1e-12, precision=precision, checkpoint_every=2, **sysk)
    ctx = fl.FloquetContext(f_nodes=f1, **kw)
    ctx.build_ut()
    ctx.set_drive(f2)
    U = ctx.build_ut().cpu().numpy()
    fresh = fl.FloquetContext(f_nodes=f2, **kw)
    Uf = fresh.build_ut().cpu().numpy()
    r, rf = ctx.report, fresh.report
    _say(layout, precision, "L", r["L"], rf["L"], "R", r["R"], "diff", np.max(np.abs(U - Uf)))
    for key in ("L", "R", "e_min", "e_max", "dE", "beta"):
        assert r[key] == rf[key], key
    assert r["term_format"] == rf["term_format"]
    assert np.max(np.abs(U - Uf)) <= 1e-14
    W = haar_unitary(n, rng)
    _, Ubar = _loss_bar(U, W)
    g, gf = ctx.grad(Ubar), fresh.grad(Ubar)
    assert np.max(np.abs(g - gf)) <= 1e-12 * np.max(np.abs(gf))


def test_set_drive_fixed_interval_and_errors(fl):
    rng = np.random.default_rng(32)
    n = 24
    H0, V = gue(n, rng), gue(n, rng)
    T, M = 1.0, 4
    f1 = drive_cos(orc.node_times(T, M), 0.0, 0.5, 1.0)
    a, b = orc.magnus4_weights(f1, T / M)
    lo, hi = orc.weyl_cover(H0, V, orc.commutator(H0, V), a, b)
    ctx = fl.FloquetContext(h0=H0, hmod=V, T=T, M=M, f_nodes=f1, e_min=lo, e_max=hi, L=20)
    U1 = ctx.build_ut().cpu().numpy()
    # a drive whose operators leave the fixed interval is refused, and so are builds after it
    with pytest.raises(FloquetError) as ei:
        ctx.set_drive(20.0 * f1)
    assert ei.value.status == FQ_ERR_SPECTRUM
    with pytest.raises(FloquetError) as ei:
        ctx.build_ut()
    assert ei.value.status == FQ_ERR_STATE
    with pytest.raises(FloquetError) as ei:
        ctx.set_drive(np.full_like(f1, math.nan))
    assert ei.value.status == FQ_ERR_NONFINITE
    ctx.set_drive(f1)   # a valid drive restores the context
    assert np.array_equal(ctx.build_ut().cpu().numpy(), U1)
    with pytest.raises(ValueError):
        ctx.set_drive(f1[:2])


def test_autograd_with_a_reused_context(fl):
    import torch
    rng = np.random.default_rng(33)
    n, M, T = 32, 6, 2.0
    H0, V = gue(n, rng), gue(n, rng)
    W = torch.from_numpy(haar_unitary(n, rng)).to("cuda")
    f0 = rng.uniform(-1, 1, (M, 2))
    kw = dict(h0=H0, hmod=V, T=T, M=M, tol=1e-12, checkpoint_every=2)
    ctx = fl.FloquetContext(f_nodes=f0, **kw)

    def run(f, context):
        ft = torch.tensor(f, dtype=torch.float64, device="cuda", requires_grad=True)
        U = fl.FloquetUT.apply(ft, context=context, **({} if context else kw))
        loss = 1.0 - torch.abs(torch.sum(torch.conj(W) * U)) ** 2 / n ** 2
        loss.backward()
        return loss.item(), ft.grad.cpu().numpy()

    for f in (f0, f0 + 0.1 * rng.standard_normal(f0.shape)):
        l1, g1 = run(f, ctx)
        l2, g2 = run(f, None)
        _say("loss", l1, l2, "grad diff", np.max(np.abs(g1 - g2)))
        assert abs(l1 - l2) <= 1e-14
        assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g2))
    # a backward after the context was rebuilt would use the wrong tape: refused
    ft = torch.tensor(f0, dtype=torch.float64, device="cuda", requires_grad=True)
    U = fl.FloquetUT.apply(ft, context=ctx)
    ctx.build_ut()
    with pytest.raises(RuntimeError):
        torch.abs(torch.sum(torch.conj(W) * U)).backward()
