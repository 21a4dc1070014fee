"""The C ABI on the CPU: the library loads, exports every declared entry point,
its host FP64 numerics match independent references, and invalid arguments are
rejected before any device work (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest
import scipy.linalg
import scipy.special

import oracle as orc
from paper_1508_07621_amd import _abi
from paper_1508_07621_amd import floquet as fl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "floquet.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:fq|floquet)_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    declared = _declared_functions()
    assert set(declared) == set(_abi.EXPORTS), (declared, _abi.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_struct_layouts_match_header():
    assert ctypes.sizeof(_abi.FqSystem) == 8 + 4 + 4 + 6 * 8
    assert ctypes.sizeof(_abi.FqParams) == 8 + 4 + 4 + 8 + 3 * 8 + 6 * 4 + 8 + 8 + 8
    assert ctypes.sizeof(_abi.FqReport) == 4 + 4 + 10 * 8 + 16 * 8 + 16 * 4 + 16 * 4 + 8 + 8


def test_struct_offsets_match_compiled_header(tmp_path):
    """sizeof / offsetof of the ABI structs from a C compilation of
    include/floquet.h against the ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    fields = {"fq_system": _abi.FqSystem, "fq_params": _abi.FqParams, "fq_report": _abi.FqReport}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "floquet.h"', "int main(void) {"]
    for cname, py in fields.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in fields.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_node_times_match_oracle():
    for T, M in [(2 * math.pi, 100), (1.0, 1), (3.3, 17)]:
        np.testing.assert_allclose(fl.node_times(T, M), orc.node_times(T, M), rtol=0, atol=1e-14)


@pytest.mark.parametrize("R", [0.0, 1e-8, 0.126, 0.251, 1.0, 10.0, 37.03, 500.0, 1762.0, 3441.0])
def test_bessel_weights_match_scipy(R):
    L = max(4, int(R * 1.1) + 40)
    w = fl.bessel_weights(R, L)
    ref = 2.0 * scipy.special.jv(np.arange(L + 1), R)
    ref[0] *= 0.5
    scale = np.max(np.abs(ref))
    # SciPy's AMOS values carry ~1e-14 relative error at arguments in the thousands
    assert np.max(np.abs(w - ref)) <= 2e-14 * max(1.0, R / 50.0) * scale


@pytest.mark.parametrize("R", [0.126, 37.03, 500.0, 1762.0])
def test_bessel_weights_match_mpmath(R):
    mpmath = pytest.importorskip("mpmath")
    w = fl.bessel_weights(R, int(R) + 40)
    for l in sorted({0, 1, 2, int(R / 2), int(R), int(R) + 20}):
        ref = float((1 if l == 0 else 2) * mpmath.besselj(l, R))
        assert abs(w[l] - ref) <= 2e-16 * max(abs(ref), 1e-3), (l, w[l], ref)


def test_bessel_weights_against_published_table():
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "bessel_table.txt"))
    for n, x, ref in rows:
        w = fl.bessel_weights(x, int(n))[int(n)] / (1.0 if n == 0 else 2.0)
        assert abs(w - ref) <= 5e-10 * max(1.0, abs(ref)) + 1e-19


@pytest.mark.parametrize("R", [0.05, 0.098, 0.126, 0.251, 1.0, 37.03, 1762.0])
def test_choose_order_matches_oracle(R):
    for tol in (1e-8, 1e-12, 1e-14):
        assert fl.choose_order(R, tol) == orc.choose_L(R, tol)


def test_tridiag_extremes_match_lapack():
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 50, 1000):
        d = rng.standard_normal(n) * 10
        e = np.abs(rng.standard_normal(max(n - 1, 0)))
        lo, hi = fl.tridiag_extremes(d, e)
        if n == 1:
            ref = np.array([d[0]])
        else:
            ref = scipy.linalg.eigvalsh_tridiagonal(d, e)
        assert abs(lo - ref[0]) <= 1e-13 * max(1, abs(ref[0]))
        assert abs(hi - ref[-1]) <= 1e-13 * max(1, abs(ref[-1]))


def test_tridiag_extremes_dimer_spectrum():
    """Spin-S matrix -2 J S_x has the exact spectrum {-2 J m}: extremes -/+ J Nb."""
    from workloads import dimer_tridiag
    nb = 999
    d, e, _ = dimer_tridiag(nb, 1.0, 0.0)
    lo, hi = fl.tridiag_extremes(d, np.abs(e))
    assert abs(lo + nb) < 1e-10 and abs(hi - nb) < 1e-10


# ---- argument validation: every path below returns before any HIP call --------------------

FAKE = 0x1000  # non-null placeholder; validation never dereferences device pointers


def _dense(n=8):
    s = _abi.FqSystem()
    s.n, s.layout, s.h0, s.hmod = n, _abi.FQ_DENSE, FAKE, FAKE
    return s


def _tridiag(n=8):
    s = _abi.FqSystem()
    s.n, s.layout, s.h0_diag, s.h0_off, s.hmod_diag = n, _abi.FQ_TRIDIAG, FAKE, FAKE, FAKE
    return s


def _params(M=4, f=None, **kw):
    p = _abi.FqParams()
    f = np.zeros(2 * M) if f is None else f
    p.T, p.M, p.L, p.tol = 1.0, M, 0, 1e-12
    p.f_nodes = _abi.dptr(f)
    p.e_min = p.e_max = math.nan
    p.precision, p.checkpoint_every = 0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    p._keep = f
    return p


def _ws(sysd, par):
    n = ctypes.c_size_t(0)
    st = _abi.lib().fq_workspace_bytes(ctypes.byref(sysd), ctypes.byref(par), ctypes.byref(n))
    return st, n.value


def test_workspace_bytes_ok_and_grows_with_n():
    st1, b1 = _ws(_dense(100), _params())
    st2, b2 = _ws(_dense(1000), _params())
    st3, b3 = _ws(_dense(1000), _params(checkpoint_every=2))
    assert st1 == st2 == st3 == _abi.FQ_OK
    assert 0 < b1 < b2 < b3
    st, b = _ws(_tridiag(1000), _params())
    assert st == _abi.FQ_OK and b > 0


@pytest.mark.parametrize("mutate,status", [
    (lambda s, p: setattr(s, "n", 0), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(s, "layout", 7), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(s, "n_drive", 5), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(s, "n_drive", 2), _abi.FQ_ERR_ARG),   # no hmods
    (lambda s, p: setattr(s, "h0", None), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "T", -1.0), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "T", math.inf), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "M", 0), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "L", -1), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "L", 10 ** 6), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "tol", 0.0), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "e_min", 0.0), _abi.FQ_ERR_ARG),
    (lambda s, p: (setattr(p, "e_min", 1.0), setattr(p, "e_max", 1.0)), _abi.FQ_ERR_SPECTRUM),
    (lambda s, p: (setattr(p, "e_min", -math.inf), setattr(p, "e_max", 1.0)), _abi.FQ_ERR_NONFINITE),
    (lambda s, p: setattr(p, "precision", 9), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "checkpoint_every", -2), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "profile", 2), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "reorthonormalize", 2), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "dtype", 2), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "scheme", 3), _abi.FQ_ERR_ARG),
    (lambda s, p: setattr(p, "scheme", -1), _abi.FQ_ERR_ARG),
])
def test_invalid_arguments_rejected(mutate, status):
    s, p = _dense(), _params()
    mutate(s, p)
    st, _ = _ws(s, p)
    assert st == status
    assert _abi.lib().fq_last_error().decode() != ""


def test_nonfinite_drive_rejected():
    f = np.zeros(8)
    f[5] = math.nan
    st, _ = _ws(_dense(), _params(M=4, f=f))
    assert st == _abi.FQ_ERR_NONFINITE
    assert "f_nodes[5]" in _abi.lib().fq_last_error().decode()


def test_tridiag_restrictions():
    st, _ = _ws(_tridiag(), _params(precision=1))
    assert st == _abi.FQ_ERR_UNSUPPORTED
    # gradient tape: per-column reverse sweep up to 2048 rows, streamed passes
    # beyond (20 more n x n16 FP64 planes for their carried state, and the
    # forward passes' two 8-plane states for the segment recompute)
    st, b0 = _ws(_tridiag(2048), _params())
    st1, b1 = _ws(_tridiag(2048), _params(checkpoint_every=4))
    assert st == st1 == _abi.FQ_OK and b1 > b0
    st2, b2 = _ws(_tridiag(2049), _params(checkpoint_every=4))
    assert st2 == _abi.FQ_OK and b2 >= b1 + 20 * 8 * 2064 * 2049
    # beyond one workgroup's column the forward build keeps its checkpoints in
    # the state blocks' type, complex64 included
    st, _ = _ws(_tridiag(5000), _params(checkpoint_every=4, dtype=_abi.FQ_C64))
    assert st == _abi.FQ_OK
    st, _ = _ws(_tridiag(4096), _params(checkpoint_every=4, dtype=_abi.FQ_C64))
    assert st == _abi.FQ_OK


def test_streamed_adjoint_switch_sizes_the_workspace(monkeypatch):
    """FQ_TRIDIAG_STREAMED_ADJOINT=1 selects the streamed reverse sweep for
    short columns too: the workspace then holds its ten carried vectors."""
    st0, b0 = _ws(_tridiag(300), _params(checkpoint_every=4))
    monkeypatch.setenv("FQ_TRIDIAG_STREAMED_ADJOINT", "1")
    st1, b1 = _ws(_tridiag(300), _params(checkpoint_every=4))
    st2, b2 = _ws(_tridiag(300), _params())            # no tape: no gradient buffers
    monkeypatch.setenv("FQ_TRIDIAG_STREAMED_ADJOINT", "0")
    st3, b3 = _ws(_tridiag(300), _params(checkpoint_every=4))
    assert st0 == st1 == st2 == st3 == _abi.FQ_OK
    assert b1 >= b0 + 10 * 16 * 300 * 300
    assert b3 == b0
    assert b2 < b0
    # columns longer than one workgroup: two streamed states of n x n doubles
    st, b = _ws(_tridiag(5000), _params())
    assert st == _abi.FQ_OK and b >= 2 * 8 * 8 * 5000 * 5000
    st, _ = _ws(_tridiag(40001), _params())
    assert st == _abi.FQ_ERR_UNSUPPORTED


def test_magnus6_restrictions_and_workspace():
    """The sixth-order scheme reads 3*M drive samples, needs the dense layout and
    no gradient tape, and holds nine more n x n complex matrices."""
    f3 = np.zeros(12)
    st, b4 = _ws(_dense(100), _params(M=4, f=np.zeros(8)))
    st6, b6 = _ws(_dense(100), _params(M=4, f=f3, scheme=_abi.FQ_MAGNUS6))
    assert st == st6 == _abi.FQ_OK
    np_ = 128  # 100 padded to the 64-row tile
    assert b6 - b4 >= 9 * 16 * np_ * np_
    st, _ = _ws(_tridiag(100), _params(M=4, f=f3, scheme=_abi.FQ_MAGNUS6))
    assert st == _abi.FQ_ERR_UNSUPPORTED
    st, _ = _ws(_dense(100), _params(M=4, f=f3, scheme=_abi.FQ_MAGNUS6, checkpoint_every=2))
    assert st == _abi.FQ_ERR_UNSUPPORTED
    # the 3*M samples are all read: a NaN in the last one is caught
    f3[11] = math.nan
    st, _ = _ws(_dense(100), _params(M=4, f=f3, scheme=_abi.FQ_MAGNUS6))
    assert st == _abi.FQ_ERR_NONFINITE
    assert "f_nodes[11]" in _abi.lib().fq_last_error().decode()


def test_cf4_runs_two_half_steps_per_step():
    """The commutator-free scheme takes the 2*M two-node samples, works for both
    layouts and the gradient, and sizes its step tables for 2*M half-steps."""
    st, b4 = _ws(_tridiag(100), _params(M=4, checkpoint_every=2))
    stc, bc = _ws(_tridiag(100), _params(M=4, checkpoint_every=2, scheme=_abi.FQ_CF4))
    assert st == stc == _abi.FQ_OK and bc > b4
    st, _ = _ws(_dense(100), _params(M=4, scheme=_abi.FQ_CF4, checkpoint_every=2))
    assert st == _abi.FQ_OK


def test_eigenbasis_layout_arguments():
    """FQ_DENSE_EIGEN takes H0 by its eigenvalues (h0_diag) and a dense hmod,
    and needs the dense workspace."""
    d = _dense(100)
    e = _dense(100)
    e.layout, e.h0, e.h0_diag = _abi.FQ_DENSE_EIGEN, None, FAKE
    st_d, b_d = _ws(d, _params())
    st_e, b_e = _ws(e, _params())
    assert st_d == st_e == _abi.FQ_OK and b_e == b_d
    e.h0_diag = None
    st, _ = _ws(e, _params())
    assert st == _abi.FQ_ERR_ARG
    e.h0_diag = FAKE
    st, _ = _ws(e, _params(M=4, f=np.zeros(12), scheme=_abi.FQ_MAGNUS6))
    assert st == _abi.FQ_OK


def test_several_drive_terms_arguments():
    """n_drive >= 2 takes hmods (dense layouts, FQ_MAGNUS4 or FQ_CF4), S values per
    node, and a drive block of 2S + S(S-1)/2 (Magnus-4) or S (CF4) matrices."""
    arr = (ctypes.c_void_p * 3)(FAKE, FAKE, FAKE)

    def sys3(layout=_abi.FQ_DENSE):
        s = _dense(128)
        s.layout, s.n_drive = layout, 3
        s.hmods = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        s.hmod = None
        return s
    f = np.zeros(4 * 2 * 3)
    st1, b1 = _ws(_dense(128), _params())
    st4, b4 = _ws(sys3(), _params(M=4, f=f))
    stc, bc = _ws(sys3(), _params(M=4, f=f, scheme=_abi.FQ_CF4))
    assert st1 == st4 == stc == _abi.FQ_OK
    plane2 = 16 * 128 * 128
    assert b4 - b1 == (9 - 2) * plane2 and bc - b1 == (3 - 2) * plane2
    st, _ = _ws(sys3(), _params(M=4, f=np.zeros(36), scheme=_abi.FQ_MAGNUS6))
    assert st == _abi.FQ_ERR_UNSUPPORTED
    t = _tridiag(128)
    t.n_drive, t.hmods = 3, ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    st, _ = _ws(t, _params(M=4, f=f))
    assert st == _abi.FQ_ERR_UNSUPPORTED
    f[-1] = math.nan   # all 2 M S samples are read
    st, _ = _ws(sys3(), _params(M=4, f=f))
    assert st == _abi.FQ_ERR_NONFINITE


def test_magnus6_node_times_match_the_oracle():
    import oracle as orc
    t = fl.node_times(2.5, 7, scheme="magnus6")
    assert t.shape == (7, 3)
    assert np.abs(t - orc.node_times6(2.5, 7)).max() < 1e-14
    with pytest.raises(_abi.FloquetError):
        fl.node_times(2.5, 0, scheme="magnus6")


def test_create_rejects_before_device_work():
    L = _abi.lib()
    s, p = _dense(), _params()
    h = ctypes.c_void_p()
    assert L.fq_create(ctypes.byref(h), ctypes.byref(s), ctypes.byref(p), None, 0, None) == _abi.FQ_ERR_ARG
    assert L.fq_create(ctypes.byref(h), ctypes.byref(s), ctypes.byref(p), 0x1001, 1 << 40, None) == _abi.FQ_ERR_ARG
    assert L.fq_create(ctypes.byref(h), ctypes.byref(s), ctypes.byref(p), 0x1000, 16, None) == _abi.FQ_ERR_ARG
    assert "too small" in L.fq_last_error().decode()
    assert L.fq_create(None, ctypes.byref(s), ctypes.byref(p), 0x1000, 16, None) == _abi.FQ_ERR_ARG


def test_null_context_calls_rejected():
    L = _abi.lib()
    g = np.zeros(8)
    assert L.floquet_build_UT(None, FAKE, None) == _abi.FQ_ERR_ARG
    assert L.floquet_propagate(None, FAKE, 1, 0, 1, FAKE, None, 0) == _abi.FQ_ERR_ARG
    assert L.floquet_grad(None, FAKE, _abi.dptr(g)) == _abi.FQ_ERR_ARG
    assert L.floquet_period_average(None, FAKE, 1, _abi.dptr(g), _abi.dptr(g)) == _abi.FQ_ERR_ARG
    assert L.fq_node_times(1.0, 0, _abi.dptr(g)) == _abi.FQ_ERR_ARG
    assert L.fq_bessel_weights(-1.0, 3, _abi.dptr(g)) == _abi.FQ_ERR_ARG
    with pytest.raises(_abi.FloquetError):
        fl.choose_order(1.0, -1.0)


def test_torch_complex_gradient_convention():
    """The backward hands floquet_grad dL/dRe U + i dL/dIm U: check that this is
    what torch supplies as the gradient of a complex tensor for a real loss."""
    torch = pytest.importorskip("torch")
    z = torch.tensor([1.0 + 2.0j, -0.5 + 0.25j], dtype=torch.complex128, requires_grad=True)
    loss = (z.real ** 3 + 2 * z.imag).sum()
    loss.backward()
    expect = 3 * z.detach().real ** 2 + 2j
    assert torch.allclose(z.grad, expect)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 (or a multi-rank launch) exits
    with status 2 and says so, before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for args, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *args],
                           capture_output=True, text=True, timeout=120,
                           env={**os.environ, **env})
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_static_build_rejects_before_device_work():
    """The allocation-free one-shot build checks its arguments and the size of
    the static scratch before any HIP call."""
    L = _abi.lib()
    rep = _abi.FqReport()

    def call(s, p):
        return L.floquet_build_UT_static(ctypes.byref(s), ctypes.byref(p), None, FAKE,
                                         ctypes.byref(rep))

    assert L.floquet_build_UT_static(ctypes.byref(_dense()), ctypes.byref(_params()), None, None,
                                     None) == _abi.FQ_ERR_ARG
    assert call(_dense(0), _params()) == _abi.FQ_ERR_ARG
    assert call(_dense(), _params(checkpoint_every=2)) == _abi.FQ_ERR_UNSUPPORTED
    assert call(_dense(), _params(profile=1)) == _abi.FQ_ERR_UNSUPPORTED
    # 1536 x 1536 FP64 planes do not fit the 256 MiB array; 1408 do
    assert call(_dense(1409), _params()) == _abi.FQ_ERR_ARG
    assert "static scratch" in L.fq_last_error().decode()
    assert _ws(_dense(1408), _params())[1] <= 256 << 20 < _ws(_dense(1409), _params())[1]
    assert call(_dense(1281), _params(precision=2)) == _abi.FQ_ERR_ARG
    assert call(_tridiag(4096), _params()) == _abi.FQ_ERR_ARG


def test_schedule_arguments_rejected():
    """Per-term formats: values, the leading FP64 run, the precision they need,
    and the error target are checked before any device work."""
    def with_formats(fmts, precision=2, tol=0.0):
        arr = (ctypes.c_int32 * max(len(fmts), 1))(*fmts)
        p = _params(precision=precision, mixed_tol=tol)
        if fmts:
            p.term_formats = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
            p.n_term_formats = len(fmts)
        p._arr = arr
        return _ws(_dense(), p)[0]

    assert with_formats([0, 0, 1, 2, 3, 4]) == _abi.FQ_OK
    assert with_formats([2, 0]) == _abi.FQ_ERR_ARG          # FP64 after a BF16 term
    assert with_formats([5]) == _abi.FQ_ERR_ARG
    assert with_formats([-1]) == _abi.FQ_ERR_ARG
    assert with_formats([2], precision=0) == _abi.FQ_ERR_ARG
    assert with_formats([], tol=-1.0) == _abi.FQ_ERR_ARG
    assert with_formats([], tol=math.nan) == _abi.FQ_ERR_ARG
    p = _params(precision=2)
    p.n_term_formats = 3                                    # count without the array
    assert _ws(_dense(), p)[0] == _abi.FQ_ERR_ARG


def test_set_drive_rejects_null_arguments():
    f = np.zeros(8)
    assert _abi.lib().fq_set_drive(None, _abi.dptr(f)) == _abi.FQ_ERR_ARG


def test_grad_pair_sums_flag_values():
    for v, want in ((0, _abi.FQ_OK), (1, _abi.FQ_OK), (2, _abi.FQ_ERR_ARG), (-1, _abi.FQ_ERR_ARG)):
        for sysd in (_dense(), _tridiag()):
            assert _ws(sysd, _params(checkpoint_every=2, grad_pair_sums=v))[0] == want


def _cover(A):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    A = np.ascontiguousarray(A, dtype=np.complex128)
    st = _abi.lib().fq_hermitian_cover(A.shape[0], A.ctypes.data, ctypes.byref(lo),
                                       ctypes.byref(hi))
    assert st == _abi.FQ_OK, _abi.lib().fq_last_error()
    return lo.value, hi.value


def _fixed_start(n):
    """A start vector fixed in advance of the operator (an xorshift sequence
    from a constant seed), for building an operator that defeats it."""
    s = 0x9E3779B97F4A7C15
    mask = (1 << 64) - 1
    out = np.empty(n, complex)
    vals = []
    for _ in range(2 * n):
        s ^= (s << 13) & mask
        s ^= s >> 7
        s ^= (s << 17) & mask
        vals.append((s >> 11) / 9007199254740992.0 - 0.5)
    out.real, out.imag = vals[0::2], vals[1::2]
    return out / np.linalg.norm(out)


def _lanczos_extremes(A, q, k):
    """Plain Lanczos from q (no reorthogonalisation), extreme Ritz values."""
    n = A.shape[0]
    alpha, beta = [], []
    qp = np.zeros(n, complex)
    b = 0.0
    for j in range(min(k, n)):
        w = A @ q - b * qp
        a = np.vdot(q, w).real
        w = w - a * q
        alpha.append(a)
        b = np.linalg.norm(w)
        if b < 1e-12:
            break
        beta.append(b)
        qp, q = q, w / b
    T = np.diag(alpha) + np.diag(beta[:len(alpha) - 1], 1) + np.diag(beta[:len(alpha) - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return ev[0], ev[-1]


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (64, 3), (300, 4), (700, 5)])
def test_hermitian_cover_contains_the_spectrum(n, seed):
    """The dense cover's bound for one operator contains its spectrum (LAPACK
    eigvalsh) and is not wider than the spectrum plus a few per cent."""
    from workloads import gue
    A = gue(n, np.random.default_rng(seed))
    ev = np.linalg.eigvalsh(A)
    lo, hi = _cover(A)
    spread = max(ev[-1] - ev[0], 1e-300)
    assert lo <= ev[0] + 1e-12 and hi >= ev[-1] - 1e-12
    if n > 1:
        assert (ev[0] - lo) < 0.05 * spread and (hi - ev[-1]) < 0.05 * spread


@pytest.mark.parametrize("gap", [4.0, 0.1, 0.02])
def test_hermitian_cover_finds_an_extreme_hidden_from_a_fixed_start(gap):
    """Operators whose largest eigenvalue sits `gap` above a semicircle bulk
    on [-2, 2], with its eigenvector orthogonal to a start vector fixed in
    advance and to the all-ones vector (the library hashes A times it): the
    cover still contains the whole spectrum. (In exact arithmetic Lanczos from
    that fixed start would never see the outlier; in floating point it surfaces
    from rounding noise only after enough steps, later the closer it is to the
    bulk, which is what the margin and the operator-dependent start are for.)"""
    from workloads import gue
    n = 400
    rng = np.random.default_rng(17)
    B = gue(n, rng)
    q0 = _fixed_start(n)
    ones = np.ones(n, complex) / math.sqrt(n)
    Qb, _ = np.linalg.qr(np.stack([q0, ones], 1))
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = v - Qb @ (Qb.conj().T @ v)
    v /= np.linalg.norm(v)
    P = np.eye(n) - np.outer(v, v.conj())
    bulk_top = np.linalg.eigvalsh(P @ B @ P)[-1]
    A = P @ B @ P + (bulk_top + gap) * np.outer(v, v.conj())
    A = 0.5 * (A + A.conj().T)
    ev = np.linalg.eigvalsh(A)
    assert abs(abs(np.vdot(v, q0))) < 1e-12 and ev[-1] > bulk_top + 0.99 * gap
    lo, hi = _cover(A)
    assert hi >= ev[-1] and lo <= ev[0]


def test_hermitian_cover_rejects_bad_arguments():
    lo, hi = ctypes.c_double(), ctypes.c_double()
    A = np.zeros((2, 2), complex)
    A[0, 1] = np.nan
    L = _abi.lib()
    assert L.fq_hermitian_cover(0, A.ctypes.data, ctypes.byref(lo), ctypes.byref(hi)) == _abi.FQ_ERR_ARG
    assert L.fq_hermitian_cover(2, None, ctypes.byref(lo), ctypes.byref(hi)) == _abi.FQ_ERR_ARG
    assert L.fq_hermitian_cover(2, A.ctypes.data, ctypes.byref(lo), ctypes.byref(hi)) == \
        _abi.FQ_ERR_NONFINITE


def test_unitary_eigenphases_match_the_general_eigensolver():
    """The Hermitian (Cayley) route to the eigenphases of a unitary U agrees
    with LAPACK's general eigensolver on Haar-random unitaries (eigenvalues
    spread over the whole circle, some near -1) and on a slightly non-unitary
    U as a mixed-precision build leaves it (second order in the departure)."""
    from paper_1508_07621_amd import analysis
    from workloads import haar_unitary
    rng = np.random.default_rng(5)
    for n in (1, 7, 200):
        U = haar_unitary(n, rng)
        th = analysis.eigenphases_unitary(U)
        ref = orc.eigenphases(U)
        assert len(th) == n and orc.quasienergy_distance(th, ref, 1.0) < 1e-11
    U = haar_unitary(150, rng)
    E = 1e-7 * (rng.standard_normal((150, 150)) + 1j * rng.standard_normal((150, 150))) / 150
    Up = U + E
    th = analysis.eigenphases_unitary(Up)
    ref = np.sort(orc.eigenphases(Up))
    assert orc.quasienergy_distance(th, ref, 1.0) < 1e-9
