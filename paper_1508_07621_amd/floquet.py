"""Python binding of libfloquet: argument marshalling around the C ABI.

PyTorch provides device memory (operators, outputs, the workspace) and the
stream; every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import _abi
from ._abi import FqParams, FqReport, FqSystem, check, dptr, lib

__all__ = ["node_times", "bessel_weights", "choose_order", "tridiag_extremes",
           "FloquetContext", "floquet_build_UT", "floquet_build_UT_static", "floquet_propagate",
           "floquet_grad", "FloquetUT"]


def _torch():
    import torch
    return torch


# ---- host numerics exported by the library ---------------------------------------------------

def node_times(T: float, M: int, scheme: str = "magnus4") -> np.ndarray:
    """Gauss-Legendre sampling times of the drive in time order: (M, 2) for
    "magnus4" and "cf4", (M, 3) for "magnus6"."""
    if scheme == "magnus6":
        out = np.empty(3 * M, dtype=np.float64)
        check(lib().fq_node_times_magnus6(float(T), int(M), dptr(out)))
        return out.reshape(M, 3)
    if scheme not in ("magnus4", "cf4"):
        raise ValueError("scheme must be magnus4, magnus6 or cf4")
    out = np.empty(2 * M, dtype=np.float64)
    check(lib().fq_node_times(float(T), int(M), dptr(out)))
    return out.reshape(M, 2)


def bessel_weights(R: float, L: int) -> np.ndarray:
    """a_0 = J_0(R), a_l = 2 J_l(R) for l = 1..L."""
    out = np.empty(L + 1, dtype=np.float64)
    check(lib().fq_bessel_weights(float(R), int(L), dptr(out)))
    return out


def choose_order(R: float, tol: float) -> int:
    import ctypes
    L = ctypes.c_int32(0)
    check(lib().fq_choose_order(float(R), float(tol), ctypes.byref(L)))
    return int(L.value)


def tridiag_extremes(d, e_abs):
    import ctypes
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e_abs, dtype=np.float64)
    if e.size == 0:
        e = np.zeros(1)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    check(lib().fq_tridiag_extremes(len(d), dptr(d), dptr(e), ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


# ---- context ---------------------------------------------------------------------------------

def _device_tensor(x, dtype, device):
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch tensor or NumPy array")
    return x.to(device=device, dtype=dtype).contiguous()


def _marshal(self, *, T: float, M: int, f_nodes, h0=None, hmod=None, h0_eigenvalues=None,
             h0_diag=None, h0_off=None, hmod_diag=None, e_min: Optional[float] = None,
             e_max: Optional[float] = None, L: int = 0, tol: float = 1e-12,
             precision: str = "fp64", checkpoint_every: int = 0, profile: bool = False,
             reorthonormalize: bool = False, dtype: str = "complex128", scheme: str = "magnus4",
             mixed_tol: float = 0.0, term_formats=None, grad_pair_sums: bool = False,
             device=None):
    """Device copies of the operators and the fq_system / fq_params structures
    of one problem (arguments as for FloquetContext), set on `self`."""
    import ctypes
    torch = _torch()
    self.device = torch.device(device if device is not None else "cuda")
    self._keep = []
    sysd = FqSystem()
    drives = list(hmod) if isinstance(hmod, (list, tuple)) else None
    self.S = len(drives) if drives else 1

    def set_drives(n):
        if drives is None:
            vt = _device_tensor(hmod, torch.complex128, self.device)
            if vt.shape != (n, n):
                raise ValueError("hmod must be n x n")
            sysd.hmod = vt.data_ptr()
            self._keep.append(vt)
            return
        vts = [_device_tensor(v, torch.complex128, self.device) for v in drives]
        if any(v.shape != (n, n) for v in vts):
            raise ValueError("every drive matrix must be n x n")
        arr = (ctypes.c_void_p * len(vts))(*[v.data_ptr() for v in vts])
        sysd.n_drive = len(vts)
        sysd.hmods = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        self._keep += vts + [arr]

    if h0_eigenvalues is not None:
        e = _device_tensor(h0_eigenvalues, torch.float64, self.device)
        self.n = int(e.shape[0])
        sysd.n, sysd.layout = self.n, _abi.FQ_DENSE_EIGEN
        sysd.h0_diag = e.data_ptr()
        self._keep.append(e)
        set_drives(self.n)
    elif h0 is not None:
        h0t = _device_tensor(h0, torch.complex128, self.device)
        self.n = int(h0t.shape[0])
        if h0t.shape != (self.n, self.n):
            raise ValueError("h0 must be square")
        sysd.n, sysd.layout = self.n, _abi.FQ_DENSE
        sysd.h0 = h0t.data_ptr()
        self._keep.append(h0t)
        set_drives(self.n)
    else:
        d = _device_tensor(h0_diag, torch.float64, self.device)
        v = _device_tensor(hmod_diag, torch.float64, self.device)
        self.n = int(d.shape[0])
        off = _device_tensor(h0_off if h0_off is not None else np.zeros(max(self.n - 1, 0)),
                             torch.complex128, self.device)
        if v.shape[0] != self.n or off.shape[0] != max(self.n - 1, 0):
            raise ValueError("tridiagonal arrays have inconsistent sizes")
        sysd.n, sysd.layout = self.n, _abi.FQ_TRIDIAG
        sysd.h0_diag, sysd.hmod_diag = d.data_ptr(), v.data_ptr()
        sysd.h0_off = off.data_ptr() if self.n > 1 else None
        self._keep += [d, v, off]
    self.layout = sysd.layout
    self.M = int(M)
    self.T = float(T)
    if scheme not in _abi.SCHEMES:
        raise ValueError("scheme must be magnus4, magnus6 or cf4")
    self.scheme = scheme
    per_step = (3 if scheme == "magnus6" else 2) * self.S
    self._f = np.ascontiguousarray(np.asarray(f_nodes, dtype=np.float64).reshape(-1))
    if self._f.size != per_step * self.M:
        raise ValueError(f"f_nodes must hold {per_step}*M values for {scheme}")
    par = FqParams()
    par.T, par.M, par.L = self.T, self.M, int(L)
    par.f_nodes = dptr(self._f)
    par.e_min = math.nan if e_min is None else float(e_min)
    par.e_max = math.nan if e_max is None else float(e_max)
    par.tol = float(tol)
    par.precision = _abi.PRECISIONS[precision]
    par.checkpoint_every = int(checkpoint_every)
    par.profile = 1 if profile else 0
    par.reorthonormalize = 1 if reorthonormalize else 0
    if dtype not in ("complex128", "complex64"):
        raise ValueError("dtype must be complex128 or complex64")
    par.dtype = _abi.FQ_C64 if dtype == "complex64" else _abi.FQ_C128
    par.scheme = _abi.SCHEMES[scheme]
    par.mixed_tol = float(mixed_tol)
    par.grad_pair_sums = 1 if grad_pair_sums else 0
    self.grad_pair_sums = bool(grad_pair_sums)
    if term_formats is not None:
        tf = [_abi.TERM_FORMATS[f] if isinstance(f, str) else int(f) for f in term_formats]
        self._tf = (ctypes.c_int32 * len(tf))(*tf)
        par.term_formats = ctypes.cast(self._tf, ctypes.POINTER(ctypes.c_int32))
        par.n_term_formats = len(tf)
    self.state_dtype = torch.complex64 if dtype == "complex64" else torch.complex128
    self.precision = precision
    self._sys, self._par = sysd, par


class FloquetContext:
    """One problem H(t) = H0 + f(t) Hmod on one GPU, set up once, built many times.

    Dense operators: h0, hmod (n x n complex; a list of 2..4 such matrices for
    H0 + sum_s f_s(t) Hmod_s, with f_nodes of shape (M, nodes, S)). In the eigenbasis of H0 (the
    paper's working basis): h0_eigenvalues (n real) and hmod (n x n complex in
    that basis). Tridiagonal: h0_diag (n real), h0_off (n-1 complex,
    H0[i][i+1]), hmod_diag (n real).
    f_nodes: drive samples at node_times(T, M, scheme): (M, 2) for "magnus4"
    and "cf4" (commutator-free, two exponentials per step), (M, 3) for
    "magnus6" (the paper's sixth-order scheme; dense operators, no gradient).
    precision: "fp64", "fp32" or "bf16x3" (arithmetic of the Chebyshev products).
    For "bf16x3" each term's product format is chosen from its Bessel weight so
    that the estimated rounding error of U_T stays below mixed_tol (0 = the
    library's default, 5e-7); term_formats (names of _abi.TERM_FORMATS or their
    values, for terms 1, 2, ...; the last repeats) fixes them instead.
    grad_pair_sums: grad() then gives only each step's node sum correctly
    (dL/dA_k for an amplitude moving both nodes of step k, returned as two
    equal halves), skipping the commutator contraction that cancels in it.
    reorthonormalize: replace U_T by its polar factor after each build (FP64
    Newton-Schulz); the report keeps the unitarity before and after.
    dtype: "complex128" or "complex64", storage of U_T, X and U_bar (the
    operators stay complex128 / float64).
    """

    def __init__(self, **kw):
        torch = _torch()
        _marshal(self, **kw)
        L_ = lib()
        sysd, par = self._sys, self._par
        import ctypes
        nbytes = ctypes.c_size_t(0)
        check(L_.fq_workspace_bytes(ctypes.byref(sysd), ctypes.byref(par), ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._stream = torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L_.fq_create(ctypes.byref(handle), ctypes.byref(sysd), ctypes.byref(par),
                               self.workspace.data_ptr(), nbytes.value, self._stream.cuda_stream))
        self._ctx = handle

    @property
    def report(self) -> dict:
        import ctypes
        r = FqReport()
        check(lib().fq_get_report(self._ctx, ctypes.byref(r)))
        return r.as_dict()

    def build_ut(self, out=None):
        """U_T as an n x n tensor of the context's dtype ([i, j] = <i|U_T|j>)."""
        import ctypes
        torch = _torch()
        self.generation = getattr(self, "generation", 0) + 1  # the tape this build records
        if out is None:
            out = torch.empty((self.n, self.n), dtype=self.state_dtype, device=self.device)
        if out.dtype != self.state_dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of the context's dtype")
        r = FqReport()
        with torch.cuda.device(self.device):
            check(lib().floquet_build_UT(self._ctx, out.data_ptr(), ctypes.byref(r)))
        self.last_report = r.as_dict()
        return out

    def propagate(self, X0, k0: int = 0, k1: Optional[int] = None, out=None, snap_every: int = 0):
        """E_k1 ... E_{k0+1} X0 for an n x ncols complex block X0 (columns = states).
        With snap_every > 0 also returns the states after steps k0 + j snap_every
        as a ((k1 - k0) // snap_every, n, ncols) tensor."""
        torch = _torch()
        k1 = self.M if k1 is None else int(k1)
        X0 = _device_tensor(X0, self.state_dtype, self.device)
        if X0.dim() != 2 or X0.shape[0] != self.n:
            raise ValueError("X0 must be n x ncols")
        if out is None:
            out = torch.empty_like(X0)
        snaps = None
        if snap_every > 0:
            count = (k1 - int(k0)) // int(snap_every)
            snaps = torch.empty((max(count, 1),) + tuple(X0.shape), dtype=self.state_dtype,
                                device=self.device)[:count]
        with torch.cuda.device(self.device):
            check(lib().floquet_propagate(self._ctx, X0.data_ptr(), int(X0.shape[1]), int(k0), k1,
                                          out.data_ptr(),
                                          snaps.data_ptr() if snaps is not None else None,
                                          int(snap_every)))
        return (out, snaps) if snaps is not None else out

    def period_average(self, X0, f_grid) -> np.ndarray:
        """(1/M) sum_k <x_k|H(t_k)|x_k> / <x_k|x_k> for each column of X0 (n x ncols),
        x_k the column propagated over k steps, t_k = k h, f_grid[k] = f(t_k)."""
        X0 = _device_tensor(X0, self.state_dtype, self.device)
        if X0.dim() != 2 or X0.shape[0] != self.n:
            raise ValueError("X0 must be n x ncols")
        fg = np.ascontiguousarray(np.asarray(f_grid, dtype=np.float64).reshape(-1))
        if fg.size != self.M * self.S:
            raise ValueError("f_grid must hold M values per drive term")
        out = np.empty(int(X0.shape[1]), dtype=np.float64)
        torch = _torch()
        with torch.cuda.device(self.device):
            check(lib().floquet_period_average(self._ctx, X0.data_ptr(), int(X0.shape[1]),
                                               dptr(fg), dptr(out)))
        return out

    def grad(self, U_bar) -> np.ndarray:
        """d loss / d f_nodes, shape (M, 2), for U_bar = dL/dRe U + i dL/dIm U."""
        torch = _torch()
        ub = _device_tensor(U_bar, self.state_dtype, self.device)
        g = np.empty(2 * self.M * self.S, dtype=np.float64)
        with torch.cuda.device(self.device):
            check(lib().floquet_grad(self._ctx, ub.data_ptr(), dptr(g)))
        return g.reshape(self.M, 2) if self.S == 1 else g.reshape(self.M, 2, self.S)

    def set_drive(self, f_nodes):
        """New drive samples (same shape as at creation) for this context:
        fq_set_drive redoes the drive-dependent setup and keeps the operators,
        their commutators and the workspace. Drops the gradient tape."""
        f = np.ascontiguousarray(np.asarray(f_nodes, dtype=np.float64).reshape(-1))
        if f.size != self._f.size:
            raise ValueError(f"f_nodes must hold {self._f.size} values")
        torch = _torch()
        with torch.cuda.device(self.device):
            check(lib().fq_set_drive(self._ctx, dptr(f)))
        self._f = f
        self.generation = getattr(self, "generation", 0) + 1

    def close(self):
        if getattr(self, "_ctx", None):
            lib().fq_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- one-shot wrappers with the entry points' names -----------------------------------------

def floquet_build_UT(**kw):
    """Build U_T in one call; returns (U_T tensor, report dict)."""
    ctx = FloquetContext(**kw)
    U = ctx.build_ut()
    rep = ctx.last_report
    ctx.close()
    return U, rep


def floquet_propagate(X0, k0=0, k1=None, **kw):
    ctx = FloquetContext(**kw)
    X = ctx.propagate(X0, k0, k1)
    ctx.close()
    return X


def floquet_grad(U_bar, **kw):
    ctx = FloquetContext(**kw)
    ctx.build_ut()
    g = ctx.grad(U_bar)
    ctx.close()
    return g


def floquet_build_UT_static(out=None, **kw):
    """U_T through the allocation-free one-shot entry point: the library takes
    its workspace from its static device array (no workspace tensor, no context
    kept). Arguments as for FloquetContext (checkpoint_every and profile must
    be off). Returns (U_T tensor, report dict); the report's ms_build is 0."""
    import ctypes
    torch = _torch()

    class _Problem:
        pass

    prob = _Problem()
    _marshal(prob, **kw)
    if out is None:
        out = torch.empty((prob.n, prob.n), dtype=prob.state_dtype, device=prob.device)
    if out.dtype != prob.state_dtype or not out.is_contiguous() or out.shape != (prob.n, prob.n):
        raise ValueError("out must be a contiguous n x n tensor of the problem's dtype")
    r = FqReport()
    stream = torch.cuda.current_stream(prob.device)
    with torch.cuda.device(prob.device):
        check(lib().floquet_build_UT_static(ctypes.byref(prob._sys), ctypes.byref(prob._par),
                                            stream.cuda_stream, out.data_ptr(), ctypes.byref(r)))
    return out, r.as_dict()


class FloquetUT:
    """torch.autograd.Function wrapper: forward builds U_T with a tape,
    backward returns d loss / d f_nodes through floquet_grad.

    apply(f_nodes, context=ctx) reuses one FloquetContext (created with
    checkpoint_every > 0) across calls: each forward sets the context's drive
    (fq_set_drive) and builds, so the operator setup runs once. A backward must
    then come before the context's next build (its tape is the last build's);
    otherwise it raises. Without a context each forward creates its own from
    the keyword arguments."""

    @staticmethod
    def apply(f_nodes, context=None, **kw):
        torch = _torch()

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx_, f):
                fn = f.detach().cpu().numpy()
                if context is None:
                    c = FloquetContext(f_nodes=fn, **kw)
                else:
                    c = context
                    c.set_drive(fn)
                ctx_.fq = c
                U = c.build_ut()
                ctx_.generation = c.generation
                return U

            @staticmethod
            def backward(ctx_, gU):
                c = ctx_.fq
                if c.generation != ctx_.generation:
                    raise RuntimeError("the context was rebuilt after this forward: its "
                                       "gradient tape belongs to a later build")
                g = c.grad(gU)
                if context is None:
                    c.close()
                return torch.from_numpy(g).to(device=f_nodes.device,
                                              dtype=f_nodes.dtype).reshape(f_nodes.shape)

        return _Fn.apply(f_nodes)
