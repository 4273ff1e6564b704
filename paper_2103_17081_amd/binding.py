"""ctypes binding of libddhelm.so (include/ddhelm.h).

Argument marshalling only: every numerical step runs in the library's HIP kernels.
Device buffers are torch tensors (complex128 / complex64, contiguous, on the GPU);
their data pointers and torch's current HIP stream are handed to the C ABI.  If the
shared library is missing, or no GPU is present, the calls raise: there is no CPU
fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddhelm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ddhelm.h")

DD_OK, DD_EINVAL, DD_ENOMEM, DD_EHIP, DD_ESINGULAR, DD_ENOTCONV, DD_EWEIGHTS = range(7)
STATUS_NAMES = {0: "DD_OK", 1: "DD_EINVAL", 2: "DD_ENOMEM", 3: "DD_EHIP", 4: "DD_ESINGULAR",
                5: "DD_ENOTCONV", 6: "DD_EWEIGHTS"}
LOCAL_BC = {"impedance": 0, "robin": 0, "dirichlet": 1}
DEFLATION = {"linear": 0, "bezier": 1}


class Params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_double),
        ("ppwl", ctypes.c_double),
        ("n_intervals", ctypes.c_int),
        ("px", ctypes.c_int),
        ("py", ctypes.c_int),
        ("cuts_x", ctypes.POINTER(ctypes.c_int)),
        ("cuts_y", ctypes.POINTER(ctypes.c_int)),
        ("overlap", ctypes.c_int),
        ("local_bc", ctypes.c_int),
        ("deflation", ctypes.c_int),
        ("inner_precision", ctypes.c_int),
        ("inner_tol", ctypes.c_double),
        ("inner_maxit", ctypes.c_int),
        ("outer_tol", ctypes.c_double),
        ("outer_maxit", ctypes.c_int),
        ("outer_restart", ctypes.c_int),
        ("nrhs", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("graph_steps", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int),
        ("precond_applies", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("inner_iters_total", ctypes.c_longlong),
        ("subdomain_solves", ctypes.c_longlong),
        ("inner_iters_max", ctypes.c_int),
        ("guesses_accepted", ctypes.c_longlong),
        ("final_res_estimate", ctypes.c_double),
        ("ms_inner", ctypes.c_double),
        ("ms_spmv", ctypes.c_double),
        ("ms_orth", ctypes.c_double),
        ("ms_other", ctypes.c_double),
        ("inner_launches", ctypes.c_int),
        ("inner_bytes", ctypes.c_double),
        ("ms_dots", ctypes.c_double),
        ("ms_update", ctypes.c_double),
        ("dots_bytes", ctypes.c_double),
        ("update_bytes", ctypes.c_double),
        ("graph_replays", ctypes.c_int),
        ("timed_steps", ctypes.c_int),
        ("ms_steps", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class DDError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_VP = ctypes.c_void_p
_SIGS = {
    "dd_default_params": (None, [ctypes.POINTER(Params)]),
    "dd_setup": (ctypes.c_int, [ctypes.POINTER(Params), _VP, ctypes.POINTER(_VP)]),
    "dd_apply_preconditioner": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dd_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(Stats)]),
    "dd_destroy": (ctypes.c_int, [_VP]),
    "dd_set_graph": (ctypes.c_int, [_VP, ctypes.c_int]),
    "dd_autotune": (ctypes.c_int, [_VP, ctypes.c_char_p, _VP, ctypes.c_char_p, ctypes.c_int]),
    "dd_last_error": (ctypes.c_char_p, []),
    "dd_num_dofs": (ctypes.c_int64, [_VP]),
    "dd_num_subdomains": (ctypes.c_int, [_VP]),
    "dd_num_intervals": (ctypes.c_int, [_VP]),
    "dd_packed_fine_size": (ctypes.c_int64, [_VP]),
    "dd_packed_coarse_size": (ctypes.c_int64, [_VP]),
    "dd_layout": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    "dd_coarse_matrix": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "dd_op_global_apply": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dd_op_local_apply": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "dd_op_deflated_apply": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "dd_op_restrict": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dd_op_prolong": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dd_op_coarse_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dd_op_gather": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "dd_op_scatter": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "dd_op_inner_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), _VP]),
}


def header_functions() -> list[str]:
    """Names of the functions include/ddhelm.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z_0-9]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load libddhelm.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_17081_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != DD_OK:
        raise DDError(status, where, lib().dd_last_error().decode())


def default_params() -> Params:
    p = Params()
    lib().dd_default_params(ctypes.byref(p))
    return p


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the ddhelm library runs only on an MI355X (gfx950)")
    return torch


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Handle on one set-up problem (dd_setup ... dd_destroy)."""

    def __init__(self, k: float, n_intervals: int = 0, ppwl: float = 10.0, px: int = 2, py: int = 2,
                 cuts_x=None, cuts_y=None, overlap: int = 1, local_bc: str = "impedance",
                 deflation: str = "linear", inner_precision: int = 64, inner_tol: float = 1e-2,
                 inner_maxit: int = 100, outer_tol: float = 1e-6, outer_maxit: int = 3000,
                 outer_restart: int = 0, nrhs: int = 1, use_graph: bool = True, graph_steps: int = 8):
        p = default_params()
        p.k, p.ppwl, p.n_intervals = k, ppwl, n_intervals
        p.px, p.py = px, py
        self._cx = self._cy = None
        if cuts_x is not None:
            self._cx = (ctypes.c_int * len(cuts_x))(*[int(c) for c in cuts_x])
            p.cuts_x = ctypes.cast(self._cx, ctypes.POINTER(ctypes.c_int))
            p.px = len(cuts_x) - 1
        if cuts_y is not None:
            self._cy = (ctypes.c_int * len(cuts_y))(*[int(c) for c in cuts_y])
            p.cuts_y = ctypes.cast(self._cy, ctypes.POINTER(ctypes.c_int))
            p.py = len(cuts_y) - 1
        p.overlap = overlap
        p.local_bc = LOCAL_BC[local_bc]
        p.deflation = DEFLATION[deflation]
        p.inner_precision = inner_precision
        p.inner_tol, p.inner_maxit = inner_tol, inner_maxit
        p.outer_tol, p.outer_maxit, p.outer_restart = outer_tol, outer_maxit, outer_restart
        p.nrhs = nrhs
        p.use_graph = 1 if use_graph else 0
        p.graph_steps = graph_steps
        self.params = p
        self._h = ctypes.c_void_p()
        torch = _torch()
        self.torch = torch
        _check(lib().dd_setup(ctypes.byref(p), _stream(torch), ctypes.byref(self._h)), "dd_setup")
        L = lib()
        self.ndof = int(L.dd_num_dofs(self._h))
        self.nsub = int(L.dd_num_subdomains(self._h))
        self.n = int(L.dd_num_intervals(self._h))
        self.nfine = int(L.dd_packed_fine_size(self._h))
        self.ncoarse = int(L.dd_packed_coarse_size(self._h))
        self.nrhs = nrhs
        self.inner_precision = inner_precision
        lay = np.zeros(self.nsub * 12, dtype=np.int32)
        _check(L.dd_layout(self._h, lay.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "dd_layout")
        self.layout = lay.reshape(self.nsub, 12)

    # -- lifetime --
    def close(self):
        if self._h:
            lib().dd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers --
    def _cdtype(self, precision: int):
        return self.torch.complex64 if precision == 32 else self.torch.complex128

    def empty_global(self, nrhs: int = 1):
        return self.torch.empty((nrhs, self.ndof) if nrhs > 1 else (self.ndof,), dtype=self.torch.complex128,
                                device="cuda")

    def coarse_matrix(self, j: int):
        """Host copy of E_j's nine coefficients per coarse node ([nc, 9] complex) and min |pivot|."""
        mx, my = int(self.layout[j, 8]), int(self.layout[j, 9])
        out = np.zeros(mx * my * 9 * 2)
        piv = ctypes.c_double()
        _check(lib().dd_coarse_matrix(self._h, j, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.byref(piv)), "dd_coarse_matrix")
        return out.view(np.complex128).reshape(mx * my, 9), piv.value

    def autotune(self, cache_path=None) -> str:
        buf = ctypes.create_string_buffer(4096)
        path = cache_path.encode() if cache_path else None
        _check(lib().dd_autotune(self._h, path, _stream(self.torch), buf, len(buf)), "dd_autotune")
        return buf.value.decode()

    def set_graph(self, on: bool):
        _check(lib().dd_set_graph(self._h, 1 if on else 0), "dd_set_graph")

    # -- the three calls of the method --
    def apply_preconditioner(self, r, z=None):
        z = self.torch.empty_like(r) if z is None else z
        _check(lib().dd_apply_preconditioner(self._h, _ptr(r), _ptr(z), _stream(self.torch)),
               "dd_apply_preconditioner")
        return z

    def solve(self, f, u=None, check: bool = True):
        u = self.torch.empty_like(f) if u is None else u
        st = Stats()
        status = lib().dd_solve(self._h, _ptr(f), _ptr(u), _stream(self.torch), ctypes.byref(st))
        if check and status not in (DD_OK, DD_ENOTCONV):
            _check(status, "dd_solve")
        out = st.as_dict()
        out["status"] = STATUS_NAMES.get(status, status)
        return u, out

    # -- kernel-level calls --
    def op_global_apply(self, v, w=None):
        w = self.torch.empty_like(v) if w is None else w
        _check(lib().dd_op_global_apply(self._h, _ptr(v), _ptr(w), _stream(self.torch)), "dd_op_global_apply")
        return w

    def op_local_apply(self, v, precision: int = 64, w=None):
        w = self.torch.empty_like(v) if w is None else w
        _check(lib().dd_op_local_apply(self._h, precision, _ptr(v), _ptr(w), _stream(self.torch)),
               "dd_op_local_apply")
        return w

    def op_deflated_apply(self, v, precision: int = 64, w=None):
        w = self.torch.empty_like(v) if w is None else w
        _check(lib().dd_op_deflated_apply(self._h, precision, _ptr(v), _ptr(w), _stream(self.torch)),
               "dd_op_deflated_apply")
        return w

    def op_restrict(self, v):
        t = self.torch.empty(self.ncoarse, dtype=self.torch.complex128, device="cuda")
        _check(lib().dd_op_restrict(self._h, _ptr(v), _ptr(t), _stream(self.torch)), "dd_op_restrict")
        return t

    def op_prolong(self, y):
        v = self.torch.empty(self.nfine, dtype=self.torch.complex128, device="cuda")
        _check(lib().dd_op_prolong(self._h, _ptr(y), _ptr(v), _stream(self.torch)), "dd_op_prolong")
        return v

    def op_coarse_solve(self, t):
        y = self.torch.empty_like(t)
        _check(lib().dd_op_coarse_solve(self._h, _ptr(t), _ptr(y), _stream(self.torch)), "dd_op_coarse_solve")
        return y

    def op_gather(self, r, precision: int = 64):
        f = self.torch.empty(self.nfine, dtype=self._cdtype(precision), device="cuda")
        _check(lib().dd_op_gather(self._h, precision, _ptr(r), _ptr(f), _stream(self.torch)), "dd_op_gather")
        return f

    def op_scatter(self, u, precision: int = 64, z=None):
        z = self.torch.zeros(self.ndof, dtype=self.torch.complex128, device="cuda") if z is None else z
        _check(lib().dd_op_scatter(self._h, precision, _ptr(u), _ptr(z), _stream(self.torch)), "dd_op_scatter")
        return z

    def op_inner_solve(self, f, guess=None):
        """Packed f ([nrhs*nfine], the handle's inner precision) -> (u, iters, flags)."""
        u = self.torch.empty_like(f)
        cnt = self.nsub * self.nrhs
        iters = np.zeros(cnt, dtype=np.int32)
        flags = np.zeros(cnt, dtype=np.int32)
        g = _ptr(guess) if guess is not None else ctypes.c_void_p()
        _check(lib().dd_op_inner_solve(self._h, _ptr(f), g, _ptr(u),
                                       iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       _stream(self.torch)), "dd_op_inner_solve")
        return u, iters, flags


def setup_status(**kw) -> tuple[int, str]:
    """dd_setup's status for parameters that fail validation (host-only, no device work)."""
    p = default_params()
    keep = []
    for key, val in kw.items():
        if key in ("cuts_x", "cuts_y"):
            arr = (ctypes.c_int * len(val))(*[int(c) for c in val])
            keep.append(arr)
            setattr(p, key, ctypes.cast(arr, ctypes.POINTER(ctypes.c_int)))
        elif key == "local_bc":
            p.local_bc = LOCAL_BC[val] if isinstance(val, str) else val
        elif key == "deflation":
            p.deflation = DEFLATION[val] if isinstance(val, str) else val
        else:
            setattr(p, key, val)
    h = ctypes.c_void_p()
    st = lib().dd_setup(ctypes.byref(p), None, ctypes.byref(h))
    msg = lib().dd_last_error().decode()
    if st == DD_OK:
        lib().dd_destroy(h)
    return st, msg
