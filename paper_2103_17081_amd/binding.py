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
LOCAL_SOLVER = {"deflated": 0, "deflated_gmres": 0, "direct": 1}
INNER_LAUNCH = {"fused": 0, "multi": 1}


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
        ("local_solver", ctypes.c_int),
        ("coarse_intervals", ctypes.c_int),
        ("inner_launch", ctypes.c_int),
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
        ("ms_guess", ctypes.c_double),
        ("ms_coarse", ctypes.c_double),
        ("coarse_bytes", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class NetParams(ctypes.Structure):
    _fields_ = [
        ("widths", ctypes.c_int * 4),
        ("tile", ctypes.c_int),
        ("max_batch", ctypes.c_int),
        ("train", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
    ]


class TileDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("edges", ctypes.c_int),
        ("robin", ctypes.c_int),
        ("kh", ctypes.c_double),
    ]


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
    "dd_op_inner_solve_static": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32), _VP]),
    "dd_net_default_params": (None, [ctypes.POINTER(NetParams)]),
    "dd_net_create": (ctypes.c_int, [ctypes.POINTER(NetParams), ctypes.POINTER(_VP)]),
    "dd_net_destroy": (ctypes.c_int, [_VP]),
    "dd_net_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)]),
    "dd_net_num_params": (ctypes.c_int64, [_VP]),
    "dd_net_set_params": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "dd_net_get_params": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "dd_net_forward": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP, _VP]),
    "dd_net_gradient": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(TileDesc), ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "dd_net_adam": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _VP]),
    "dd_set_guess": (ctypes.c_int, [_VP, _VP]),
    "dd_tiles": (ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP, _VP, _VP]),
    "dd_packed_to_tiles": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP, _VP]),
    "dd_tile_descs": (ctypes.c_int, [_VP, ctypes.POINTER(TileDesc)]),
    "dd_outer_basis": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP]),
    "dd_last_inner": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _VP]),
    "dd_global_coarse_size": (ctypes.c_int64, [_VP]),
    "dd_global_coarse_matrix": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "dd_op_global_restrict": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dd_op_global_coarse_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "dd_op_global_correct": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
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
        # torch ships its own HIP runtime: load it first so that this library binds to the
        # same runtime instance (two runtimes in one process cannot see each other's code)
        import torch  # noqa: F401
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
                 outer_restart: int = 0, nrhs: int = 1, use_graph: bool = True, graph_steps: int = 8,
                 local_solver: str = "deflated", coarse_intervals: int = 0, inner_launch: str = "fused"):
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
        p.local_solver = LOCAL_SOLVER[local_solver]
        p.coarse_intervals = coarse_intervals
        p.inner_launch = INNER_LAUNCH[inner_launch]
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
        self.nglobal_coarse = int(L.dd_global_coarse_size(self._h))
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
        """Host copy of E_j's coefficients per coarse node ([nc, 9] complex for linear deflation,
        [nc, 25] for Bezier) and min |pivot|."""
        mx, my = int(self.layout[j, 8]), int(self.layout[j, 9])
        K = 9 if self.params.deflation == 0 else 25
        out = np.zeros(mx * my * K * 2)
        piv = ctypes.c_double()
        _check(lib().dd_coarse_matrix(self._h, j, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.byref(piv)), "dd_coarse_matrix")
        return out.view(np.complex128).reshape(mx * my, K), piv.value

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

    def op_inner_solve_static(self, f, u=None, counts: bool = True):
        """dd_op_inner_solve_static: packed f -> (u, iters, flags); with counts=False nothing is
        copied back and the call does not synchronise (iters, flags are None)."""
        u = self.torch.empty_like(f) if u is None else u
        if counts:
            cnt = self.nsub * self.nrhs
            iters = np.zeros(cnt, dtype=np.int32)
            flags = np.zeros(cnt, dtype=np.int32)
            ip = iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            fp = flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        else:
            iters = flags = None
            ip = fp = None
        _check(lib().dd_op_inner_solve_static(self._h, _ptr(f), _ptr(u), ip, fp, _stream(self.torch)),
               "dd_op_inner_solve_static")
        return u, iters, flags

    # -- two-level method --
    def global_coarse_matrix(self):
        """E_0's coefficients ([(M-1)^2, 9] float64, neighbour (dx, dy) at 3(dy+1) + (dx+1)) and
        the smallest |pivot| of its block cyclic reduction."""
        out = np.zeros(self.nglobal_coarse * 9)
        piv = ctypes.c_double()
        _check(lib().dd_global_coarse_matrix(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             ctypes.byref(piv)), "dd_global_coarse_matrix")
        return out.reshape(self.nglobal_coarse, 9), piv.value

    def op_global_restrict(self, r):
        t = self.torch.empty(self.nglobal_coarse, dtype=self.torch.complex128, device="cuda")
        _check(lib().dd_op_global_restrict(self._h, _ptr(r), _ptr(t), _stream(self.torch)), "dd_op_global_restrict")
        return t

    def op_global_coarse_solve(self, t):
        y = self.torch.empty_like(t)
        _check(lib().dd_op_global_coarse_solve(self._h, _ptr(t), _ptr(y), _stream(self.torch)),
               "dd_op_global_coarse_solve")
        return y

    def op_global_correct(self, r, y):
        """(q, w) = (Z_0 y, r - A Z_0 y)."""
        q = self.torch.empty_like(r)
        w = self.torch.empty_like(r)
        _check(lib().dd_op_global_correct(self._h, _ptr(r), _ptr(y), _ptr(q), _ptr(w), _stream(self.torch)),
               "dd_op_global_correct")
        return q, w

    # -- learned initial guess --
    def set_guess(self, net):
        """Attach a GuessNet (None detaches); the network must outlive the attachment."""
        _check(lib().dd_set_guess(self._h, net._n if net is not None else None), "dd_set_guess")
        self._net = net

    def tiles(self, r, tile: int):
        """Network input tiles of R_j r for every subdomain / rhs and their scales."""
        B = self.nsub * self.nrhs
        x = self.torch.empty((B, tile, tile, 4), dtype=self.torch.float32, device="cuda")
        s = self.torch.empty(B, dtype=self.torch.float64, device="cuda")
        _check(lib().dd_tiles(self._h, _ptr(r), tile, _ptr(x), _ptr(s), _stream(self.torch)), "dd_tiles")
        return x, s

    def packed_to_tiles(self, u, scale, tile: int):
        B = self.nsub * self.nrhs
        t = self.torch.empty((B, tile, tile, 2), dtype=self.torch.float32, device="cuda")
        _check(lib().dd_packed_to_tiles(self._h, _ptr(u), _ptr(scale), tile, _ptr(t), _stream(self.torch)),
               "dd_packed_to_tiles")
        return t

    def tile_descs(self):
        arr = (TileDesc * self.nsub)()
        _check(lib().dd_tile_descs(self._h, arr), "dd_tile_descs")
        return arr

    def last_inner(self):
        """Per-solve inner iteration counts and flags of the last batched launch."""
        cnt = self.nsub * self.nrhs
        iters = np.zeros(cnt, dtype=np.int32)
        flags = np.zeros(cnt, dtype=np.int32)
        _check(lib().dd_last_inner(self._h, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream(self.torch)),
               "dd_last_inner")
        return iters, flags

    def outer_basis(self, j: int):
        v = self.torch.empty((self.nrhs, self.ndof) if self.nrhs > 1 else (self.ndof,),
                             dtype=self.torch.complex128, device="cuda")
        _check(lib().dd_outer_basis(self._h, j, _ptr(v), _stream(self.torch)), "dd_outer_basis")
        return v


def weights_header(path: str) -> dict:
    """JSON header of a guess-network weights file (magic, uint32 length, JSON)."""
    import json
    import struct
    with open(path, "rb") as fh:
        fh.read(8)
        (hl,) = struct.unpack("<I", fh.read(4))
        return json.loads(fh.read(hl).decode())


def default_net_params() -> NetParams:
    p = NetParams()
    lib().dd_net_default_params(ctypes.byref(p))
    return p


class GuessNet:
    """Handle on one guess network (dd_net_create ... dd_net_destroy)."""

    def __init__(self, widths=(16, 32, 64, 64), tile: int = 64, max_batch: int = 256, train: bool = False,
                 seed: int | None = None):
        p = default_net_params()
        for i, w in enumerate(widths):
            p.widths[i] = int(w)
        p.tile, p.max_batch, p.train = tile, max_batch, 1 if train else 0
        if seed is not None:
            p.seed = seed
        torch = _torch()
        self.torch = torch
        self._n = ctypes.c_void_p()
        _check(lib().dd_net_create(ctypes.byref(p), ctypes.byref(self._n)), "dd_net_create")
        self.widths, self.tile, self.max_batch = tuple(int(w) for w in widths), tile, max_batch
        self.nparams = int(lib().dd_net_num_params(self._n))

    @classmethod
    def load(cls, path: str, max_batch: int, tile: int = 0) -> "GuessNet":
        """Inference network from a weights file, read and validated by dd_net_load
        (DD_EWEIGHTS for a bad file); tile 0 takes the file's tile."""
        torch = _torch()
        h = ctypes.c_void_p()
        _check(lib().dd_net_load(os.fsencode(path), int(tile), int(max_batch), ctypes.byref(h)), "dd_net_load")
        self = cls.__new__(cls)
        self.torch, self._n, self.max_batch = torch, h, max_batch
        self.nparams = int(lib().dd_net_num_params(h))
        head = weights_header(path)      # already validated by the library
        self.widths = tuple(int(w) for w in head["widths"])
        self.tile = int(tile) if tile > 0 else int(head["tile"])
        return self

    def close(self):
        if self._n:
            lib().dd_net_destroy(self._n)
            self._n = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().dd_net_get_params(self._n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), self.nparams),
               "dd_net_get_params")
        return out

    def set_params(self, v):
        v = np.ascontiguousarray(v, dtype=np.float32)
        _check(lib().dd_net_set_params(self._n, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), v.size),
               "dd_net_set_params")

    def forward(self, x):
        """x: float32 GPU tensor [B, T, T, 4] -> y [B, T, T, 2]."""
        y = self.torch.empty(x.shape[:3] + (2,), dtype=self.torch.float32, device="cuda")
        _check(lib().dd_net_forward(self._n, _ptr(x), x.shape[0], _ptr(y), _stream(self.torch)), "dd_net_forward")
        return y

    def gradient(self, x, t, desc, w_res: float = 1.0, w_err: float = 0.0, want_grad: bool = False):
        """Loss (and, if asked, the gradient as a GPU tensor) for a batch; desc: TileDesc array."""
        g = self.torch.empty(self.nparams, dtype=self.torch.float32, device="cuda") if want_grad else None
        loss = ctypes.c_double()
        _check(lib().dd_net_gradient(self._n, _ptr(x), _ptr(t), desc, x.shape[0], w_res, w_err,
                                     _ptr(g) if g is not None else None, ctypes.byref(loss), _stream(self.torch)),
               "dd_net_gradient")
        return loss.value, g

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(lib().dd_net_adam(self._n, lr, beta1, beta2, eps, _stream(self.torch)), "dd_net_adam")


def net_create_status(**kw) -> tuple[int, str]:
    """dd_net_create's status for parameters that fail validation (host-only, no device work)."""
    p = default_net_params()
    for key, val in kw.items():
        if key == "widths":
            for i, w in enumerate(val):
                p.widths[i] = w
        else:
            setattr(p, key, val)
    n = ctypes.c_void_p()
    st = lib().dd_net_create(ctypes.byref(p), ctypes.byref(n))
    msg = lib().dd_last_error().decode()
    if st == DD_OK:
        lib().dd_net_destroy(n)
    return st, msg


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
        elif key == "local_solver":
            p.local_solver = LOCAL_SOLVER[val] if isinstance(val, str) else val
        elif key == "inner_launch":
            p.inner_launch = INNER_LAUNCH[val] if isinstance(val, str) else val
        else:
            setattr(p, key, val)
    h = ctypes.c_void_p()
    st = lib().dd_setup(ctypes.byref(p), None, ctypes.byref(h))
    msg = lib().dd_last_error().decode()
    if st == DD_OK:
        lib().dd_destroy(h)
    return st, msg
