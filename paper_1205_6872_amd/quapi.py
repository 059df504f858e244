"""Thin Python binding of libquapi.so (argument marshalling only).

Every computation runs in the HIP library; this module converts NumPy inputs
into the C structs of include/quapi.h, calls the C ABI through ctypes, and
turns status codes into exceptions.  The functions keep the C names without
the ``quapi_`` prefix (``create``, ``propagate``, ``propagate_async``,
``footprint``, ...).  PyTorch is used only to hand over device memory and
streams (``workspace=`` / ``stream=``).

The library must be built (``python -m paper_1205_6872_amd.build`` or the
repository's build step); importing this module on a machine without it
raises ``ImportError`` -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
from pathlib import Path
from typing import Optional, Sequence

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "_lib" / "libquapi.so"

OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_STATE = 0, 1, 2, 3, 4
C128, C64, C64_F64 = 0, 1, 2
DTYPES = {"c128": C128, "c64": C64, "c64f64": C64_F64}
BATH_OHMIC, BATH_TABLE = 0, 1
SETUP_G, SETUP_ETA, SETUP_U, SETUP_K = 0, 1, 2, 3

EXPORTED_SYMBOLS = (
    "quapi_footprint", "quapi_paper_pmc_bytes", "quapi_create", "quapi_propagate",
    "quapi_propagate_async", "quapi_step_count", "quapi_fused_steps", "quapi_set_fused_steps",
    "quapi_mirror", "quapi_set_mirror",
    "quapi_get_setup", "quapi_read_tensor", "quapi_restore",
    "quapi_tensor_size", "quapi_set_timing", "quapi_get_timing", "quapi_destroy",
    "quapi_last_error", "quapi_copy_bandwidth", "quapi_propagate_static",
    "quapi_persistent", "quapi_propagate_batch",
    "quapi_filtered_footprint", "quapi_create_filtered", "quapi_filter_stats", "quapi_filter_read",
)

_DP = ctypes.POINTER(ctypes.c_double)


class Bath(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("xi", ctypes.c_double), ("omega_c", ctypes.c_double),
                ("omega", _DP), ("J", _DP), ("n_tab", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("s", _DP), ("H", _DP), ("rho0", _DP), ("bath", Bath),
                ("kT", ctypes.c_double), ("dt", ctypes.c_double), ("dk_max", ctypes.c_int),
                ("dtype", ctypes.c_int), ("H_t", _DP), ("n_H", ctypes.c_int)]


class Timing(ctypes.Structure):
    _fields_ = [("setup_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("step_launches", ctypes.c_longlong), ("step_steps", ctypes.c_longlong),
                ("grow_ms", ctypes.c_double),
                ("grow_launches", ctypes.c_longlong), ("finalize_ms", ctypes.c_double),
                ("finalize_launches", ctypes.c_longlong), ("width_ms", ctypes.c_double * 4),
                ("width_launches", ctypes.c_longlong * 4)]


class QuapiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[status {status}] {message}")
        self.status = status


def load_library() -> ctypes.CDLL:
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is not built; run the build step (hipcc for gfx950) first")
    lib = ctypes.CDLL(str(LIB_PATH))
    vp, sz, ip = ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int)
    lib.quapi_footprint.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(sz)]
    lib.quapi_paper_pmc_bytes.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.quapi_paper_pmc_bytes.restype = sz
    lib.quapi_create.argtypes = [ctypes.POINTER(Params), vp, vp, sz, ctypes.POINTER(vp)]
    lib.quapi_propagate.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, _DP]
    lib.quapi_propagate_async.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, vp]
    lib.quapi_step_count.argtypes = [vp, ip]
    lib.quapi_fused_steps.argtypes = [vp, ip]
    lib.quapi_set_fused_steps.argtypes = [vp, ctypes.c_int]
    lib.quapi_mirror.argtypes = [vp, ip]
    lib.quapi_set_mirror.argtypes = [vp, ctypes.c_int]
    lib.quapi_get_setup.argtypes = [vp, ctypes.c_int, _DP, sz]
    lib.quapi_read_tensor.argtypes = [vp, sz, sz, _DP]
    lib.quapi_restore.argtypes = [vp, ctypes.c_int, _DP, sz]
    lib.quapi_tensor_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.quapi_set_timing.argtypes = [vp, ctypes.c_int]
    lib.quapi_get_timing.argtypes = [vp, ctypes.POINTER(Timing)]
    lib.quapi_destroy.argtypes = [vp]
    lib.quapi_copy_bandwidth.argtypes = [vp, vp, sz, sz, ctypes.c_int, vp]
    lib.quapi_propagate_static.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ip, ctypes.c_int, vp, vp]
    lib.quapi_persistent.argtypes = [vp, ip]
    lib.quapi_propagate_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ip, ip, ctypes.POINTER(vp)]
    lib.quapi_filtered_footprint.argtypes = [ctypes.POINTER(Params), sz, ctypes.POINTER(sz)]
    lib.quapi_create_filtered.argtypes = [ctypes.POINTER(Params), ctypes.c_double, sz, vp, ctypes.POINTER(vp)]
    lib.quapi_filter_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ip]
    lib.quapi_filter_read.argtypes = [vp, sz, sz, ctypes.POINTER(ctypes.c_longlong), _DP]
    lib.quapi_last_error.argtypes = [vp]
    lib.quapi_last_error.restype = ctypes.c_char_p
    for name in EXPORTED_SYMBOLS:
        if name not in ("quapi_paper_pmc_bytes", "quapi_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(status: int, ctx=None):
    if status != OK:
        msg = lib().quapi_last_error(ctx).decode(errors="replace")
        raise QuapiError(status, msg)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _c128_ri(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).view(np.float64)


def _ptr(a: Optional[np.ndarray]):
    return a.ctypes.data_as(_DP) if a is not None else None


class _ParamsHolder:
    """Params struct plus the arrays it points into (kept alive together)."""

    def __init__(self, M: int, s, H, rho0, kT: float, dt: float, L: int, dtype: str = "c128",
                 bath_kind: str = "ohmic", xi: float = 0.0, omega_c: float = 1.0,
                 omega_tab=None, J_tab=None, H_t=None):
        self.s = _f64(s)
        self.H = np.ascontiguousarray(_c128_ri(H))
        self.rho0 = np.ascontiguousarray(_c128_ri(rho0))
        self.omega = _f64(omega_tab) if omega_tab is not None else None
        self.J = _f64(J_tab) if J_tab is not None else None
        kind = {"ohmic": BATH_OHMIC, "table": BATH_TABLE}[bath_kind]
        n_tab = int(len(self.omega)) if self.omega is not None else 0
        bath = Bath(kind, float(xi), float(omega_c), _ptr(self.omega), _ptr(self.J), n_tab)
        self.H_t = None if H_t is None else np.ascontiguousarray(_c128_ri(np.asarray(H_t).reshape(-1, M, M)))
        n_H = 0 if H_t is None else int(np.asarray(H_t).reshape(-1, M, M).shape[0])
        self.p = Params(int(M), _ptr(self.s), _ptr(self.H), _ptr(self.rho0), bath, float(kT), float(dt),
                        int(L), DTYPES[dtype], _ptr(self.H_t), n_H)

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(M=w.M, s=w.s, H=w.H, rho0=w.rho0, kT=w.kT, dt=w.dt, L=w.L, dtype=w.dtype,
                  bath_kind=w.bath_kind, xi=w.xi, omega_c=w.omega_c, omega_tab=w.omega_tab,
                  J_tab=w.J_tab, H_t=getattr(w, "H_t", None))
        kw.update(over)
        return cls(**kw)


def params(**kw) -> _ParamsHolder:
    return _ParamsHolder(**kw)


def params_from(w, **over) -> _ParamsHolder:
    return _ParamsHolder.from_workload(w, **over)


def footprint(p: _ParamsHolder) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().quapi_footprint(ctypes.byref(p.p), ctypes.byref(out)))
    return int(out.value)


def paper_pmc_bytes(M: int, dk_max: int) -> int:
    return int(lib().quapi_paper_pmc_bytes(int(M), int(dk_max)))


def _sel_array(sel) -> tuple:
    """int32 copy of a selection and its length; an empty selection still gets
    a valid (one-element) buffer, so the library never sees NULL ('all steps')."""
    arr = np.ascontiguousarray(np.asarray(sel, dtype=np.int32).reshape(-1))
    n = len(arr)
    return (arr if n else np.zeros(1, dtype=np.int32)), n


class Context:
    """A quapi_ctx.  Use ``create`` to make one."""

    def __init__(self, handle: ctypes.c_void_p, M: int, L: int, keep=()):
        self._h = handle
        self.M = M
        self.N = M * M
        self.L = L
        self._keep = keep          # workspace owner (e.g. a torch tensor) stays alive

    @property
    def handle(self):
        return self._h

    def _live(self):
        if not self._h:
            raise QuapiError(ERR_STATE, "context destroyed")
        return self._h

    def propagate(self, n_steps: int, sel: Optional[Sequence[int]] = None) -> np.ndarray:
        """Blocking: rho at the selected steps, shape (n_out, M, M) complex128."""
        h = self._live()
        if sel is None:
            n_out, sel_arr, psel, n_sel = n_steps, None, None, 0
        else:
            sel_arr, n_sel = _sel_array(sel)
            n_out = n_sel
            psel = sel_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        out = np.zeros(2 * self.N * max(n_out, 1), dtype=np.float64)
        _check(lib().quapi_propagate(h, int(n_steps), psel, n_sel, _ptr(out)), h)
        return out.view(np.complex128)[: self.N * n_out].reshape(n_out, self.M, self.M)

    def propagate_async(self, n_steps: int, sel: Optional[Sequence[int]], rho_out_dev: int) -> None:
        """Enqueue on the context's stream; rho goes to device memory at rho_out_dev."""
        h = self._live()
        if sel is None:
            psel, n_sel = None, 0
        else:
            sel_arr, n_sel = _sel_array(sel)
            psel = sel_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        _check(lib().quapi_propagate_async(h, int(n_steps), psel, n_sel, ctypes.c_void_p(rho_out_dev)), h)

    def fused_steps(self) -> int:
        """Full-window steps per launch (3, 2 or 1): calls that end on a multiple
        of it past L give the same bits as one call."""
        v = ctypes.c_int(0)
        _check(lib().quapi_fused_steps(self._live(), ctypes.byref(v)))
        return int(v.value)

    def set_fused_steps(self, steps: int) -> None:
        """Pin the full-window steps per launch (1, 2, 3; 0 = default)."""
        h = self._live()
        _check(lib().quapi_set_fused_steps(h, int(steps)), h)

    def mirror(self) -> int:
        """Mirror mode (half of the tensor's entries read and written per
        pass): 0 off, 1 on where it pays (default), 2 on at every size."""
        v = ctypes.c_int(0)
        _check(lib().quapi_mirror(self._live(), ctypes.byref(v)))
        return int(v.value)

    def set_mirror(self, enable) -> None:
        """enable: 0 / False, 1 / True, or 2 (every size, e.g. in tests)."""
        h = self._live()
        _check(lib().quapi_set_mirror(h, int(enable)), h)

    def persistent(self) -> int:
        """0: multi-block kernels; 1: persistent path, tensor in LDS; 2: persistent, tensor in HBM."""
        v = ctypes.c_int(0)
        _check(lib().quapi_persistent(self._live(), ctypes.byref(v)))
        return int(v.value)

    def step_count(self) -> int:
        v = ctypes.c_int(0)
        _check(lib().quapi_step_count(self._live(), ctypes.byref(v)))
        return int(v.value)

    def get_setup(self, what: int) -> np.ndarray:
        n = {SETUP_G: 2 * self.L + 3, SETUP_ETA: 4 * self.L + 2, SETUP_U: self.M * self.M,
             SETUP_K: self.N * self.N}[what]
        out = np.zeros(2 * n, dtype=np.float64)
        h = self._live()
        _check(lib().quapi_get_setup(h, int(what), _ptr(out), out.size), h)
        return out.view(np.complex128).copy()

    def tensor_size(self) -> int:
        v = ctypes.c_size_t(0)
        _check(lib().quapi_tensor_size(self._live(), ctypes.byref(v)))
        return int(v.value)

    def read_tensor(self, first: int, count: int) -> np.ndarray:
        out = np.zeros(2 * max(count, 1), dtype=np.float64)
        h = self._live()
        _check(lib().quapi_read_tensor(h, int(first), int(count), _ptr(out)), h)
        return out.view(np.complex128)[:count].copy()

    def checkpoint(self) -> tuple:
        """(step, tensor): the state quapi_restore takes back."""
        return self.step_count(), self.read_tensor(0, self.tensor_size())

    def restore(self, step: int, tensor) -> None:
        t = np.ascontiguousarray(np.asarray(tensor, dtype=np.complex128).reshape(-1))
        buf = t.view(np.float64)
        h = self._live()
        _check(lib().quapi_restore(h, int(step), _ptr(buf), t.size), h)

    def filter_stats(self) -> tuple:
        """Filtered context: (entries kept after the last step, overflow flag)."""
        n = ctypes.c_longlong(0)
        ov = ctypes.c_int(0)
        h = self._live()
        _check(lib().quapi_filter_stats(h, ctypes.byref(n), ctypes.byref(ov)), h)
        return int(n.value), int(ov.value)

    def filter_read(self, first: int = 0, count: Optional[int] = None) -> tuple:
        """Filtered context: (keys int64, values complex128) of kept entries
        [first, first + count) in index order (count None: all from first)."""
        if count is None:
            count = self.filter_stats()[0] - first
        keys = np.zeros(max(count, 1), dtype=np.int64)
        vals = np.zeros(2 * max(count, 1), dtype=np.float64)
        h = self._live()
        _check(lib().quapi_filter_read(h, int(first), int(count),
                                       keys.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _ptr(vals)), h)
        return keys[:count].copy(), vals.view(np.complex128)[:count].copy()

    def set_timing(self, enable: bool = True) -> None:
        _check(lib().quapi_set_timing(self._live(), int(bool(enable))))

    def get_timing(self) -> dict:
        t = Timing()
        h = self._live()
        _check(lib().quapi_get_timing(h, ctypes.byref(t)), h)
        out = {}
        for k, _ in Timing._fields_:
            v = getattr(t, k)
            out[k] = list(v) if k.startswith("width_") else v
        return out

    def destroy(self) -> None:
        if self._h:
            _check(lib().quapi_destroy(self._h))
            self._h = None
            self._keep = ()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            if self._h:
                lib().quapi_destroy(self._h)
        except Exception:
            pass


def copy_bandwidth(src: int, dst: int, nbytes: int, chunk_bytes: int, nontemporal: bool,
                   stream: Optional[int] = None) -> None:
    """quapi_copy_bandwidth: enqueue one chunked device copy (a measurement aid)."""
    _check(lib().quapi_copy_bandwidth(ctypes.c_void_p(src), ctypes.c_void_p(dst), int(nbytes),
                                      int(chunk_bytes), int(bool(nontemporal)),
                                      ctypes.c_void_p(stream) if stream else None))


def propagate_static(p: _ParamsHolder, n_steps: int, sel: Optional[Sequence[int]], rho_out_dev: int,
                     stream: Optional[int] = None) -> None:
    """quapi_propagate_static: setup + n_steps steps in the library's static
    scratch (no device allocation); rho at the selected steps (None: every
    step 1..n_steps) goes to device memory at rho_out_dev."""
    if sel is None:
        psel, n_sel = None, 0
    else:
        sel_arr, n_sel = _sel_array(sel)
        psel = sel_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    _check(lib().quapi_propagate_static(ctypes.byref(p.p), int(n_steps), psel, n_sel,
                                        ctypes.c_void_p(rho_out_dev) if rho_out_dev else None,
                                        ctypes.c_void_p(stream) if stream else None))


def propagate_batch(ctxs: Sequence["Context"], n_steps: Sequence[int], rho_mode: Sequence[int],
                    rho_out_dev: Sequence[int]) -> None:
    """quapi_propagate_batch: advance persistent-path contexts (same M, dtype)
    together; rho_mode 0 none, 1 every step, 2 the last step; enqueued on the
    first context's stream."""
    n = len(ctxs)
    hs = (ctypes.c_void_p * max(n, 1))(*[c._live() for c in ctxs])
    ns = np.ascontiguousarray(np.asarray(list(n_steps) or [0], dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(list(rho_mode) or [0], dtype=np.int32))
    outs = (ctypes.c_void_p * max(n, 1))(*[ctypes.c_void_p(int(p)) if p else None for p in rho_out_dev])
    ip = ctypes.POINTER(ctypes.c_int)
    _check(lib().quapi_propagate_batch(hs, n, ns.ctypes.data_as(ip), ms.ctypes.data_as(ip), outs))


def create(p: _ParamsHolder, stream: Optional[int] = None, workspace: Optional[int] = None,
           ws_bytes: int = 0, keep=()) -> Context:
    """quapi_create.  stream: a hipStream_t as int (e.g. torch.cuda.current_stream().cuda_stream);
    workspace: device pointer of ws_bytes bytes (e.g. a torch tensor's data_ptr())."""
    h = ctypes.c_void_p(None)
    _check(lib().quapi_create(ctypes.byref(p.p), ctypes.c_void_p(stream) if stream else None,
                              ctypes.c_void_p(workspace) if workspace else None, int(ws_bytes),
                              ctypes.byref(h)))
    return Context(h, p.p.M, p.p.dk_max, keep=keep)


def filtered_footprint(p: _ParamsHolder, capacity: int) -> int:
    """Device bytes of a filtered context holding up to `capacity` kept entries."""
    v = ctypes.c_size_t(0)
    _check(lib().quapi_filtered_footprint(ctypes.byref(p.p), int(capacity), ctypes.byref(v)))
    return int(v.value)


def create_filtered(p: _ParamsHolder, theta: float, capacity: int, stream: Optional[int] = None) -> Context:
    """quapi_create_filtered: entries with |A| <= theta are dropped as they form;
    at most `capacity` kept entries."""
    h = ctypes.c_void_p(None)
    _check(lib().quapi_create_filtered(ctypes.byref(p.p), float(theta), int(capacity),
                                       ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
    return Context(h, p.p.M, p.p.dk_max)


def create_in_torch(p: _ParamsHolder, stream=None, device: str = "cuda:0") -> Context:
    """quapi_create with the workspace held by a torch uint8 tensor and a torch stream."""
    import torch
    nbytes = footprint(p)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    st = stream if stream is not None else torch.cuda.current_stream(device)
    return create(p, stream=st.cuda_stream, workspace=ws.data_ptr(), ws_bytes=nbytes, keep=(ws, st))
