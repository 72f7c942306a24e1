"""Thin ctypes binding of libbccb (include/bccb.h).

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are torch tensors (complex64, CUDA/HIP device); torch provides memory
and the current stream, nothing else.  Importing this module loads the library
and raises if it has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
import sys

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbccb.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "bccb.h")

BCCB_OK = 0
BCCB_E_INVALID = -1
BCCB_E_UNSUPPORTED = -2
BCCB_E_NOMEM = -3
BCCB_E_DEVICE = -4
BCCB_E_NONFINITE = -5
BCCB_E_SCRATCH = -6


class Config(ctypes.Structure):
    """bccb_config: launch shape of a plan's row and column passes."""
    _fields_ = [("row_elems", ctypes.c_int), ("row_rows_per_block", ctypes.c_int),
                ("col_elems", ctypes.c_int), ("col_cols_per_block", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("spectral_support", ctypes.c_int),
                ("row_spread", ctypes.c_int), ("col_spread", ctypes.c_int),
                ("sparse_iterate", ctypes.c_int), ("support_columns", ctypes.c_int),
                ("prow_elems", ctypes.c_int), ("prow_rows_per_block", ctypes.c_int),
                ("pcol_elems", ctypes.c_int), ("pcol_cols_per_block", ctypes.c_int),
                ("resident_groups", ctypes.c_int), ("resident_spread", ctypes.c_int),
                ("resident_block", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BCCBError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


class NonFiniteError(BCCBError):
    pass


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    return ctypes.CDLL(LIB_PATH)


lib = _load()

_vp = ctypes.c_void_p
_i = ctypes.c_int
_f = ctypes.c_float
_d = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int)

_SIGS = {
    "bccb_status_string": (ctypes.c_char_p, [_i]),
    "bccb_plan": (_i, [_vp, _i, _i, _i, _i, _vp, ctypes.POINTER(_vp)]),
    "bccb_plan_destroy": (_i, [_vp]),
    "bccb_plan_spaced": (_i, [_vp, _i, _i, _i, _i, _d, _d, _vp, ctypes.POINTER(_vp)]),
    "bccb_plan_embedding": (_i, [_vp, _pi, _pi, _vp]),
    "bccb_extract_peaks": (_i, [_vp, _vp, _i, _i, _f, _vp, _vp]),
    "bccb_adjoint_f64": (_i, [_vp, _vp, _vp]),
    "bccb_gram_apply_f64": (_i, [_vp, _vp, _vp]),
    "lasso_solve_ista_f64": (_i, [_vp, _vp, _d, _i, _vp, _vp]),
    "lasso_solve_fista_f64": (_i, [_vp, _vp, _d, _i, _vp, _vp]),
    "lasso_solve_admm_f64": (_i, [_vp, _vp, _d, _d, _i, _vp, _vp]),
    "bccb_set_stream": (_i, [_vp, _vp]),
    "bccb_plan_info": (_i, [_vp, _pi, _pd, _vp]),
    "bccb_adjoint": (_i, [_vp, _vp, _vp]),
    "bccb_adjoint_maxabs": (_i, [_vp, _vp, _pd]),
    "bccb_gram_apply": (_i, [_vp, _vp, _vp]),
    "lasso_solve_ista": (_i, [_vp, _vp, _f, _i, _vp, _vp]),
    "lasso_solve_fista": (_i, [_vp, _vp, _f, _i, _vp, _vp]),
    "lasso_solve_fista_noalloc": (_i, [_vp, _vp, _f, _i, _vp, _vp]),
    "lasso_solve_admm": (_i, [_vp, _vp, _f, _f, _i, _vp, _vp]),
    "bccb_objective_kkt": (_i, [_vp, _vp, _f, _vp, _pd, _pd, _pd]),
    "bccb_kkt": (_i, [_vp, _vp, _f, _vp, _pd, _pd]),
    "bccb_plan_omega_device": (_i, [_vp, _vp]),
    "bccb_profile_passes": (_i, [_vp, _i, _i, _pd, _pd]),
    "bccb_profile_resident": (_i, [_vp, _i, _i, _i, _pd]),
    "bccb_plan_get_config": (_i, [_vp, _vp]),
    "bccb_plan_set_config": (_i, [_vp, _vp]),
    "bccb_plan_autotune": (_i, [_vp, _i, _vp]),
    "bccb_batch_create": (_i, [_vp, _i, _vp, ctypes.POINTER(_vp)]),
    "bccb_batch_destroy": (_i, [_vp]),
    "bccb_batch_info": (_i, [_vp, _pi, _vp, _vp, _vp]),
    "lasso_solve_batch_fista": (_i, [_vp, _vp, _vp, _i, _vp]),
    "bccb_batch_autotune": (_i, [_vp, _i]),
    "lista_create": (_i, [_vp, _i, _i, _i, ctypes.POINTER(_vp)]),
    "lista_destroy": (_i, [_vp]),
    "lista_forward": (_i, [_vp, _vp, _vp, _vp, _i, _vp]),
    "lista_backward": (_i, [_vp, _vp, _vp, _vp, _pd]),
    "lista_adam": (_i, [_vp, _vp, _vp, _vp, _i, _i, _f, _f, _f, _f, _vp, _vp]),
    "lista_solve": (_i, [_vp, _vp, _vp, _vp, _i, _d, _i, _i, _i, _vp, _vp, _vp]),
    "bccb_dense_create": (_i, [_vp, _i, _f, ctypes.POINTER(_vp)]),
    "bccb_dense_destroy": (_i, [_vp]),
    "bccb_dense_apply": (_i, [_vp, _vp, _vp]),
    "lasso_solve_dense": (_i, [_vp, _i, _vp, _f, _i, _vp]),
    "bccb_plan_support_columns": (_i, [_vp, _pi, _pi]),
    "bccb_batch_set_sparse_iterate": (_i, [_vp, _i]),
    "bccb_batch_set_support_columns": (_i, [_vp, _i]),
    "bccb_batch_set_resident": (_i, [_vp, _i]),
    "bccb_batch_resident_info": (_i, [_vp, _pi, _pi, _pi, _pi]),
    "bccb_batch_class_config": (_i, [_vp, _i, _pi]),
    "lista_autotune": (_i, [_vp, _i]),
    "lista_set_resident": (_i, [_vp, _i]),
    "bccb_stream_copy": (_i, [_vp, _vp, ctypes.c_size_t, _i, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def declared_functions() -> list[str]:
    """Names of the functions declared in include/bccb.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)))


def status_string(code: int) -> str:
    return lib.bccb_status_string(code).decode()


def check(code: int, where: str) -> int:
    if code == BCCB_E_NONFINITE:
        raise NonFiniteError(code, where, status_string(code))
    if code < 0:
        raise BCCBError(code, where, status_string(code))
    return code


def _ptr(t, numel: int | None = None, what: str = "tensor") -> int | None:
    """Device address of a contiguous complex64 GPU tensor of exactly `numel` elements.

    Every size is checked here, before the library is called: an undersized output would
    make the kernels write past its allocation."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if t.dtype != torch.complex64:
        raise TypeError(f"{what}: expected complex64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor must live on the GPU")
    return t.data_ptr()


def _ptrs(*specs) -> list:
    """Addresses of several arguments, each (tensor or None, numel, name): every type and
    size is checked before any device check, so a wrong size is always reported as one."""
    for t, n, what in specs:
        _check_host_side(t, n, what, torch.complex64)
    return [_ptr(t, n, what) for t, n, what in specs]


def _check_host_side(t, numel, what, dtype):
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")


def _raw_ptr(t) -> int:
    """Device address of a contiguous GPU tensor of any dtype."""
    if not isinstance(t, torch.Tensor) or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return t.data_ptr()


def _release(obj, _finalizing=sys.is_finalizing) -> None:
    """Finalizer of the handle classes: frees the library object, except while the interpreter
    is shutting down -- then the HIP runtime, torch's streams and the library may already be
    torn down in any order, so nothing is called into and the process exit reclaims the device
    memory.  Explicit close() calls are unaffected.  (Bound as a default argument of every
    __del__, since module globals may already be cleared when a finalizer runs at shutdown.)"""
    if _finalizing():
        return
    try:
        obj.close()
    except Exception:
        pass


def current_stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """A per-geometry plan: mask (uint8 [M2][M1]) and grid size L1 x L2."""

    def __init__(self, mask, L1: int, L2: int, stream: int | None = None):
        mask = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
        if mask.ndim != 2:
            raise ValueError("mask must be 2-D [M2][M1]")
        self.mask = mask
        self.M2, self.M1 = mask.shape
        self.L1, self.L2 = int(L1), int(L2)
        self.L = self.L1 * self.L2
        self._h = _vp()
        s = current_stream() if stream is None else stream
        self._create(mask, s)
        M = ctypes.c_int()
        mu = ctypes.c_double()
        check(lib.bccb_plan_info(self._h, ctypes.byref(M), ctypes.byref(mu), None), "bccb_plan_info")
        self.M = M.value
        self.mu = mu.value

    def _create(self, mask, s):
        check(lib.bccb_plan(mask.ctypes.data, self.M1, self.M2, self.L1, self.L2, s, ctypes.byref(self._h)),
              "bccb_plan")

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib.bccb_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self, _release=_release):
        _release(self)

    def _args(self, y, **grids):
        """Addresses of a snapshot (complex64 [M]) and of coefficient grids (complex64
        [L2][L1], None passes through), all sizes checked first."""
        if y is None:
            raise ValueError("y: a snapshot is required")
        return _ptrs((y, self.M, "y"), *[(t, self.L, k) for k, t in grids.items()])

    def set_stream(self, stream: int):
        check(lib.bccb_set_stream(self._h, stream), "bccb_set_stream")

    def omega(self) -> np.ndarray:
        out = np.empty((self.L2, self.L1), dtype=np.float32)
        check(lib.bccb_plan_info(self._h, None, None, out.ctypes.data), "bccb_plan_info")
        return out

    def grid(self, device="cuda") -> torch.Tensor:
        return torch.empty((self.L2, self.L1), dtype=torch.complex64, device=device)

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.grid(y.device) if out is None else out
        py, po = self._args(y, out=out)
        check(lib.bccb_adjoint(self._h, py, po), "bccb_adjoint")
        return out

    def adjoint_maxabs(self, y: torch.Tensor) -> float:
        m = ctypes.c_double()
        (py,) = self._args(y)
        check(lib.bccb_adjoint_maxabs(self._h, py, ctypes.byref(m)), "bccb_adjoint_maxabs")
        return m.value

    def gram_apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.grid(x.device) if out is None else out
        px, po = _ptrs((x, self.L, "x"), (out, self.L, "out"))
        check(lib.bccb_gram_apply(self._h, px, po), "bccb_gram_apply")
        return out

    def ista(self, y, tau: float, iters: int, c0=None, out=None) -> torch.Tensor:
        out = self.grid(y.device) if out is None else out
        py, pc, po = self._args(y, c0=c0, out=out)
        check(lib.lasso_solve_ista(self._h, py, float(tau), int(iters), pc, po),
              "lasso_solve_ista")
        return out

    def fista(self, y, tau: float, iters: int, c0=None, out=None) -> torch.Tensor:
        out = self.grid(y.device) if out is None else out
        py, pc, po = self._args(y, c0=c0, out=out)
        check(lib.lasso_solve_fista(self._h, py, float(tau), int(iters), pc, po),
              "lasso_solve_fista")
        return out

    # --- FP64 variants (complex128 device tensors) ---
    def _args64(self, y, **grids):
        for t, n, what in [(y, self.M, "y")] + [(t, self.L, k) for k, t in grids.items()]:
            _check_host_side(t, n, what, torch.complex128)
        return [_raw_ptr(y)] + [None if t is None else _raw_ptr(t) for t in grids.values()]

    def grid64(self, device="cuda") -> torch.Tensor:
        return torch.empty((self.L2, self.L1), dtype=torch.complex128, device=device)

    def adjoint_f64(self, y, out=None):
        out = self.grid64(y.device) if out is None else out
        py, po = self._args64(y, out=out)
        check(lib.bccb_adjoint_f64(self._h, py, po), "bccb_adjoint_f64")
        return out

    def gram_apply_f64(self, x, out=None):
        out = self.grid64(x.device) if out is None else out
        _check_host_side(x, self.L, "x", torch.complex128)
        _check_host_side(out, self.L, "out", torch.complex128)
        check(lib.bccb_gram_apply_f64(self._h, _raw_ptr(x), _raw_ptr(out)), "bccb_gram_apply_f64")
        return out

    def ista_f64(self, y, tau: float, iters: int, c0=None, out=None):
        out = self.grid64(y.device) if out is None else out
        py, pc, po = self._args64(y, c0=c0, out=out)
        check(lib.lasso_solve_ista_f64(self._h, py, float(tau), int(iters), pc, po), "lasso_solve_ista_f64")
        return out

    def fista_f64(self, y, tau: float, iters: int, c0=None, out=None):
        out = self.grid64(y.device) if out is None else out
        py, pc, po = self._args64(y, c0=c0, out=out)
        check(lib.lasso_solve_fista_f64(self._h, py, float(tau), int(iters), pc, po), "lasso_solve_fista_f64")
        return out

    def admm_f64(self, y, tau: float, rho: float, iters: int, want_c=False):
        z = self.grid64(y.device)
        c = self.grid64(y.device) if want_c else None
        py, pz, pc = self._args64(y, z=z, c=c)
        check(lib.lasso_solve_admm_f64(self._h, py, float(tau), float(rho), int(iters), pz, pc),
              "lasso_solve_admm_f64")
        return (z, c) if want_c else z

    def extract_peaks(self, c, max_peaks: int, min_mag2: float = 0.0):
        return extract_peaks(self, c, max_peaks, min_mag2)

    def fista_noalloc(self, y, tau: float, iters: int, c0=None, out=None) -> torch.Tensor:
        """lasso_solve_fista_noalloc: FISTA with the library's static work array (no device
        allocation inside the call; `out` is allocated here when not given)."""
        out = self.grid(y.device) if out is None else out
        py, pc, po = self._args(y, c0=c0, out=out)
        check(lib.lasso_solve_fista_noalloc(self._h, py, float(tau), int(iters), pc, po),
              "lasso_solve_fista_noalloc")
        return out

    def admm(self, y, tau: float, rho: float, iters: int, z_out=None, c_out=None, want_c=False):
        z_out = self.grid(y.device) if z_out is None else z_out
        if want_c and c_out is None:
            c_out = self.grid(y.device)
        py, pz, pc = self._args(y, z_out=z_out, c_out=c_out)
        check(lib.lasso_solve_admm(self._h, py, float(tau), float(rho), int(iters), pz, pc), "lasso_solve_admm")
        return (z_out, c_out) if want_c else z_out

    def objective_kkt(self, y, tau: float, c) -> tuple[float, float, float]:
        obj, r, mx = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        py, pc = self._args(y, c=c)
        check(lib.bccb_objective_kkt(self._h, py, float(tau), pc, ctypes.byref(obj), ctypes.byref(r),
                                     ctypes.byref(mx)), "bccb_objective_kkt")
        return obj.value, r.value, mx.value


    def kkt(self, y, tau: float, c) -> tuple[float, float]:
        """(r_kkt, objective) of c through bccb_kkt."""
        r, obj = ctypes.c_double(), ctypes.c_double()
        py, pc = self._args(y, c=c)
        check(lib.bccb_kkt(self._h, py, float(tau), pc, ctypes.byref(r), ctypes.byref(obj)), "bccb_kkt")
        return r.value, obj.value

    def omega_device(self, out=None) -> torch.Tensor:
        """The FP32 eigenvalue grid Omega [L2][L1] copied into a device tensor."""
        out = torch.empty((self.L2, self.L1), dtype=torch.float32, device="cuda") if out is None else out
        check(lib.bccb_plan_omega_device(self._h, _fptr(out, self.L, "out")), "bccb_plan_omega_device")
        return out

    def get_config(self) -> dict:
        c = Config()
        check(lib.bccb_plan_get_config(self._h, ctypes.byref(c)), "bccb_plan_get_config")
        return c.as_dict()

    def set_config(self, **kw) -> dict:
        cur = self.get_config()
        cur.update(kw)
        c = Config(**cur)
        check(lib.bccb_plan_set_config(self._h, ctypes.byref(c)), "bccb_plan_set_config")
        return self.get_config()

    def support_columns(self) -> tuple[int, int]:
        """(spectral columns holding support bins, how ISTA/FISTA use them: 0 = full passes or
        the full cooperative form, 1 = the pruned passes, 2 = the pruned cooperative form)."""
        n, pr = ctypes.c_int(), ctypes.c_int()
        check(lib.bccb_plan_support_columns(self._h, ctypes.byref(n), ctypes.byref(pr)), "bccb_plan_support_columns")
        return n.value, pr.value

    def autotune(self, reps: int = 50) -> dict:
        c = Config()
        check(lib.bccb_plan_autotune(self._h, int(reps), ctypes.byref(c)), "bccb_plan_autotune")
        return c.as_dict()

    def profile_passes(self, solver: str, reps: int = 200) -> tuple[float, float]:
        """Average ms per launch of (column pass, row pass) of one iteration of `solver`."""
        code = {"ista": 0, "fista": 1, "admm": 2}[solver]
        col, row = ctypes.c_double(), ctypes.c_double()
        check(lib.bccb_profile_passes(self._h, code, int(reps), ctypes.byref(col), ctypes.byref(row)),
              "bccb_profile_passes")
        return col.value, row.value

    def profile_resident(self, solver: str, iters: int, reps: int = 20) -> float:
        """Average ms per cooperative solve of `iters` iterations (plans whose solves take it)."""
        code = {"ista": 0, "fista": 1, "admm": 2}[solver]
        ms = ctypes.c_double()
        check(lib.bccb_profile_resident(self._h, code, int(iters), int(reps), ctypes.byref(ms)),
              "bccb_profile_resident")
        return ms.value


def stream_copy(src: torch.Tensor, dst: torch.Tensor, variant: int = 0, stream: int | None = None):
    """Device-to-device copy through the library's streaming kernel (bandwidth ceiling)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("destination smaller than source")
    s = current_stream() if stream is None else stream
    check(lib.bccb_stream_copy(_vp(_raw_ptr(src)), _vp(_raw_ptr(dst)), ctypes.c_size_t(nbytes), int(variant), s),
          "bccb_stream_copy")


# bccb_peak (include/bccb.h), 32 bytes
PEAK_DTYPE = np.dtype([("index", np.int32), ("mag2", np.float32), ("f1", np.float32), ("f2", np.float32),
                       ("phi", np.float32), ("theta", np.float32), ("amp_re", np.float32), ("amp_im", np.float32)])


def extract_peaks_device(plan: "Plan", c: torch.Tensor, max_peaks: int, min_mag2: float = 0.0, peaks=None,
                         counts=None):
    """bccb_extract_peaks into device buffers: (peaks, counts), peaks a uint8 tensor of
    batch * max_peaks bccb_peak records (PEAK_DTYPE), counts int32 [batch] (-1: more than 4096
    local maxima above min_mag2).  c: [L2][L1] or [batch][L2][L1] complex64 on the GPU."""
    batch = 1 if c.dim() == 2 else int(c.shape[0])
    (pc,) = _ptrs((c, batch * plan.L, "c"))
    nbytes = batch * int(max_peaks) * PEAK_DTYPE.itemsize
    if peaks is None:
        peaks = torch.empty(nbytes, dtype=torch.uint8, device=c.device)
    if counts is None:
        counts = torch.empty(batch, dtype=torch.int32, device=c.device)
    if peaks.dtype != torch.uint8 or peaks.numel() != nbytes or counts.dtype != torch.int32 or counts.numel() != batch:
        raise ValueError("peaks: uint8 [batch * max_peaks * 32], counts: int32 [batch]")
    check(lib.bccb_extract_peaks(plan.handle, pc, batch, int(max_peaks), float(min_mag2), _raw_ptr(peaks),
                                 _raw_ptr(counts)), "bccb_extract_peaks")
    return peaks, counts


def extract_peaks(plan: "Plan", c: torch.Tensor, max_peaks: int, min_mag2: float = 0.0):
    """bccb_extract_peaks over c ([L2][L1] or [batch][L2][L1], complex64 on the GPU, the plan's
    grid): a list per grid of PEAK_DTYPE records, strongest first (None for a grid with more
    than 4096 local maxima above min_mag2)."""
    batch = 1 if c.dim() == 2 else int(c.shape[0])
    peaks, counts = extract_peaks_device(plan, c, max_peaks, min_mag2)
    rec = peaks.cpu().numpy().view(PEAK_DTYPE).reshape(batch, int(max_peaks))
    n = counts.cpu().numpy()
    return [None if n[i] < 0 else rec[i, :n[i]].copy() for i in range(batch)]


class SpacedPlan(Plan):
    """bccb_plan_spaced: element spacing (gamma1, gamma2) wavelengths and any grid lengths
    L1, L2 in [2, 512] (the Gram is block Toeplitz; products through a padded embedding)."""

    def __init__(self, mask, L1: int, L2: int, gamma1: float = 0.5, gamma2: float = 0.5,
                 stream: int | None = None):
        self.gamma1, self.gamma2 = float(gamma1), float(gamma2)
        super().__init__(mask, L1, L2, stream)

    def _create(self, mask, s):
        check(lib.bccb_plan_spaced(mask.ctypes.data, self.M1, self.M2, self.L1, self.L2, self.gamma1,
                                   self.gamma2, s, ctypes.byref(self._h)), "bccb_plan_spaced")

    def embedding(self):
        """(P1, P2, Omega_e [P2][P1] float32) of the padded embedding, or None for a plan that
        needs none (gamma = 1/2 on power-of-two grids)."""
        P1, P2 = ctypes.c_int(), ctypes.c_int()
        rc = lib.bccb_plan_embedding(self._h, ctypes.byref(P1), ctypes.byref(P2), None)
        if rc == BCCB_E_UNSUPPORTED:
            return None
        check(rc, "bccb_plan_embedding")
        om = np.empty((P2.value, P1.value), dtype=np.float32)
        check(lib.bccb_plan_embedding(self._h, None, None, om.ctypes.data), "bccb_plan_embedding")
        return P1.value, P2.value, om


def to_device(y: np.ndarray, device="cuda") -> torch.Tensor:
    """complex64 numpy array -> contiguous complex64 device tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(y, dtype=np.complex64))).to(device)


class Batch:
    """Many independent scenes (each with its own Plan) solved together."""

    def __init__(self, plans, stream: int | None = None):
        self.plans = list(plans)
        n = len(self.plans)
        arr = (_vp * n)(*[p.handle for p in self.plans])
        self._h = _vp()
        s = current_stream() if stream is None else stream
        check(lib.bccb_batch_create(arr, n, s, ctypes.byref(self._h)), "bccb_batch_create")
        self.n = n

    def close(self):
        if self._h:
            lib.bccb_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self, _release=_release):
        _release(self)

    def classes(self):
        nc = ctypes.c_int()
        check(lib.bccb_batch_info(self._h, ctypes.byref(nc), None, None, None), "bccb_batch_info")
        L1 = (ctypes.c_int * nc.value)()
        L2 = (ctypes.c_int * nc.value)()
        cnt = (ctypes.c_int * nc.value)()
        check(lib.bccb_batch_info(self._h, ctypes.byref(nc), L1, L2, cnt), "bccb_batch_info")
        return [(L1[i], L2[i], cnt[i]) for i in range(nc.value)]

    def autotune(self, reps: int = 10):
        check(lib.bccb_batch_autotune(self._h, int(reps)), "bccb_batch_autotune")

    def class_configs(self):
        """Per size class: (row E, rows/block, column E, columns/block, pruned, columns transformed)."""
        out = []
        for i in range(len(self.classes())):
            cfg = (ctypes.c_int * 6)()
            check(lib.bccb_batch_class_config(self._h, i, cfg), "bccb_batch_class_config")
            out.append(tuple(cfg))
        return out

    def set_support_columns(self, on: bool):
        check(lib.bccb_batch_set_support_columns(self._h, 1 if on else 0), "bccb_batch_set_support_columns")

    def set_sparse_iterate(self, on: bool):
        check(lib.bccb_batch_set_sparse_iterate(self._h, 1 if on else 0), "bccb_batch_set_sparse_iterate")

    def set_resident(self, on):
        """False / True, or a workgroup size (256, 512, 1024) for the persistent launch."""
        v = int(on) if not isinstance(on, bool) else (1 if on else 0)
        check(lib.bccb_batch_set_resident(self._h, v), "bccb_batch_set_resident")

    def resident_info(self):
        """{"on": 1 | 0 | -1 (unsupported), "threads", "blocks", "lds_bytes"} of the persistent launch."""
        v = [ctypes.c_int() for _ in range(4)]
        check(lib.bccb_batch_resident_info(self._h, *[ctypes.byref(x) for x in v]), "bccb_batch_resident_info")
        return dict(zip(("on", "threads", "blocks", "lds_bytes"), (x.value for x in v)))

    def fista(self, ys, taus, iters: int, outs=None):
        n = self.n
        if outs is None:
            outs = [p.grid(ys[i].device) for i, p in enumerate(self.plans)]
        if len(ys) != n or len(outs) != n or len(taus) != n:
            raise ValueError(f"expected {n} snapshots, outputs and weights, got {len(ys)}, {len(outs)}, {len(taus)}")
        ptrs = _ptrs(*[(t, p.M, f"ys[{i}]") for i, (t, p) in enumerate(zip(ys, self.plans))],
                     *[(t, p.L, f"outs[{i}]") for i, (t, p) in enumerate(zip(outs, self.plans))])
        ya = (_vp * n)(*ptrs[:n])
        oa = (_vp * n)(*ptrs[n:])
        ta = (ctypes.c_float * n)(*[float(t) for t in taus])
        check(lib.lasso_solve_batch_fista(self._h, ya, ta, int(iters), oa), "lasso_solve_batch_fista")
        return outs


LISTA_PER_LAYER = 52


def _fptr(t, numel: int | None = None, what: str = "tensor"):
    """Device address of a contiguous float32 GPU tensor of exactly `numel` elements."""
    if t is None:
        return None
    _check_host_side(t, numel, what, torch.float32)
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor must live on the GPU")
    return t.data_ptr()


def lista_init_params(layers: int, device="cuda") -> torch.Tensor:
    """s = theta = 1, Delta = 0: every layer one plain FISTA iteration."""
    p = torch.zeros((layers, LISTA_PER_LAYER), dtype=torch.float32)
    p[:, 0] = 1.0
    p[:, 1] = 1.0
    return p.to(device)


class Lista:
    """Learned unrolled FISTA on one plan's geometry (device workspace for max_batch scenes)."""

    def __init__(self, plan: Plan, layers: int = 16, max_batch: int = 256, train: bool = False):
        self.plan = plan
        self.layers = layers
        self.max_batch = max_batch
        self._h = _vp()
        self._batch = 0       # batch of the last forward (what lista_backward differentiates)
        check(lib.lista_create(plan.handle, layers, max_batch, 1 if train else 0, ctypes.byref(self._h)),
              "lista_create")

    def close(self):
        if self._h:
            lib.lista_destroy(self._h)
            self._h = _vp()

    def __del__(self, _release=_release):
        _release(self)

    @staticmethod
    def _taus(tau, B):
        arr = np.ascontiguousarray(np.asarray(tau, dtype=np.float32).reshape(-1))
        if arr.size != B:
            raise ValueError(f"taus: expected {B} weights, got {arr.size}")
        return arr, arr.ctypes.data

    def _batch_of(self, ys):
        if not isinstance(ys, torch.Tensor) or ys.dim() != 2 or ys.shape[1] != self.plan.M:
            raise ValueError(f"ys: expected complex64 [batch][{self.plan.M}]")
        B = int(ys.shape[0])
        if not 1 <= B <= self.max_batch:
            raise ValueError(f"ys: expected a batch of 1..{self.max_batch} scenes, got {B}")
        return B

    def _host_checks(self, params, grad=None, **grids):
        """Every size of a learned call, checked before any device check."""
        n = self.layers * LISTA_PER_LAYER
        _check_host_side(params, n, "params", torch.float32)
        _check_host_side(grad, n, "grad", torch.float32)
        for k, (t, numel) in grids.items():
            _check_host_side(t, numel, k, torch.complex64)

    def _params(self, params, what="params"):
        return _fptr(params, self.layers * LISTA_PER_LAYER, what)

    def forward(self, params, ys, taus, out=None):
        """ys: complex64 [batch][M] device; taus: host floats [batch]."""
        B = self._batch_of(ys)
        if out is None:
            out = torch.empty((B, self.plan.L2, self.plan.L1), dtype=torch.complex64, device=ys.device)
        arr, tp = self._taus(taus, B)
        self._host_checks(params, ys=(ys, B * self.plan.M), out=(out, B * self.plan.L))
        check(lib.lista_forward(self._h, self._params(params), _ptr(ys, B * self.plan.M, "ys"), tp, B,
                                _ptr(out, B * self.plan.L, "out")), "lista_forward")
        self._batch = B
        return out

    def backward(self, params, labels, grad=None):
        if grad is None:
            grad = torch.zeros_like(params)
        if self._batch < 1:
            raise ValueError("backward needs a training-mode forward first")
        loss = ctypes.c_double()
        self._host_checks(params, grad=grad, labels=(labels, self._batch * self.plan.L))
        check(lib.lista_backward(self._h, self._params(params), _ptr(labels, self._batch * self.plan.L, "labels"),
                                 self._params(grad, "grad"), ctypes.byref(loss)), "lista_backward")
        return grad, loss.value

    def autotune(self, reps: int = 5):
        """Tune the fallback FISTA's pruned pass shapes (where the plan has kept columns)."""
        check(lib.lista_autotune(self._h, int(reps)), "lista_autotune")

    def set_resident(self, on: bool):
        """Run the fallback's check intervals as persistent launches (the default) or as passes."""
        check(lib.lista_set_resident(self._h, 1 if on else 0), "lista_set_resident")

    def solve(self, params, ys, taus, kkt_target=1e-4, check_every=10, max_iters=20000, out=None, restart=False):
        """KKT-gated solve (params=None: plain FISTA from zero); restart=True restarts the
        fallback momentum instead of continuing the unrolled FISTA.  Returns (c, iters, rkkt, status)."""
        B = self._batch_of(ys)
        if out is None:
            out = torch.empty((B, self.plan.L2, self.plan.L1), dtype=torch.complex64, device=ys.device)
        arr, tp = self._taus(taus, B)
        iters = np.zeros(B, dtype=np.int32)
        rk = np.zeros(B, dtype=np.float64)
        self._host_checks(params, ys=(ys, B * self.plan.M), out=(out, B * self.plan.L))
        rc = check(lib.lista_solve(self._h, self._params(params) if params is not None else None,
                                   _ptr(ys, B * self.plan.M, "ys"), tp, B,
                                   float(kkt_target), int(check_every), int(max_iters), 1 if restart else 0,
                                   _ptr(out, B * self.plan.L, "out"),
                                   iters.ctypes.data, rk.ctypes.data), "lista_solve")
        return out, iters, rk, rc


def lista_lr_scale(layers: int, delta_scale: float = 0.02, device="cuda") -> torch.Tensor:
    """Per-parameter learning-rate multipliers: 1 for s_k and theta_k, delta_scale for the taps."""
    sc = torch.full((layers, LISTA_PER_LAYER), float(delta_scale), dtype=torch.float32)
    sc[:, :2] = 1.0
    return sc.to(device)


class Adam:
    """Adam state for a float32 device parameter tensor; the update runs in the HIP library."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, lr_scale=None):
        self.p = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.lr, self.b1, self.b2, self.eps = lr, betas[0], betas[1], eps
        self.lr_scale = lr_scale
        self.t = 0

    def step(self, grad):
        self.t += 1
        n = self.p.numel()
        for t, what in ((grad, "grad"), (self.m, "m"), (self.v, "v"), (self.lr_scale, "lr_scale")):
            _check_host_side(t, n, what, torch.float32)
        check(lib.lista_adam(_fptr(self.p, n, "params"), _fptr(grad, n, "grad"), _fptr(self.m, n), _fptr(self.v, n),
                             n, self.t, self.lr, self.b1, self.b2, self.eps, _fptr(self.lr_scale, n, "lr_scale"),
                             current_stream()),
              "lista_adam")


class Dense:
    """The explicit L x L iteration matrix (kind 0: I - mu G; kind 1: (G + rho I)^-1)."""

    def __init__(self, plan: Plan, kind: int = 0, rho: float = 1.0):
        self.plan = plan
        self.kind = kind
        self._h = _vp()
        check(lib.bccb_dense_create(plan.handle, int(kind), float(rho), ctypes.byref(self._h)), "bccb_dense_create")

    def close(self):
        if self._h:
            lib.bccb_dense_destroy(self._h)
            self._h = _vp()

    def __del__(self, _release=_release):
        _release(self)

    def apply(self, x, out=None):
        out = self.plan.grid(x.device) if out is None else out
        px, po = _ptrs((x, self.plan.L, "x"), (out, self.plan.L, "out"))
        check(lib.bccb_dense_apply(self._h, px, po), "bccb_dense_apply")
        return out

    def solve(self, solver: str, y, tau: float, iters: int, out=None):
        code = {"ista": 0, "fista": 1, "admm": 2}[solver]
        out = self.plan.grid(y.device) if out is None else out
        py, po = self.plan._args(y, out=out)
        check(lib.lasso_solve_dense(self._h, code, py, float(tau), int(iters), po), "lasso_solve_dense")
        return out
