"""Python binding of libqpe (ctypes). Argument marshalling only.

Every step of the QPE path runs in the HIP kernels behind the C ABI declared
in include/qpe.h; this module only checks tensor shapes and dtypes, sizes and
allocates outputs and workspaces with torch on the tensors' device, and
passes raw device pointers plus torch's current HIP stream. There is no CPU
fallback: if libqpe.so is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqpe.so")

FORM_FP64 = 0
FORM_MIXED = 1
FORMS = {"fp64": FORM_FP64, "mixed": FORM_MIXED}
NO_POLAR = 1
PREFIX_DOUBLING = 2
MIX_TARGET = 4
NO_MIX_TARGET = 8
SPLIT_BF16 = 16
REPORT_NOT_UNITARY = 1
REPORT_NUMERIC = 2
REPORT_CONCENTRATED = 4

STATUS_NAMES = {
    0: "QPE_OK", 1: "QPE_ERR_ARG", 2: "QPE_ERR_SIZE", 3: "QPE_ERR_ALIGN", 4: "QPE_ERR_WORKSPACE",
    5: "QPE_ERR_OOM", 6: "QPE_ERR_NO_DEVICE", 7: "QPE_ERR_HIP", 8: "QPE_ERR_UNSUPPORTED",
}

# Every symbol include/qpe.h declares.
EXPORTS = (
    "qpe_ctx_create", "qpe_ctx_set_stream", "qpe_ctx_destroy", "qpe_workspace_size", "qpe_run",
    "qpe_powers_workspace_size", "qpe_powers", "qpe_controlled_step_workspace_size",
    "qpe_controlled_step", "qpe_iqft_workspace_size", "qpe_iqft_probs", "qpe_zgemm",
    "qpe_status_string", "qpe_last_error", "qpe_version", "qpe_check_run",
    "qpe_ctx_enable_timing", "qpe_ctx_set_timing_mask", "qpe_ctx_reset_timing", "qpe_ctx_read_timing",
    "qpe_kernel_variants", "qpe_ctx_set_variant", "qpe_estimate_workspace_size", "qpe_estimate",
    "qpe_run_state", "qpe_ctx_get_variant", "qpe_autotune", "qpe_autotune_batch", "qpe_run_static",
)

# Size of the static device workspace of qpe_run_static (QPE_STATIC_WORKSPACE_BYTES).
STATIC_WORKSPACE_BYTES = 64 << 20

KERNEL_CLASSES = {"ctrl_mixed": 0, "zgemm": 1, "ctrl_f64": 2, "batch_ctrl": 3, "batch_gemm": 4, "batch_sched": 5}
TUNE_MAX_VARIANTS = 12

TIMERS = {"ctrl_gemm": 0, "powers": 1, "split": 2, "qft": 3, "prob": 4, "hlayer": 5}


class QpeError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {STATUS_NAMES.get(status, status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


class Problem(ctypes.Structure):
    _fields_ = [("n_meas", ctypes.c_int32), ("n_mat", ctypes.c_int32), ("U", ctypes.c_void_p),
                ("psi", ctypes.c_void_p), ("prob", ctypes.c_void_p)]


REPORT_DTYPE = np.dtype([("unitarity_defect", "<f8"), ("prob_sum", "<f8"), ("psi_norm2", "<f8"),
                         ("input_peak", "<f8"), ("flags", "<u4"), ("reserved", "<u4")])
REPORT_BYTES = 40

ESTIMATES_DTYPE = np.dtype([("argmax_phase", "<f8"), ("weighted_phase", "<f8"), ("circular_phase", "<f8"),
                            ("prob_sum", "<f8"), ("argmax_index", "<i8"), ("reserved", "<i8")])
ESTIMATES_BYTES = 48

_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqpe.so and declare its signatures. Raises if it is missing."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(
                f"libqpe.so not found at {path}: build it with `python -m paper_2507_17175_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(path)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        st = ctypes.c_int
        sig = {
            "qpe_ctx_create": (st, [ctypes.POINTER(vp), i32, vp]),
            "qpe_ctx_set_stream": (st, [vp, vp]),
            "qpe_ctx_destroy": (st, [vp]),
            "qpe_workspace_size": (st, [ctypes.POINTER(Problem), i32, i32, ctypes.c_uint, ctypes.POINTER(sz)]),
            "qpe_run": (st, [vp, ctypes.POINTER(Problem), i32, i32, ctypes.c_uint, vp, sz, vp]),
            "qpe_run_static": (st, [vp, ctypes.POINTER(Problem), i32, i32, ctypes.c_uint, vp]),
            "qpe_powers_workspace_size": (st, [i32, ctypes.POINTER(sz)]),
            "qpe_powers": (st, [vp, i32, vp, i32, ctypes.c_uint, vp, vp, sz, vp]),
            "qpe_controlled_step_workspace_size": (st, [i32, i32, i32, ctypes.POINTER(sz)]),
            "qpe_controlled_step": (st, [vp, i32, i32, i32, i32, vp, vp, vp, sz]),
            "qpe_iqft_workspace_size": (st, [i32, i32, i32, ctypes.POINTER(sz)]),
            "qpe_iqft_probs": (st, [vp, i32, i32, i32, vp, vp, vp, sz]),
            "qpe_zgemm": (st, [vp, ctypes.c_char, ctypes.c_char, i32, i32, i32, ctypes.POINTER(ctypes.c_double),
                               vp, i32, vp, i32, ctypes.POINTER(ctypes.c_double), vp, i32, vp, i32]),
            "qpe_check_run": (st, [ctypes.POINTER(Problem), i32, i32, ctypes.c_uint, vp, sz, vp]),
            "qpe_ctx_enable_timing": (st, [vp, i32]),
            "qpe_ctx_set_timing_mask": (st, [vp, ctypes.c_uint]),
            "qpe_ctx_reset_timing": (st, [vp]),
            "qpe_kernel_variants": (st, [i32, ctypes.POINTER(i32)]),
            "qpe_ctx_set_variant": (st, [vp, i32, i32, i32]),
            "qpe_ctx_read_timing": (st, [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
            "qpe_run_state": (st, [vp, ctypes.POINTER(Problem), i32, ctypes.c_uint, vp, sz, vp, vp]),
            "qpe_ctx_get_variant": (st, [vp, i32, i32, ctypes.POINTER(i32)]),
            "qpe_autotune": (st, [vp, ctypes.POINTER(Problem), i32, ctypes.c_uint, vp, sz, i32,
                                  ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
            "qpe_autotune_batch": (st, [vp, ctypes.POINTER(Problem), i32, i32, ctypes.c_uint, vp, sz, i32,
                                        ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
            "qpe_estimate_workspace_size": (st, [i32, ctypes.POINTER(sz)]),
            "qpe_estimate": (st, [vp, ctypes.POINTER(Problem), i32, vp, vp, sz]),
            "qpe_status_string": (ctypes.c_char_p, [i32]),
            "qpe_last_error": (ctypes.c_char_p, [vp]),
            "qpe_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return L


def _check(status: int, where: str, ctx: Optional[int] = None) -> None:
    if status != 0:
        detail = ""
        if ctx:
            detail = (load_library().qpe_last_error(ctx) or b"").decode()
        raise QpeError(status, where, detail)


class Context:
    """A libqpe context bound to one device and (re-bound per call) to torch's
    current stream on that device."""

    def __init__(self, device: int = 0):
        L = load_library()
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        _check(L.qpe_ctx_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream)), "qpe_ctx_create")
        self.handle = h.value
        self.device = device

    def bind_current_stream(self) -> None:
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().qpe_ctx_set_stream(self.handle, ctypes.c_void_p(stream)), "qpe_ctx_set_stream")

    def set_variant(self, kernel_class: str, variant: int, n_mat: int = -1) -> None:
        """Select tile variant `variant` (0 = default) of a kernel class for
        operators of 2^n_mat (-1: all sizes)."""
        _check(load_library().qpe_ctx_set_variant(self.handle, KERNEL_CLASSES[kernel_class], int(n_mat),
                                                  int(variant)), "qpe_ctx_set_variant", self.handle)

    def get_variant(self, kernel_class: str, n_mat: int) -> int:
        v = ctypes.c_int()
        _check(load_library().qpe_ctx_get_variant(self.handle, KERNEL_CLASSES[kernel_class], int(n_mat),
                                                  ctypes.byref(v)), "qpe_ctx_get_variant", self.handle)
        return v.value

    def tuning_table(self) -> Dict[str, Dict[int, int]]:
        """Every non-default choice, {class: {n_mat: variant}} (JSON-friendly)."""
        out: Dict[str, Dict[int, int]] = {}
        for name in KERNEL_CLASSES:
            for t in range(0, 16):
                v = self.get_variant(name, t)
                if v:
                    out.setdefault(name, {})[t] = v
        return out

    def apply_tuning_table(self, table: Dict[str, Dict[int, int]]) -> None:
        for name, per in table.items():
            for t, v in per.items():
                self.set_variant(name, int(v), int(t))

    def autotune(self, U: torch.Tensor, psi: torch.Tensor, n_meas: int, form="mixed", flags: int = 0,
                 reps: int = 3) -> Dict:
        """Time every tile variant of the kernel classes this problem uses and
        keep the fastest in this context (see qpe_autotune). Synchronises."""
        d = U.shape[0]
        t = d.bit_length() - 1
        _need(U, torch.complex128, (d, d), "U")
        _need(psi, torch.complex128, (d,), "psi")
        f = _form(form)
        arr = (Problem * 1)()
        prob = torch.empty(1 << int(n_meas), dtype=torch.float64, device=U.device)
        arr[0].n_meas, arr[0].n_mat = int(n_meas), t
        arr[0].U, arr[0].psi, arr[0].prob = U.data_ptr(), psi.data_ptr(), prob.data_ptr()
        L = load_library()
        self.bind_current_stream()
        need = ctypes.c_size_t()
        _check(L.qpe_workspace_size(arr, 1, f, flags, ctypes.byref(need)), "qpe_workspace_size")
        ws = _alloc_ws(need.value, self.device)
        chosen = (ctypes.c_int * len(KERNEL_CLASSES))()
        ms = (ctypes.c_double * (len(KERNEL_CLASSES) * TUNE_MAX_VARIANTS))()
        _check(L.qpe_autotune(self.handle, arr, f, flags, ws.data_ptr(), ws.numel(), int(reps), chosen, ms),
               "qpe_autotune", self.handle)
        out = {"n_mat": t, "chosen": {}, "ms_per_circuit": {}}
        for name, c in KERNEL_CLASSES.items():
            tried = [round(ms[c * TUNE_MAX_VARIANTS + v], 4) for v in range(TUNE_MAX_VARIANTS)
                     if ms[c * TUNE_MAX_VARIANTS + v] >= 0]
            if tried:
                out["chosen"][name] = chosen[c]
                out["ms_per_circuit"][name] = tried
        return out

    def enable_timing(self, max_pairs: int = 4096) -> None:
        _check(load_library().qpe_ctx_enable_timing(self.handle, int(max_pairs)), "qpe_ctx_enable_timing",
               self.handle)

    def set_timing_mask(self, classes=None) -> None:
        """Time only the named classes (None: all of them)."""
        mask = (1 << len(TIMERS)) - 1 if classes is None else sum(1 << TIMERS[c] for c in classes)
        _check(load_library().qpe_ctx_set_timing_mask(self.handle, ctypes.c_uint(mask)), "qpe_ctx_set_timing_mask",
               self.handle)
        self.timing_classes = None if classes is None else list(classes)

    def reset_timing(self) -> None:
        _check(load_library().qpe_ctx_reset_timing(self.handle), "qpe_ctx_reset_timing")

    def read_timing(self) -> Dict[str, Tuple[int, float]]:
        """{class: (timed launches, summed ms)}; synchronises the events."""
        out = {}
        for name, idx in TIMERS.items():
            cnt, ms = ctypes.c_int(), ctypes.c_double()
            _check(load_library().qpe_ctx_read_timing(self.handle, idx, ctypes.byref(cnt), ctypes.byref(ms)),
                   "qpe_ctx_read_timing", self.handle)
            out[name] = (cnt.value, ms.value)
        return out

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.qpe_ctx_destroy(self.handle)
        except Exception:
            pass


_contexts: Dict[int, Context] = {}


def context(device: int) -> Context:
    c = _contexts.get(device)
    if c is None:
        c = Context(device)
        _contexts[device] = c
    c.bind_current_stream()
    return c


def _dev_index(t: torch.Tensor) -> int:
    if t.device.type != "cuda":
        raise ValueError("tensors must live on a HIP device (torch 'cuda' device)")
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


def _need(t: torch.Tensor, dtype: torch.dtype, shape: Tuple[int, ...], name: str) -> None:
    if t.dtype != dtype or tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError(f"{name}: need contiguous {dtype} of shape {shape}, got {t.dtype} {tuple(t.shape)}")


def _form(form) -> int:
    if isinstance(form, str):
        return FORMS[form]
    return int(form)


def workspace_bytes(shapes: Sequence[Tuple[int, int]], form="mixed", flags: int = 0) -> int:
    """Workspace qpe_run needs for (n_meas, n_mat) instances (host-only query)."""
    L = load_library()
    arr = (Problem * len(shapes))()
    for i, (n, t) in enumerate(shapes):
        arr[i].n_meas, arr[i].n_mat = int(n), int(t)
    out = ctypes.c_size_t()
    _check(L.qpe_workspace_size(arr, len(shapes), _form(form), flags, ctypes.byref(out)), "qpe_workspace_size")
    return out.value


def _alloc_ws(nbytes: int, device: int) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=f"cuda:{device}")


def run_batch(problems: Sequence[Tuple[torch.Tensor, torch.Tensor, int]], form="mixed", flags: int = 0,
              workspace: Optional[torch.Tensor] = None, report: bool = False):
    """QPE probabilities for each (U, psi, n_meas); U complex128 (d, d), psi
    complex128 (d,), all on one device. Returns a list of float64 tensors
    (and the per-instance reports as a numpy structured array if asked)."""
    if not problems:
        return []
    dev = _dev_index(problems[0][0])
    arr = (Problem * len(problems))()
    probs: List[torch.Tensor] = []
    for i, (U, psi, n) in enumerate(problems):
        d = U.shape[0]
        t = d.bit_length() - 1
        if d != (1 << t):
            raise ValueError("U must be 2^t x 2^t")
        _need(U, torch.complex128, (d, d), "U")
        _need(psi, torch.complex128, (d,), "psi")
        if _dev_index(U) != dev or _dev_index(psi) != dev:
            raise ValueError("all tensors must be on one device")
        p = torch.empty(1 << int(n), dtype=torch.float64, device=U.device)
        probs.append(p)
        arr[i].n_meas, arr[i].n_mat = int(n), t
        arr[i].U, arr[i].psi, arr[i].prob = U.data_ptr(), psi.data_ptr(), p.data_ptr()
    L = load_library()
    ctx = context(dev)
    f = _form(form)
    need = ctypes.c_size_t()
    _check(L.qpe_workspace_size(arr, len(problems), f, flags, ctypes.byref(need)), "qpe_workspace_size")
    if workspace is None or workspace.numel() < need.value:
        workspace = _alloc_ws(need.value, dev)
    rep = torch.empty(REPORT_BYTES * len(problems), dtype=torch.uint8, device=f"cuda:{dev}") if report else None
    _check(L.qpe_run(ctx.handle, arr, len(problems), f, flags, workspace.data_ptr(), workspace.numel(),
                     rep.data_ptr() if rep is not None else None), "qpe_run", ctx.handle)
    if report:
        torch.cuda.current_stream(dev).synchronize()
        r = np.frombuffer(rep.cpu().numpy().tobytes(), dtype=REPORT_DTYPE)
        return probs, r
    return probs


def run_batch_static(problems: Sequence[Tuple[torch.Tensor, torch.Tensor, int]], form="mixed", flags: int = 0,
                     report: bool = False):
    """run_batch through qpe_run_static: no workspace is allocated (the
    library's static device array serves as the workspace; problems that need
    more than STATIC_WORKSPACE_BYTES raise QpeError QPE_ERR_WORKSPACE). The
    outputs (P, and the report buffer if asked) are still allocated here."""
    if not problems:
        return []
    dev = _dev_index(problems[0][0])
    arr = (Problem * len(problems))()
    probs: List[torch.Tensor] = []
    for i, (U, psi, n) in enumerate(problems):
        d = U.shape[0]
        t = d.bit_length() - 1
        _need(U, torch.complex128, (d, d), "U")
        _need(psi, torch.complex128, (d,), "psi")
        p = torch.empty(1 << int(n), dtype=torch.float64, device=U.device)
        probs.append(p)
        arr[i].n_meas, arr[i].n_mat = int(n), t
        arr[i].U, arr[i].psi, arr[i].prob = U.data_ptr(), psi.data_ptr(), p.data_ptr()
    L = load_library()
    ctx = context(dev)
    rep = torch.empty(REPORT_BYTES * len(problems), dtype=torch.uint8, device=f"cuda:{dev}") if report else None
    _check(L.qpe_run_static(ctx.handle, arr, len(problems), _form(form), flags,
                            rep.data_ptr() if rep is not None else None), "qpe_run_static", ctx.handle)
    if report:
        torch.cuda.current_stream(dev).synchronize()
        return probs, np.frombuffer(rep.cpu().numpy().tobytes(), dtype=REPORT_DTYPE)
    return probs


def run(U: torch.Tensor, psi: torch.Tensor, n_meas: int, form="mixed", flags: int = 0,
        workspace: Optional[torch.Tensor] = None, report: bool = False):
    """QPE measurement probabilities (float64 tensor of length 2^n_meas)."""
    out = run_batch([(U, psi, n_meas)], form, flags, workspace, report)
    if report:
        return out[0][0], out[1][0]
    return out[0]


def run_state(U: torch.Tensor, psi: torch.Tensor, n_meas: int, form="mixed", flags: int = 0):
    """QPE probabilities and the final statevector A (2^n_meas x d, natural
    outcome order; complex64 for the mixed form, complex128 for FP64)."""
    d = U.shape[0]
    t = d.bit_length() - 1
    if d != (1 << t):
        raise ValueError("U must be 2^t x 2^t")
    _need(U, torch.complex128, (d, d), "U")
    _need(psi, torch.complex128, (d,), "psi")
    dev = _dev_index(U)
    f = _form(form)
    arr = (Problem * 1)()
    prob = torch.empty(1 << int(n_meas), dtype=torch.float64, device=U.device)
    state = torch.empty((1 << int(n_meas), d), dtype=torch.complex64 if f == FORM_MIXED else torch.complex128,
                        device=U.device)
    arr[0].n_meas, arr[0].n_mat = int(n_meas), t
    arr[0].U, arr[0].psi, arr[0].prob = U.data_ptr(), psi.data_ptr(), prob.data_ptr()
    L = load_library()
    ctx = context(dev)
    need = ctypes.c_size_t()
    _check(L.qpe_workspace_size(arr, 1, f, flags, ctypes.byref(need)), "qpe_workspace_size")
    ws = _alloc_ws(need.value, dev)
    _check(L.qpe_run_state(ctx.handle, arr, f, flags, ws.data_ptr(), ws.numel(), state.data_ptr(), None),
           "qpe_run_state", ctx.handle)
    return prob, state


def estimate(probs: Sequence[torch.Tensor]) -> np.ndarray:
    """Phase estimators (max-norm, weighted average, circular mean) of each
    float64 probability vector, computed on the device. Returns a numpy
    structured array with ESTIMATES_DTYPE fields, one entry per vector."""
    if not probs:
        return np.zeros(0, dtype=ESTIMATES_DTYPE)
    dev = _dev_index(probs[0])
    arr = (Problem * len(probs))()
    for i, p in enumerate(probs):
        N = p.numel()
        n = N.bit_length() - 1
        if N != (1 << n) or p.dtype != torch.float64 or not p.is_contiguous() or _dev_index(p) != dev:
            raise ValueError("each P must be a contiguous float64 vector of length 2^n on one device")
        arr[i].n_meas, arr[i].n_mat, arr[i].prob = n, 0, p.data_ptr()
    L = load_library()
    ctx = context(dev)
    need = ctypes.c_size_t()
    _check(L.qpe_estimate_workspace_size(len(probs), ctypes.byref(need)), "qpe_estimate_workspace_size")
    ws = _alloc_ws(need.value, dev)
    out = torch.empty(ESTIMATES_BYTES * len(probs), dtype=torch.uint8, device=f"cuda:{dev}")
    _check(L.qpe_estimate(ctx.handle, arr, len(probs), out.data_ptr(), ws.data_ptr(), ws.numel()),
           "qpe_estimate", ctx.handle)
    torch.cuda.current_stream(dev).synchronize()
    return np.frombuffer(out.cpu().numpy().tobytes(), dtype=ESTIMATES_DTYPE).copy()


def powers(U: torch.Tensor, count_k: int, flags: int = 0, report: bool = False):
    """V_k = U^(2^k), k < count_k, as a complex128 tensor (count_k, d, d)."""
    d = U.shape[0]
    t = d.bit_length() - 1
    _need(U, torch.complex128, (d, d), "U")
    dev = _dev_index(U)
    L = load_library()
    ctx = context(dev)
    need = ctypes.c_size_t()
    _check(L.qpe_powers_workspace_size(t, ctypes.byref(need)), "qpe_powers_workspace_size")
    ws = _alloc_ws(need.value, dev)
    V = torch.empty((count_k, d, d), dtype=torch.complex128, device=U.device)
    rep = torch.zeros(REPORT_BYTES, dtype=torch.uint8, device=U.device) if report else None
    _check(L.qpe_powers(ctx.handle, t, U.data_ptr(), int(count_k), flags, V.data_ptr(), ws.data_ptr(), ws.numel(),
                        rep.data_ptr() if rep is not None else None), "qpe_powers", ctx.handle)
    if report:
        torch.cuda.current_stream(dev).synchronize()
        return V, float(np.frombuffer(rep.cpu().numpy().tobytes()[:8], dtype="<f8")[0])
    return V


def controlled_step(V: torch.Tensor, state: torch.Tensor, k: int, form="mixed") -> torch.Tensor:
    """In place: rows j of state (N x d) with bit k set become row V^T."""
    f = _form(form)
    N, d = state.shape
    n, t = N.bit_length() - 1, d.bit_length() - 1
    _need(V, torch.complex128, (d, d), "V")
    _need(state, torch.complex64 if f == FORM_MIXED else torch.complex128, (N, d), "state")
    dev = _dev_index(state)
    L = load_library()
    ctx = context(dev)
    need = ctypes.c_size_t()
    _check(L.qpe_controlled_step_workspace_size(n, t, f, ctypes.byref(need)), "qpe_controlled_step_workspace_size")
    ws = _alloc_ws(need.value, dev)
    _check(L.qpe_controlled_step(ctx.handle, n, t, f, int(k), V.data_ptr(), state.data_ptr(), ws.data_ptr(),
                                 ws.numel()), "qpe_controlled_step", ctx.handle)
    return state


def iqft_probs(state: torch.Tensor, form="mixed") -> torch.Tensor:
    """Inverse QFT along rows of state (N x d, destroyed) and the readout."""
    f = _form(form)
    N, d = state.shape
    n, t = N.bit_length() - 1, d.bit_length() - 1
    _need(state, torch.complex64 if f == FORM_MIXED else torch.complex128, (N, d), "state")
    dev = _dev_index(state)
    L = load_library()
    ctx = context(dev)
    need = ctypes.c_size_t()
    _check(L.qpe_iqft_workspace_size(n, t, f, ctypes.byref(need)), "qpe_iqft_workspace_size")
    ws = _alloc_ws(need.value, dev)
    prob = torch.empty(N, dtype=torch.float64, device=state.device)
    _check(L.qpe_iqft_probs(ctx.handle, n, t, f, state.data_ptr(), prob.data_ptr(), ws.data_ptr(), ws.numel()),
           "qpe_iqft_probs", ctx.handle)
    return prob


def zgemm(opA: str, opB: str, A: torch.Tensor, B: torch.Tensor, alpha=1.0, beta=0.0,
          Cin: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """C = alpha op(A) op(B) + beta Cin on the FP64 matrix cores."""
    if A.dtype != torch.complex128 or B.dtype != torch.complex128:
        raise ValueError("zgemm takes complex128")
    A, B = A.contiguous(), B.contiguous()
    M = A.shape[0] if opA == "N" else A.shape[1]
    K = A.shape[1] if opA == "N" else A.shape[0]
    N = B.shape[1] if opB == "N" else B.shape[0]
    dev = _dev_index(A)
    C = out if out is not None else torch.empty((M, N), dtype=torch.complex128, device=A.device)
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    cin_ptr = Cin.data_ptr() if Cin is not None else None
    L = load_library()
    ctx = context(dev)
    _check(L.qpe_zgemm(ctx.handle, opA.encode(), opB.encode(), M, N, K, al, A.data_ptr(), A.shape[1], B.data_ptr(),
                       B.shape[1], be, cin_ptr, Cin.shape[1] if Cin is not None else N, C.data_ptr(), N),
           "qpe_zgemm", ctx.handle)
    return C


class Runner:
    """Pre-marshalled qpe_run call: problem array, outputs and workspace are
    prepared once, so repeated calls enqueue the kernels with no allocation
    (the form used by the benchmark and by HIP-graph capture)."""

    def __init__(self, problems: Sequence[Tuple[torch.Tensor, torch.Tensor, int]], form="mixed", flags: int = 0,
                 report: bool = True):
        if not problems:
            raise ValueError("no problems")
        self.dev = _dev_index(problems[0][0])
        self.form = _form(form)
        self.flags = int(flags)
        self.count = len(problems)
        self.arr = (Problem * self.count)()
        self.inputs = []
        self.probs: List[torch.Tensor] = []
        for i, (U, psi, n) in enumerate(problems):
            d = U.shape[0]
            t = d.bit_length() - 1
            _need(U, torch.complex128, (d, d), "U")
            _need(psi, torch.complex128, (d,), "psi")
            p = torch.empty(1 << int(n), dtype=torch.float64, device=U.device)
            self.inputs.append((U, psi))
            self.probs.append(p)
            self.arr[i].n_meas, self.arr[i].n_mat = int(n), t
            self.arr[i].U, self.arr[i].psi, self.arr[i].prob = U.data_ptr(), psi.data_ptr(), p.data_ptr()
        L = load_library()
        need = ctypes.c_size_t()
        _check(L.qpe_workspace_size(self.arr, self.count, self.form, self.flags, ctypes.byref(need)),
               "qpe_workspace_size")
        self.workspace = _alloc_ws(need.value, self.dev)
        self.report_buf = (torch.zeros(REPORT_BYTES * self.count, dtype=torch.uint8, device=f"cuda:{self.dev}")
                           if report else None)
        self.ctx = context(self.dev)

    def __call__(self) -> List[torch.Tensor]:
        L = load_library()
        self.ctx.bind_current_stream()  # the capture stream while a graph is recorded
        _check(L.qpe_run(self.ctx.handle, self.arr, self.count, self.form, self.flags, self.workspace.data_ptr(),
                         self.workspace.numel(),
                         self.report_buf.data_ptr() if self.report_buf is not None else None),
               "qpe_run", self.ctx.handle)
        return self.probs

    def autotune(self, reps: int = 2) -> Dict:
        """Batched runs (count >= 2): time every variant of the batched kernel
        classes over whole runs of this batch and keep the fastest in the
        context (qpe_autotune_batch). Synchronises; overwrites the outputs."""
        L = load_library()
        self.ctx.bind_current_stream()
        chosen = (ctypes.c_int * len(KERNEL_CLASSES))()
        ms = (ctypes.c_double * (len(KERNEL_CLASSES) * TUNE_MAX_VARIANTS))()
        _check(L.qpe_autotune_batch(self.ctx.handle, self.arr, self.count, self.form, self.flags,
                                    self.workspace.data_ptr(), self.workspace.numel(), int(reps), chosen, ms),
               "qpe_autotune_batch", self.ctx.handle)
        out = {"chosen": {}, "ms_per_batch": {}}
        for name, c in KERNEL_CLASSES.items():
            tried = [round(ms[c * TUNE_MAX_VARIANTS + v], 4) for v in range(TUNE_MAX_VARIANTS)
                     if ms[c * TUNE_MAX_VARIANTS + v] >= 0]
            if tried:
                out["chosen"][name] = chosen[c]
                out["ms_per_batch"][name] = tried
        return out

    def reports(self):
        torch.cuda.current_stream(self.dev).synchronize()
        if self.report_buf is None:
            return None
        return np.frombuffer(self.report_buf.cpu().numpy().tobytes(), dtype=REPORT_DTYPE)


def kernel_variants(kernel_class: str) -> int:
    """Number of tile variants of a kernel class (variant 0 = default)."""
    c = ctypes.c_int()
    _check(load_library().qpe_kernel_variants(KERNEL_CLASSES[kernel_class], ctypes.byref(c)), "qpe_kernel_variants")
    return c.value


class CapturedRun:
    """A Runner captured once into a HIP graph (through torch.cuda.CUDAGraph)
    and replayed: every launch of the batched run, including the device-side
    setup of descriptors and tables, is a graph node, so a replay costs one
    graph launch. Outputs are the Runner's tensors, rewritten by each replay."""

    def __init__(self, runner: Runner, warmup: int = 1):
        self.runner = runner
        side = torch.cuda.Stream(runner.dev)
        side.wait_stream(torch.cuda.current_stream(runner.dev))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                runner()
        torch.cuda.current_stream(runner.dev).wait_stream(side)
        torch.cuda.synchronize(runner.dev)
        # the per-kernel timers record events, which a graph must not hold
        saved = getattr(runner.ctx, "timing_classes", None)
        runner.ctx.set_timing_mask([])
        try:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                runner()
            torch.cuda.synchronize(runner.dev)
        finally:
            runner.ctx.set_timing_mask(saved)

    def __call__(self) -> List[torch.Tensor]:
        self.graph.replay()
        return self.runner.probs
