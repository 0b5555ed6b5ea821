"""NN-sort on MI355X: Python binding of libnnsort (the C ABI in include/nnsort.h).

Argument marshalling only: every step of the sort and of the fit runs in the
library's HIP kernels.  PyTorch supplies device memory and the current stream.
The binding fails loudly when the library has not been built; there is no CPU
fallback.

Keys are 1-D CUDA tensors of torch.float64 (IEEE binary64, sorted by
totalOrder) or torch.uint64 / torch.int64 (raw unsigned 64-bit integers).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnsort.so")

NNSORT_ABI_VERSION = 1
MAX_HIDDEN = 64
MAX_EPS = 8
F64, U64 = 0, 1
FORM_FP32, FORM_BF16, FORM_PWL = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "EWORKSPACE", -3: "EHIP", -4: "EMODEL", -5: "EIO", -6: "EINTERNAL",
          -7: "ETOOBIG"}


class NNSortError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib().nnsort_strerror(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")


class SortParams(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("eps", ctypes.c_int32), ("form", ctypes.c_int32),
                ("tau", ctypes.c_int64), ("bf16_terms", ctypes.c_int32), ("stats_level", ctypes.c_int32)]


class FitParams(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("batch", ctypes.c_int32), ("sample_frac", ctypes.c_double),
                ("steps", ctypes.c_int32), ("lr", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("loss", ctypes.c_int32), ("huber_delta", ctypes.c_float), ("init", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Model(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("hidden", ctypes.c_int32), ("lo", ctypes.c_double),
                ("inv_range", ctypes.c_double), ("w1", ctypes.c_float * MAX_HIDDEN),
                ("b1", ctypes.c_float * MAX_HIDDEN), ("w2", ctypes.c_float * (MAX_HIDDEN * MAX_HIDDEN)),
                ("b2", ctypes.c_float * MAX_HIDDEN), ("w3", ctypes.c_float * MAX_HIDDEN),
                ("b3", ctypes.c_float), ("reserved", ctypes.c_float * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rounds", ctypes.c_int32), ("form", ctypes.c_int32),
                ("collided", ctypes.c_int64 * MAX_EPS), ("placed", ctypes.c_int64 * MAX_EPS),
                ("residue", ctypes.c_int64), ("unmapped", ctypes.c_int64), ("big_buckets", ctypes.c_int64),
                ("big_bucket_keys", ctypes.c_int64), ("boundary_keys", ctypes.c_int64),
                ("fallback", ctypes.c_int32), ("range_resorts", ctypes.c_int32), ("pos_err", ctypes.c_double),
                ("t_infer_ms", ctypes.c_double), ("t_place_ms", ctypes.c_double),
                ("t_polish_ms", ctypes.c_double), ("t_residue_ms", ctypes.c_double),
                ("t_merge_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double), ("t_fit_ms", ctypes.c_double)]


_LIB = None


def _lib():
    """Load libnnsort.so; raise if it is not built (no fallback exists)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1907_08817_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
        pS, pF, pM, pT = (ctypes.POINTER(SortParams), ctypes.POINTER(FitParams), ctypes.POINTER(Model),
                          ctypes.POINTER(Stats))
        sig = {
            "nnsort_default_params": (None, [pS, pF]),
            "nnsort_workspace_size": (i32, [i64, i32, pS, pF, ctypes.POINTER(sz)]),
            "nnsort_fit": (i32, [P, i64, i32, pF, pM, P, sz, P]),
            "nnsort_fit_history": (i32, [P, i64, i32, pF, pM, P, sz, ctypes.POINTER(f32), i32, P]),
            "nnsort_sort_with_model": (i32, [pM, P, P, i64, i32, pS, P, sz, pT, P]),
            "nnsort_sort_with_model_noalloc": (i32, [pM, P, P, i64, i32, pS, pT, P]),
            "nnsort_sort": (i32, [P, P, i64, i32, pF, pS, P, sz, pM, pT, P]),
            "nnsort_model_device_bytes": (sz, []),
            "nnsort_predict": (i32, [pM, P, i64, i32, pS, P, P, P, sz, P]),
            "nnsort_sort_with_slots": (i32, [P, P, P, i64, i32, pS, P, sz, pT, P]),
            "nnsort_radix_workspace_size": (sz, [i64]),
            "nnsort_radix_sort": (i32, [P, P, i64, i32, P, sz, P]),
            "nnsort_mlp_saved_floats": (sz, [i32, i64]),
            "nnsort_mlp_backward_ws_floats": (sz, [i32, i64]),
            "nnsort_mlp_forward": (i32, [i32, P, P, i64, P, P, P]),
            "nnsort_mlp_backward": (i32, [i32, P, P, i64, P, P, P, P, P]),
            "nnsort_loss_ws_floats": (sz, []),
            "nnsort_fit_gradient_ws_floats": (sz, [i32, i64]),
            "nnsort_fit_gradient": (i32, [i32, P, P, P, i64, i64, ctypes.c_uint64, i64, i32, f32, P, P, P, sz, P]),
            "nnsort_loss_grad": (i32, [P, P, i64, i32, f32, P, P, P, P]),
            "nnsort_adam_step": (i32, [P, P, P, P, i64, i64, f32, f32, f32, f32, P]),
            "nnsort_model_save": (i32, [pM, ctypes.c_char_p]),
            "nnsort_model_load": (i32, [pM, ctypes.c_char_p]),
            "nnsort_strerror": (ctypes.c_char_p, [i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def exported_symbols() -> list:
    return [n for n in ("nnsort_default_params", "nnsort_workspace_size", "nnsort_fit", "nnsort_fit_history",
                        "nnsort_sort_with_model", "nnsort_sort_with_model_noalloc", "nnsort_sort", "nnsort_model_device_bytes", "nnsort_predict",
                        "nnsort_sort_with_slots", "nnsort_radix_workspace_size", "nnsort_radix_sort",
                        "nnsort_mlp_saved_floats", "nnsort_mlp_backward_ws_floats", "nnsort_mlp_forward",
                        "nnsort_mlp_backward", "nnsort_loss_ws_floats", "nnsort_loss_grad", "nnsort_adam_step",
                        "nnsort_fit_gradient_ws_floats", "nnsort_fit_gradient",
                        "nnsort_model_save", "nnsort_model_load", "nnsort_strerror")
            if hasattr(_lib(), n)]


def _check(rc: int, where: str):
    if rc != 0:
        raise NNSortError(rc, where)


# ---------------------------------------------------------------------------
# parameters and models
# ---------------------------------------------------------------------------
def default_params() -> tuple[SortParams, FitParams]:
    sp, fp = SortParams(), FitParams()
    _lib().nnsort_default_params(ctypes.byref(sp), ctypes.byref(fp))
    return sp, fp


def _set_fields(st, kw):
    names = {f[0] for f in type(st)._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"{type(st).__name__} has no field {k!r}")
        setattr(st, k, v)
    return st


def sort_params(**kw) -> SortParams:
    sp, _ = default_params()
    return _set_fields(sp, kw)


def fit_params(**kw) -> FitParams:
    _, fp = default_params()
    return _set_fields(fp, kw)


def model_from_dict(d: dict) -> Model:
    """Build the C model from {"H", "lo", "inv_range", "theta"} with theta the
    packed float32 vector w1 | b1 | W2 (row = hidden-2 unit) | b2 | w3 | b3."""
    H = int(d["H"])
    th = np.ascontiguousarray(d["theta"], np.float32)
    assert th.size == H * H + 4 * H + 1
    m = Model()
    m.version = NNSORT_ABI_VERSION
    m.hidden = H
    m.lo = float(d["lo"])
    m.inv_range = float(d["inv_range"])
    o = 0
    for name, cnt in (("w1", H), ("b1", H), ("w2", H * H), ("b2", H), ("w3", H)):
        arr = getattr(m, name)
        ctypes.memmove(arr, th[o:o + cnt].ctypes.data, cnt * 4)
        o += cnt
    m.b3 = float(th[o])
    return m


def model_to_dict(m: Model) -> dict:
    H = m.hidden
    parts = [np.ctypeslib.as_array(m.w1)[:H], np.ctypeslib.as_array(m.b1)[:H],
             np.ctypeslib.as_array(m.w2)[:H * H], np.ctypeslib.as_array(m.b2)[:H],
             np.ctypeslib.as_array(m.w3)[:H], np.array([m.b3], np.float32)]
    return {"H": H, "lo": m.lo, "inv_range": m.inv_range,
            "theta": np.concatenate(parts).astype(np.float32)}


def stats_to_dict(s: Stats) -> dict:
    t = s.rounds
    return {"n": s.n, "rounds": t, "form": s.form, "collided": list(s.collided)[:t],
            "placed": list(s.placed)[:t], "residue": s.residue, "unmapped": s.unmapped,
            "big_buckets": s.big_buckets, "big_bucket_keys": s.big_bucket_keys,
            "boundary_keys": s.boundary_keys, "fallback": s.fallback, "range_resorts": s.range_resorts, "pos_err": s.pos_err,
            "t_infer_ms": s.t_infer_ms, "t_place_ms": s.t_place_ms, "t_polish_ms": s.t_polish_ms,
            "t_residue_ms": s.t_residue_ms, "t_merge_ms": s.t_merge_ms, "t_total_ms": s.t_total_ms,
            "t_fit_ms": s.t_fit_ms}


def model_save(m: Model, path: str):
    _check(_lib().nnsort_model_save(ctypes.byref(m), path.encode()), "nnsort_model_save")


def model_load(path: str) -> Model:
    m = Model()
    _check(_lib().nnsort_model_load(ctypes.byref(m), path.encode()), "nnsort_model_load")
    return m


# ---------------------------------------------------------------------------
# tensors
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype in (torch.int64, getattr(torch, "uint64", torch.int64)):
        return U64
    raise TypeError("keys must be float64, uint64 or int64 (raw bits)")


def _keys(t):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dim() == 1 and t.is_contiguous()):
        raise ValueError("keys must be a contiguous 1-D CUDA tensor")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace_size(n: int, dtype: int, sp: SortParams, fp: FitParams | None = None) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib().nnsort_workspace_size(int(n), int(dtype), ctypes.byref(sp),
                                        ctypes.byref(fp) if fp is not None else None, ctypes.byref(out)),
           "nnsort_workspace_size")
    return int(out.value)


def alloc_workspace(nbytes: int, device=None):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def nnsort_fit(keys, fp: FitParams | None = None, ws=None, stream=None, history: bool = False):
    """Fit the CDF model on the device; returns the Model (and the batch loss
    history when history=True)."""
    keys = _keys(keys)
    fp = fp or default_params()[1]
    sp = default_params()[0]
    dt = _dtype_code(keys)
    if ws is None:
        ws = alloc_workspace(workspace_size(keys.numel(), dt, sp, fp), keys.device)
    m = Model()
    if history:
        hist = (ctypes.c_float * max(1, fp.steps))()
        rc = _lib().nnsort_fit_history(_ptr(keys), keys.numel(), dt, ctypes.byref(fp), ctypes.byref(m),
                                       _ptr(ws), ws.numel(), hist, fp.steps, _stream(stream))
        _check(rc, "nnsort_fit_history")
        return m, [float(v) for v in hist[:fp.steps]]
    rc = _lib().nnsort_fit(_ptr(keys), keys.numel(), dt, ctypes.byref(fp), ctypes.byref(m), _ptr(ws),
                           ws.numel(), _stream(stream))
    _check(rc, "nnsort_fit")
    return m


def nnsort_sort_with_model(model: Model, keys, out=None, sp: SortParams | None = None, ws=None, stream=None):
    """Sort keys with a given model; returns (sorted tensor, stats dict)."""
    torch = _torch()
    keys = _keys(keys)
    sp = sp or default_params()[0]
    dt = _dtype_code(keys)
    if out is None:
        out = torch.empty_like(keys)
    if ws is None:
        ws = alloc_workspace(workspace_size(keys.numel(), dt, sp), keys.device)
    st = Stats()
    rc = _lib().nnsort_sort_with_model(ctypes.byref(model), _ptr(keys), _ptr(out), keys.numel(), dt,
                                       ctypes.byref(sp), _ptr(ws), ws.numel(), ctypes.byref(st), _stream(stream))
    _check(rc, "nnsort_sort_with_model")
    return out, stats_to_dict(st)


def nnsort_sort_with_model_noalloc(model: Model, keys, out=None, sp: SortParams | None = None, stream=None):
    """Sort keys with a given model in the library's static device scratch (no
    workspace; inputs up to about 1.5M keys); returns (sorted tensor, stats)."""
    torch = _torch()
    keys = _keys(keys)
    sp = sp or default_params()[0]
    if out is None:
        out = torch.empty_like(keys)
    st = Stats()
    rc = _lib().nnsort_sort_with_model_noalloc(ctypes.byref(model), _ptr(keys), _ptr(out), keys.numel(),
                                               _dtype_code(keys), ctypes.byref(sp), ctypes.byref(st),
                                               _stream(stream))
    _check(rc, "nnsort_sort_with_model_noalloc")
    return out, stats_to_dict(st)


def nnsort_sort(keys, fp: FitParams | None = None, sp: SortParams | None = None, out=None, ws=None, stream=None):
    """Fit on the keys, then sort them; returns (sorted, model, stats)."""
    torch = _torch()
    keys = _keys(keys)
    sp0, fp0 = default_params()
    sp = sp or sp0
    fp = fp or fp0
    dt = _dtype_code(keys)
    if out is None:
        out = torch.empty_like(keys)
    if ws is None:
        ws = alloc_workspace(workspace_size(keys.numel(), dt, sp, fp), keys.device)
    m, st = Model(), Stats()
    rc = _lib().nnsort_sort(_ptr(keys), _ptr(out), keys.numel(), dt, ctypes.byref(fp), ctypes.byref(sp), _ptr(ws),
                            ws.numel(), ctypes.byref(m), ctypes.byref(st), _stream(stream))
    _check(rc, "nnsort_sort")
    return out, m, stats_to_dict(st)


def nnsort_predict(model: Model, keys, sp: SortParams | None = None, want_slots=True, want_F=True, stream=None):
    """Per-key slot (uint32 as int64 tensor) and F (float64) of the model map."""
    torch = _torch()
    keys = _keys(keys)
    sp = sp or default_params()[0]
    n = keys.numel()
    slots = torch.empty(n, dtype=torch.int32, device=keys.device) if want_slots else None
    F = torch.empty(n, dtype=torch.float64, device=keys.device) if want_F else None
    ws = alloc_workspace(_lib().nnsort_model_device_bytes(), keys.device)
    rc = _lib().nnsort_predict(ctypes.byref(model), _ptr(keys), n, _dtype_code(keys), ctypes.byref(sp),
                               _ptr(slots), _ptr(F), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "nnsort_predict")
    if slots is not None:
        slots = slots.to(torch.int64) & 0xFFFFFFFF
    return slots, F


def nnsort_sort_with_slots(slots, keys, out=None, sp: SortParams | None = None, ws=None, stream=None):
    """Sorting and polish phases from caller-given slots (uint32 values in an
    int32/int64 tensor; 0xFFFFFFFF = no slot)."""
    torch = _torch()
    keys = _keys(keys)
    sp = sp or default_params()[0]
    dt = _dtype_code(keys)
    s32 = slots.to(torch.int64).to(torch.int32) if slots.dtype != torch.int32 else slots.contiguous()
    if out is None:
        out = torch.empty_like(keys)
    if ws is None:
        ws = alloc_workspace(workspace_size(keys.numel(), dt, sp), keys.device)
    st = Stats()
    rc = _lib().nnsort_sort_with_slots(_ptr(s32), _ptr(keys), _ptr(out), keys.numel(), dt, ctypes.byref(sp),
                                       _ptr(ws), ws.numel(), ctypes.byref(st), _stream(stream))
    _check(rc, "nnsort_sort_with_slots")
    return out, stats_to_dict(st)


def nnsort_radix_sort(keys, out=None, ws=None, stream=None):
    torch = _torch()
    keys = _keys(keys)
    if out is None:
        out = torch.empty_like(keys)
    if ws is None:
        ws = alloc_workspace(_lib().nnsort_radix_workspace_size(keys.numel()), keys.device)
    rc = _lib().nnsort_radix_sort(_ptr(keys), _ptr(out), keys.numel(), _dtype_code(keys), _ptr(ws), ws.numel(),
                                  _stream(stream))
    _check(rc, "nnsort_radix_sort")
    return out


# ---------------------------------------------------------------------------
# training pieces and the autograd Function
# ---------------------------------------------------------------------------
def nnsort_mlp_forward(hidden: int, theta, x, saved=None, stream=None):
    torch = _torch()
    F = torch.empty(x.numel(), dtype=torch.float32, device=x.device)
    rc = _lib().nnsort_mlp_forward(hidden, _ptr(theta), _ptr(x), x.numel(), _ptr(F), _ptr(saved), _stream(stream))
    _check(rc, "nnsort_mlp_forward")
    return F


def nnsort_mlp_backward(hidden: int, theta, x, saved, gF, stream=None):
    torch = _torch()
    B = x.numel()
    g = torch.empty(theta.numel(), dtype=torch.float32, device=x.device)
    ws = torch.empty(int(_lib().nnsort_mlp_backward_ws_floats(hidden, B)), dtype=torch.float32, device=x.device)
    rc = _lib().nnsort_mlp_backward(hidden, _ptr(theta), _ptr(x), B, _ptr(saved), _ptr(gF), _ptr(g), _ptr(ws),
                                    _stream(stream))
    _check(rc, "nnsort_mlp_backward")
    return g


def nnsort_loss_grad(F, y, loss: int = 0, delta: float = 1.0, stream=None):
    torch = _torch()
    gF = torch.empty_like(F)
    L = torch.empty(1, dtype=torch.float32, device=F.device)
    ws = torch.empty(int(_lib().nnsort_loss_ws_floats()), dtype=torch.float32, device=F.device)
    rc = _lib().nnsort_loss_grad(_ptr(F), _ptr(y), F.numel(), loss, float(delta), _ptr(gF), _ptr(L), _ptr(ws),
                                 _stream(stream))
    _check(rc, "nnsort_loss_grad")
    return L, gF


def nnsort_fit_gradient(hidden: int, theta, x, y, batch: int, seed: int, step: int, loss: int = 0,
                        delta: float = 1.0, stream=None):
    """Gradient and loss of one fit step (the fused kernel nnsort_fit runs for
    hidden 32 and 64) on a batch drawn from the sample (x float64, y float32);
    returns (loss tensor [1], gtheta tensor [P])."""
    torch = _torch()
    g = torch.empty(theta.numel(), dtype=torch.float32, device=x.device)
    L = torch.empty(1, dtype=torch.float32, device=x.device)
    wf = int(_lib().nnsort_fit_gradient_ws_floats(hidden, batch))
    ws = torch.empty(wf, dtype=torch.float32, device=x.device)
    rc = _lib().nnsort_fit_gradient(hidden, _ptr(theta), _ptr(x), _ptr(y), x.numel(), int(batch), int(seed),
                                    int(step), int(loss), float(delta), _ptr(g), _ptr(L), _ptr(ws), wf,
                                    _stream(stream))
    _check(rc, "nnsort_fit_gradient")
    return L, g


def nnsort_adam_step(theta, g, m1, m2, t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                     eps: float = 1e-8, stream=None):
    rc = _lib().nnsort_adam_step(_ptr(theta), _ptr(g), _ptr(m1), _ptr(m2), theta.numel(), int(t), float(lr),
                                 float(beta1), float(beta2), float(eps), _stream(stream))
    _check(rc, "nnsort_adam_step")


def _autograd_fn():
    torch = _torch()

    class NNSortMLPFn(torch.autograd.Function):
        """F = f(x; theta) through the hand-written forward/backward kernels.
        x: (B,) float64 normalised inputs; theta: packed float32 parameters."""

        @staticmethod
        def forward(ctx, x, theta, hidden: int):
            saved = torch.empty(int(_lib().nnsort_mlp_saved_floats(hidden, x.numel())), dtype=torch.float32,
                                device=x.device)
            F = nnsort_mlp_forward(hidden, theta.contiguous(), x.contiguous(), saved)
            ctx.save_for_backward(x, theta, saved)
            ctx.hidden = hidden
            return F

        @staticmethod
        def backward(ctx, gF):
            x, theta, saved = ctx.saved_tensors
            g = nnsort_mlp_backward(ctx.hidden, theta.contiguous(), x.contiguous(), saved,
                                    gF.contiguous().to(torch.float32))
            return None, g, None

    return NNSortMLPFn


_FN = None


def NNSortMLPFn():
    global _FN
    if _FN is None:
        _FN = _autograd_fn()
    return _FN


def mlp(x, theta, hidden: int):
    """Differentiable model evaluation (hand-written kernels)."""
    return NNSortMLPFn().apply(x, theta, hidden)
