"""NN-sort oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow CPU statement of what the NN-sort hot path computes (Zhu et al.,
"Deep Learning Service for Efficient Data Distribution Aware Sorting", arXiv
1907.08817).  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library: the two meet only through plain numpy arrays handed over by the tests.

The arithmetic lives in ``nnsort_oracle.c`` (plain C, FP64 unless a function
says otherwise, built with ``-ffp-contract=off``).  This module is the ctypes
wrapper plus the parts of the procedure that are plain orchestration (the fit
loop, the sample sort -- a library sort serves as that step).

Every model here is a dict ``{"H", "lo", "inv_range", "theta"}``; ``theta`` is
the packed float32 vector w1[H] | b1[H] | W2[H*H] (row = hidden-2 unit) |
b2[H] | w3[H] | b3.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnsort_oracle.c")
# NNSORT_ORACLE_LIB names another build of the same source (the sanitizer
# test loads an ASan/UBSan build this way); it is then used as it is.
_LIB_PATH = os.environ.get("NNSORT_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

UNMAPPED = 0xFFFFFFFF
FORM_FP32C, FORM_FP64, FORM_BF16W = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (the checker, never the product)."""
    if os.environ.get("NNSORT_ORACLE_LIB"):
        return _LIB_PATH
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("collided", ctypes.c_int64 * 8), ("placed", ctypes.c_int64 * 8),
                ("extracted", ctypes.c_int64 * 8), ("residue", ctypes.c_int64),
                ("pos_err", ctypes.c_double)]


def _L():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64, u64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        lib.orc_order_key.restype = u64
        lib.orc_order_key.argtypes = [u64, i32]
        lib.orc_sort_bits.argtypes = [P, i64, i32, P]
        lib.orc_f_fp64.restype = f64
        lib.orc_f_fp64.argtypes = [i32, P, f64]
        lib.orc_f_fp32c.restype = f64
        lib.orc_f_fp32c.argtypes = [i32, P, f64]
        lib.orc_f_bf16w.restype = f64
        lib.orc_f_bf16w.argtypes = [i32, P, f64]
        lib.orc_round_bf16.restype = ctypes.c_float
        lib.orc_round_bf16.argtypes = [ctypes.c_float]
        lib.orc_slot.restype = ctypes.c_uint32
        lib.orc_slot.argtypes = [f64, f64]
        lib.orc_num_slots.restype = i64
        lib.orc_num_slots.argtypes = [i64, f64]
        lib.orc_predict_slots.argtypes = [P, i64, i32, i32, P, f64, f64, f64, i32, P]
        lib.orc_translate_many.argtypes = [P, i64, i32, f64, f64, P, P]
        lib.orc_eval_many.argtypes = [P, i64, i32, P, i32, P]
        lib.orc_nnsort.restype = i32
        lib.orc_nnsort.argtypes = [P, i64, i32, P, f64, i32, i64, P, ctypes.POINTER(_Stats)]
        lib.orc_pos_err.restype = f64
        lib.orc_pos_err.argtypes = [P, i64, i32, i32, P, f64, f64, i32, P]
        lib.orc_loss_grad_f64.restype = f64
        lib.orc_loss_grad_f64.argtypes = [i32, P, P, P, i64, i32, f64, P]
        lib.orc_loss_f64.restype = f64
        lib.orc_loss_f64.argtypes = [i32, P, P, P, i64, i32, f64]
        lib.orc_adam_step.argtypes = [P, P, P, P, i32, i64, f64, f64, f64, f64]
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_sample_indices.argtypes = [u64, i64, i64, P]
        lib.orc_batch_indices.argtypes = [u64, i64, i64, i64, P]
        lib.orc_init_uniform.restype = f64
        lib.orc_init_uniform.argtypes = [u64, i64, f64]
        lib.orc_slots_from_F.argtypes = [P, i64, f64, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _bits(x: np.ndarray) -> tuple[np.ndarray, int]:
    """Raw 64-bit patterns of a float64 or uint64 array, and the is_f64 flag."""
    x = np.ascontiguousarray(x)
    if x.dtype == np.float64:
        return x.view(np.uint64), 1
    if x.dtype == np.uint64:
        return x, 0
    raise TypeError("keys must be float64 or uint64")


def num_params(H: int) -> int:
    return H * H + 4 * H + 1


# --------------------------------------------------------------------------
# Definition of the result and order keys
# --------------------------------------------------------------------------
def order_keys(x: np.ndarray) -> np.ndarray:
    """totalOrder keys (uint64) of float64 keys; identity for uint64."""
    b, f = _bits(x)
    if not f:
        return b.copy()
    neg = (b >> np.uint64(63)).astype(bool)
    return np.where(neg, ~b, b | np.uint64(1 << 63))


def from_order_keys(k: np.ndarray, like_dtype) -> np.ndarray:
    if np.dtype(like_dtype) == np.uint64:
        return k.copy()
    top = (k >> np.uint64(63)).astype(bool)
    b = np.where(top, k & np.uint64(0x7FFFFFFFFFFFFFFF), ~k)
    return b.view(np.float64)


def sort_reference(x: np.ndarray) -> np.ndarray:
    """The plain definition of NN-sort's output: keys sorted by totalOrder.
    Uses numpy's sort on the order keys (a library sort as the step)."""
    return from_order_keys(np.sort(order_keys(x), kind="stable"), x.dtype)


def sort_reference_qsort(x: np.ndarray) -> np.ndarray:
    """Same definition through the C qsort (for small inputs)."""
    b, f = _bits(x)
    out = np.empty_like(b)
    _L().orc_sort_bits(_p(b), b.size, f, _p(out))
    return out.view(x.dtype)


# --------------------------------------------------------------------------
# Model evaluation and slots
# --------------------------------------------------------------------------
def translate(x: np.ndarray, lo: float, inv_range: float):
    b, f = _bits(x)
    xh = np.empty(b.size, np.float64)
    ok = np.empty(b.size, np.uint8)
    _L().orc_translate_many(_p(b), b.size, f, float(lo), float(inv_range), _p(xh), _p(ok))
    return xh, ok.astype(bool)


def eval_F(xhat: np.ndarray, model: dict, form: int = FORM_FP64) -> np.ndarray:
    xhat = np.ascontiguousarray(xhat, np.float64)
    th = np.ascontiguousarray(model["theta"], np.float32)
    F = np.empty(xhat.size, np.float64)
    _L().orc_eval_many(_p(xhat), xhat.size, int(model["H"]), _p(th), int(form), _p(F))
    return F


def num_slots(n: int, m: float = 1.25) -> int:
    return int(_L().orc_num_slots(int(n), float(m)))


def slot_of(F: float, M: float) -> int:
    return int(_L().orc_slot(float(F), float(M)))


def slots_from_F(F: np.ndarray, M: float) -> np.ndarray:
    F = np.ascontiguousarray(F, np.float64)
    out = np.empty(F.size, np.uint32)
    _L().orc_slots_from_F(_p(F), F.size, float(M), _p(out))
    return out


def predict_slots(x: np.ndarray, model: dict, m: float = 1.25, form: int = FORM_FP32C) -> np.ndarray:
    b, f = _bits(x)
    th = np.ascontiguousarray(model["theta"], np.float32)
    out = np.empty(b.size, np.uint32)
    _L().orc_predict_slots(_p(b), b.size, f, int(model["H"]), _p(th), float(model["lo"]),
                           float(model["inv_range"]), float(m), int(form), _p(out))
    return out


def round_bf16(v: float) -> float:
    return float(_L().orc_round_bf16(float(v)))


# --------------------------------------------------------------------------
# The method
# --------------------------------------------------------------------------
def nnsort(x: np.ndarray, model: dict, m: float = 1.25, eps: int = 3, tau: int = 1024,
           form: int = FORM_FP32C, slots: np.ndarray | None = None):
    """Procedure NN-sort with polish; returns (sorted keys, stats dict)."""
    b, f = _bits(x)
    if slots is None:
        slots = predict_slots(x, model, m, form)
    slots = np.ascontiguousarray(slots, np.uint32)
    out = np.empty_like(b)
    st = _Stats()
    rc = _L().orc_nnsort(_p(b), b.size, f, _p(slots), float(m), int(eps), int(tau), _p(out),
                         ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (eps out of range or slot >= S)")
    t = int(st.rounds)
    stats = {"n": int(st.n), "rounds": t,
             "collided": [int(st.collided[i]) for i in range(t)],
             "placed": [int(st.placed[i]) for i in range(t)],
             "extracted": [int(st.extracted[i]) for i in range(t)],
             "residue": int(st.residue)}
    return out.view(x.dtype), stats


def cost_operations(n: int, collided, placed, extracted, theta: float) -> float:
    """Operations of the procedure as Sec. 3 (Model Analysis) counts them,
    summed iteration by iteration from sizes, T = s(n) + p(n):
      s(n): iteration i feeds its input (n keys, then the conflict array left
            by iteration i - 1) through f at theta operations per key, and the
            last conflict array is sorted conventionally, |w| log2 |w|;
      p(n): each out-of-order key of o_i is inserted at half the size of
            iteration i's input; every other key of o_i, and every key of the
            conflict array after iteration i, is appended once.
    collided[i] = |c_{i+1}|, placed[i] = keys stored in o_{i+1},
    extracted[i] = those out of order (this oracle's round statistics)."""
    if n <= 1:
        return 1.0
    total = 0.0
    w = float(n)  # input of the current iteration
    for c, p, x in zip(collided, placed, extracted):
        total += theta * w
        total += x * w / 2.0
        total += (p - x) + c
        w = float(c)
    if w > 0:
        total += w * math.log2(w)
    return total


def pos_err(sorted_x: np.ndarray, model: dict, form: int = FORM_FP64) -> float:
    b, f = _bits(sorted_x)
    th = np.ascontiguousarray(model["theta"], np.float32)
    cnt = ctypes.c_int64(0)
    return float(_L().orc_pos_err(_p(b), b.size, f, int(model["H"]), _p(th), float(model["lo"]),
                                  float(model["inv_range"]), int(form), ctypes.byref(cnt)))


# --------------------------------------------------------------------------
# Training (FP64 reference)
# --------------------------------------------------------------------------
def loss_grad(theta64: np.ndarray, H: int, x: np.ndarray, y: np.ndarray, loss: int = 0,
              delta: float = 1.0):
    th = np.ascontiguousarray(theta64, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    g = np.empty(num_params(H), np.float64)
    L = _L().orc_loss_grad_f64(H, _p(th), _p(x), _p(y), x.size, int(loss), float(delta), _p(g))
    return float(L), g


def loss_value(theta64: np.ndarray, H: int, x: np.ndarray, y: np.ndarray, loss: int = 0,
               delta: float = 1.0) -> float:
    th = np.ascontiguousarray(theta64, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    return float(_L().orc_loss_f64(H, _p(th), _p(x), _p(y), x.size, int(loss), float(delta)))


def adam_step(theta: np.ndarray, g: np.ndarray, m1: np.ndarray, m2: np.ndarray, t: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """In-place Adam update of float64 arrays."""
    for a in (theta, g, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _L().orc_adam_step(_p(theta), _p(g), _p(m1), _p(m2), theta.size, int(t), float(lr),
                       float(beta1), float(beta2), float(eps))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.empty(4, np.uint32)
    _L().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def sample_indices(seed: int, n: int, k: int) -> np.ndarray:
    out = np.empty(k, np.int64)
    _L().orc_sample_indices(int(seed), int(n), int(k), _p(out))
    return out


def batch_indices(seed: int, step: int, k: int, B: int) -> np.ndarray:
    out = np.empty(B, np.int64)
    _L().orc_batch_indices(int(seed), int(step), int(k), int(B), _p(out))
    return out


def init_uniform(seed: int, p: int, bound: float) -> float:
    return float(_L().orc_init_uniform(int(seed), int(p), float(bound)))


RAMP_MIN_WIDTH = 2.0 ** -40


def sample_count(n: int, frac: float) -> int:
    return max(1, int(math.floor(frac * n + 0.5)))


def fit_sample(x: np.ndarray, sample_frac: float, seed: int):
    """Training set of the fit: a random sample (with replacement) of the keys,
    finite keys only, sorted; returns (sorted sample, lo, inv_range, xhat, y)
    with label y_j = (j + 0.5)/k, the normalised rank."""
    n = x.size
    k = sample_count(n, sample_frac)
    idx = sample_indices(seed, n, k)
    s = x[idx]
    if x.dtype == np.float64:
        s = s[np.isfinite(s)]
    s = sort_reference(s)
    k2 = s.size
    if k2 == 0:
        return s, 0.0, 0.0, np.zeros(0), np.zeros(0)
    lo = float(s[0])
    hi = float(s[-1])
    inv = 1.0 / (hi - lo) if hi > lo else 0.0
    xh, _ = translate(s, lo, inv)
    y = (np.arange(k2, dtype=np.float64) + 0.5) / k2
    return s, lo, inv, xh, y


def greedy_knot_indices(xs: np.ndarray, H: int) -> np.ndarray:
    """Knots of the piecewise-linear interpolant of the sample CDF by greedy
    splitting: starting from one piece over the sorted sample xs (ranks
    y_j = (j + 0.5)/k), repeatedly split the piece whose points deviate most
    (in rank) from the chord between its ends, at the point of largest
    deviation, until H pieces.  Ties: the piece with the smaller start, then
    the smaller point index.  A piece with fewer than 3 points, zero width, or
    no point farther than one rank step (1/k) from the chord is never split.  Returns H + 1 sorted sample indices (the last repeated
    if fewer than H pieces arise)."""
    k = xs.size
    y = (np.arange(k, dtype=np.float64) + 0.5) / k

    def dev(a, b):
        if b - a < 2 or xs[b] == xs[a]:
            return 0.0, -1
        j = np.arange(a + 1, b)
        lin = y[a] + (y[b] - y[a]) * (xs[j] - xs[a]) / (xs[b] - xs[a])
        d = np.abs(y[j] - lin)
        m = int(np.argmax(d))   # first maximum
        if not d[m] > 1.0 / k:
            return 0.0, -1
        return float(d[m]), int(j[m])

    pieces = {0: (k - 1,) + dev(0, k - 1)}    # start -> (end, deviation, split point)
    while len(pieces) < H:
        best = None
        for a in sorted(pieces):
            b, d, j = pieces[a]
            if j >= 0 and d > 0 and (best is None or d > pieces[best][1]):
                best = a
        if best is None:
            break
        b, d, j = pieces[best]
        pieces[best] = (j,) + dev(best, j)
        pieces[j] = (b,) + dev(j, b)
    idx = sorted(pieces) + [k - 1]
    while len(idx) < H + 1:
        idx.append(k - 1)
    return np.array(idx, np.int64)


def init_theta(H: int, init: int, seed: int, xhat_sorted: np.ndarray) -> np.ndarray:
    """Initial weights (float64 holding float32-rounded values).

    init 1 and 2 (ramps): the piecewise-linear interpolant of the sample CDF
    through knots (q_i, F_i), i = 0..H (q_i = sample value at knot index
    idx_i, F_i = (idx_i + 0.5)/k), written as a network: hidden-1 unit i is
    u_i = relu(s_i (x - q_i)) with s_i = 1/max(q_{i+1} - q_i, RAMP_MIN_WIDTH),
    hidden-2 unit i is v_i = relu(1 - u_i) (a ramp from 1 down to 0 across
    piece i), and F = F_H - sum_i (F_{i+1} - F_i) v_i.  Slopes sit in layer 1 so
    that an Adam step (about lr whatever a parameter's scale) moves a knot by
    about lr times the piece width.  init 1 places the knots by greedy
    maximum-deviation splitting (greedy_knot_indices), init 2 at the quantiles
    j/H.
    init 0: uniform(+-1/sqrt(fan_in)) from Philox."""
    P = num_params(H)
    th = np.zeros(P, np.float64)
    w1, b1 = slice(0, H), slice(H, 2 * H)
    W2 = slice(2 * H, 2 * H + H * H)
    b2 = slice(2 * H + H * H, 3 * H + H * H)
    w3 = slice(3 * H + H * H, 4 * H + H * H)
    if init in (1, 2):
        k = xhat_sorted.size
        if k == 0:
            return th.astype(np.float32).astype(np.float64)
        if init == 1:
            idx = greedy_knot_indices(xhat_sorted, H)
        else:
            idx = np.array([(j * (k - 1)) // H for j in range(H + 1)], np.int64)
        q = xhat_sorted[idx]
        Fk = (idx.astype(np.float64) + 0.5) / k
        width = np.maximum(q[1:] - q[:-1], RAMP_MIN_WIDTH)
        s = 1.0 / width
        th[w1] = s
        th[b1] = -s * q[:H]
        Wm = np.zeros((H, H))
        np.fill_diagonal(Wm, -1.0)
        th[W2] = Wm.ravel()
        th[b2] = 1.0
        th[w3] = -(Fk[1:] - Fk[:-1])
        th[P - 1] = Fk[H]
    else:
        bound2 = 1.0 / math.sqrt(H)
        for p in range(P):
            bound = 1.0 if p < 2 * H else bound2
            th[p] = init_uniform(seed, p, bound)
    return th.astype(np.float32).astype(np.float64)


def fit(x: np.ndarray, H: int = 32, sample_frac: float = 0.01, batch: int = 65536,
        steps: int = 200, lr: float = 1e-7, seed: int = 0, init: int = 1, loss: int = 0,
        delta: float = 1.0, return_history: bool = False):
    """CPU FP64 fit of the CDF model: Adam on MSE (loss 0) or the paper's Huber
    loss (loss 1) to the normalised rank of a random sample.  Returns the
    parameters with the lowest batch loss seen (a step's loss is measured
    before its update), unless they move F backwards along the sorted sample
    more than the initial parameters do (disorder sum_j max(0, F_j - F_{j+1}));
    then the initial parameters."""
    s, lo, inv, xh, y = fit_sample(x, sample_frac, seed)
    th = init_theta(H, init, seed, xh)
    th0 = th.copy()
    best, best_loss = th.copy(), math.inf
    m1 = np.zeros_like(th)
    m2 = np.zeros_like(th)
    hist = []
    k2 = xh.size
    for t in range(1, steps + 1):
        if k2 == 0:
            break
        bi = batch_indices(seed, t, k2, batch)
        L, g = loss_grad(th, H, xh[bi], y[bi], loss, delta)
        hist.append(L)
        if L < best_loss:
            best, best_loss = th.copy(), L
        adam_step(th, g, m1, m2, t, lr)
    if steps > 0 and k2 > 1:
        def disorder(t):
            F = eval_F(xh, {"H": H, "theta": t.astype(np.float32)}, FORM_FP64)
            return float(np.maximum(F[:-1] - F[1:], 0.0).sum())
        if disorder(best) > disorder(th0):
            best = th0
    model = {"H": H, "lo": lo, "inv_range": inv, "theta": best.astype(np.float32)}
    if return_history:
        return model, hist
    return model
