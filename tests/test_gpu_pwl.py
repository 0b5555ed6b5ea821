"""The piecewise-linear form of the model map (NNSORT_FORM_PWL) against the
oracle.

The form evaluates the FP64 model through the affine pieces between its ReLU
breakpoints, compiled on the device from the weights.  Its F is checked against
the oracle's direct FP64 evaluation of the same weights within an a-priori
bound: both sides round sums whose terms are at most the un-cancelled
magnitude M = |b3| + sum_i |w3_i| (|b2_i| + sum_k |W2_ik| (|w1_k| + |b1_k|))
for x in [0, 1] (the compile forms z2 = A x + B from such terms), so
|F_pwl - F_fp64| <= (4H + 16) 2^-53 M.  Sorted output: bit-exact with the
oracle's sort.  Round counts: the slot-histogram identity on the form's own
slots.
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_1907_08817_amd as nn
from paper_1907_08817_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U64 = 2.0 ** -53


def to_dev(x: np.ndarray):
    if x.dtype == np.float64:
        return torch.from_numpy(x.copy()).to(DEV)
    return torch.from_numpy(x.view(np.int64).copy()).to(DEV)


def random_model(H, seed, lo=0.0, inv=1.0):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-1, 1, O.num_params(H)).astype(np.float32)
    th[2 * H:2 * H + H * H] /= math.sqrt(H)
    return {"H": H, "lo": lo, "inv_range": inv, "theta": th}


def zigzag_model(H=64):
    """Layer-1 knots at (k + 1/2) / H; every layer-2 unit's slope alternates
    between +1 and -1 from one layer-1 interval to the next, around an offset
    that makes it change sign once inside every interval but the first: about
    1 + H * H pieces, more than the map kernel keeps in LDS."""
    th = np.zeros(O.num_params(H), np.float32)
    th[:H] = 1.0
    th[H:2 * H] = -(np.arange(H) + 0.5) / H
    W2 = np.empty((H, H), np.float32)
    W2[:, 0] = 1.0
    W2[:, 1:] = 2.0 * (-1.0) ** np.arange(1, H)
    th[2 * H:2 * H + H * H] = W2.ravel()
    th[2 * H + H * H:3 * H + H * H] = -1.0 / (2 * H) + (np.arange(H) - (H - 1) / 2) / (H * H * 4)
    th[3 * H + H * H:4 * H + H * H] = np.random.default_rng(5).uniform(-1, 1, H).astype(np.float32) / H
    th[-1] = 0.5
    return {"H": H, "lo": 0.0, "inv_range": 1.0, "theta": th}


def magnitude(model):
    H = model["H"]
    th = model["theta"].astype(np.float64)
    w1, b1 = th[:H], th[H:2 * H]
    W2 = th[2 * H:2 * H + H * H].reshape(H, H)
    b2, w3, b3 = th[2 * H + H * H:3 * H + H * H], th[3 * H + H * H:4 * H + H * H], th[-1]
    return abs(b3) + float(np.abs(w3) @ (np.abs(b2) + np.abs(W2) @ (np.abs(w1) + np.abs(b1))))


def pwl_params(**kw):
    return nn.sort_params(form=nn.FORM_PWL, **kw)


def check_F(x, model):
    """F of every key within the bound of the oracle's FP64 evaluation; the
    same keys unmapped.  Returns the largest error as a share of the bound."""
    _, F = nn.nnsort_predict(nn.model_from_dict(model), to_dev(x), pwl_params(), want_slots=False)
    got = F.cpu().numpy()
    xh, ok = O.translate(x, model["lo"], model["inv_range"])
    ref = O.eval_F(xh, model, O.FORM_FP64)
    assert np.array_equal(np.isnan(got), ~ok)
    bound = (4 * model["H"] + 16) * U64 * magnitude(model)
    d = np.abs(got[ok] - ref[ok])
    assert d.size == 0 or float(d.max()) <= bound, (float(d.max()), bound)
    return float(d.max()) / bound if d.size else 0.0


def check_sort_and_counts(x, model, eps=3):
    m = nn.model_from_dict(model)
    xd = to_dev(x)
    sp = pwl_params(tau=0, eps=eps, stats_level=1)
    out, st = nn.nnsort_sort_with_model(m, xd, sp=sp)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = got.view(np.uint64) if x.dtype == np.uint64 else got
    assert np.array_equal(np.ascontiguousarray(got).view(np.uint64), O.sort_reference(x).view(np.uint64))
    slots, _ = nn.nnsort_predict(m, xd, sp, want_F=False)
    s = slots.cpu().numpy().astype(np.int64)
    unm = int(np.count_nonzero(s == 0xFFFFFFFF))
    k = np.bincount(s[s != 0xFFFFFFFF]) if s.size > unm else np.zeros(1, np.int64)
    want = [int(np.maximum(0, k - r).sum()) + unm for r in range(1, eps + 1)]
    t = st["rounds"]
    assert st["collided"] == want[:t]
    # rounds stop early only once the conflict array is empty (tau = 0)
    assert t == eps or want[t - 1] == 0
    return st


# ---------------------------------------------------------------------------
# F against the direct FP64 evaluation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("H,seed", [(20, 1), (32, 2), (64, 3)])
def test_pwl_F_random_models(H, seed):
    x = np.random.default_rng(seed).random(300_001)
    r = check_F(x, random_model(H, seed))
    print(f"H {H}: max error {r:.3g} of the bound")


@pytest.mark.parametrize("name,H", [("gauss_mix", 64), ("lognormal", 32), ("zipf_u64", 64)])
def test_pwl_F_fitted_models(name, H):
    x = W.make(name, 400_000)
    model = O.fit(x, H=H, sample_frac=0.01, batch=4096, steps=20)
    r = check_F(x, model)
    print(f"{name}: max error {r:.3g} of the bound")


def test_pwl_F_many_pieces_and_edge_keys():
    """More pieces than LDS holds (the kernel reads them from global memory),
    on keys spread over [0, 1] and on the edge keys (signed zeros, denormals,
    extremes, infinities, NaNs)."""
    model = zigzag_model()
    x = np.concatenate([np.random.default_rng(8).random(200_000), np.linspace(0.0, 1.0, 4097), W.edge_keys()])
    check_F(x, model)
    check_F(W.edge_keys(), random_model(64, 4, lo=-2.0, inv=0.25))


# ---------------------------------------------------------------------------
# whole sorts
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,n,H", [("uniform", 500_000, 32), ("lognormal", 400_000, 32),
                                      ("gauss_mix", 300_007, 64), ("zipf_u64", 300_000, 64)])
def test_pwl_sort_exact_and_counts(name, n, H):
    x = W.make(name, n)
    model = O.fit(x, H=H, sample_frac=0.01, batch=4096, steps=5)
    check_sort_and_counts(x, model)


def test_pwl_sort_many_pieces():
    x = np.random.default_rng(9).random(200_003)
    check_sort_and_counts(x, zigzag_model())


def test_pwl_sort_edge_keys_and_tiny():
    model = random_model(32, 6, lo=-1.0, inv=0.5)
    for x in (W.edge_keys(), np.array([0.5]), np.array([2.0, 1.0])):
        check_sort_and_counts(x, model)


def test_pwl_same_output_as_other_forms():
    """The three forms give different slots but the same sorted output."""
    x = W.gauss_mix(250_000, seed=11)
    m = nn.model_from_dict(O.fit(x, H=64, sample_frac=0.01, batch=4096, steps=5))
    xd = to_dev(x)
    outs = []
    for form in (nn.FORM_FP32, nn.FORM_BF16, nn.FORM_PWL):
        out, _ = nn.nnsort_sort_with_model(m, xd, sp=nn.sort_params(form=form))
        outs.append(out.cpu().numpy().view(np.uint64))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
