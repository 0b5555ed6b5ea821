"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Sorted output: bit-exact.  Round counts |c_r| and stored keys per round: equal
(they depend only on the slots, and the FP32 form's slots are reproduced bit
for bit).  BF16 form: its slots are checked against an a-priori error bound
around the oracle's FP64 evaluation of the bf16-rounded model, and its round
counts against the slot-histogram identity.  Every input is seeded synthetic
data; models come from the oracle's fit or from closed forms.
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


def to_dev(x: np.ndarray):
    if x.dtype == np.float64:
        return torch.from_numpy(x.copy()).to(DEV)
    return torch.from_numpy(x.view(np.int64).copy()).to(DEV)


def to_host(t, like_dtype) -> np.ndarray:
    a = t.cpu().numpy()
    return a.view(np.uint64) if np.dtype(like_dtype) == np.uint64 else a


def bits(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a).view(np.uint64)


def assert_same_bits(got: np.ndarray, expect: np.ndarray):
    g, e = bits(got), bits(expect)
    assert g.shape == e.shape
    bad = np.nonzero(g != e)[0]
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"


def random_model(H, seed, lo=0.0, inv=1.0):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-1, 1, O.num_params(H)).astype(np.float32)
    th[2 * H:2 * H + H * H] /= math.sqrt(H)
    return {"H": H, "lo": lo, "inv_range": inv, "theta": th}


def gpu_sort(x, model, **kw):
    sp = nn.sort_params(stats_level=2, **kw)
    out, st = nn.nnsort_sort_with_model(nn.model_from_dict(model), to_dev(x), sp=sp)
    torch.cuda.synchronize()
    return to_host(out, x.dtype), st


# ---------------------------------------------------------------------------
# FP32 form: slots reproduced bit for bit
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,n,H", [("uniform", 1_000_000, 32), ("lognormal", 300_001, 32),
                                      ("gauss_mix", 200_003, 64), ("zipf_u64", 100_000, 64)])
def test_fp32_slots_bit_exact(name, n, H):
    x = W.make(name, n)
    model = O.fit(x, H=H, sample_frac=0.01, batch=4096, steps=5)
    slots, F = nn.nnsort_predict(nn.model_from_dict(model), to_dev(x), nn.sort_params())
    s_gpu = slots.cpu().numpy().astype(np.uint32)
    s_orc = O.predict_slots(x, model, form=O.FORM_FP32C)
    assert np.array_equal(s_gpu, s_orc), np.count_nonzero(s_gpu != s_orc)
    xh, ok = O.translate(x, model["lo"], model["inv_range"])
    F_orc = O.eval_F(xh, model, O.FORM_FP32C)
    assert np.array_equal(F.cpu().numpy()[ok], F_orc[ok])


def test_fp32_slots_random_weights_and_edge_keys():
    x = np.concatenate([W.edge_keys(), W.gauss_mix(5000, seed=9) * 1e-3])
    for H, seed in ((32, 1), (64, 2), (20, 3)):
        model = random_model(H, seed, lo=-2.0, inv=0.25)
        slots, _ = nn.nnsort_predict(nn.model_from_dict(model), to_dev(x), nn.sort_params())
        assert np.array_equal(slots.cpu().numpy().astype(np.uint32), O.predict_slots(x, model))


# ---------------------------------------------------------------------------
# full procedure, FP32 form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,n,H", [("uniform", 1_000_000, 32), ("lognormal", 500_000, 32),
                                      ("gauss_mix", 300_000, 64), ("zipf_u64", 300_000, 64),
                                      ("piecewise_uniform", 400_000, 32)])
def test_sort_matches_oracle(name, n, H):
    x = W.make(name, n)
    model = O.fit(x, H=H, sample_frac=0.01, batch=4096, steps=5)
    out, st = gpu_sort(x, model)
    ref, ost = O.nnsort(x, model)
    assert_same_bits(out, ref)
    assert st["rounds"] == ost["rounds"]
    assert st["collided"] == ost["collided"]
    assert st["placed"] == ost["placed"]
    assert st["residue"] == ost["residue"]
    if st["fallback"] == 0:
        assert st["boundary_keys"] < n


@pytest.mark.parametrize("n", [0, 1, 2, 100, 1024, 1025, 2049, 4097, 65_537, 131_071])
def test_sort_ragged_sizes(n):
    x = W.lognormal(n, seed=n)
    model = O.fit(x, H=32, sample_frac=0.5, batch=256, steps=2) if n else random_model(32, 0)
    out, st = gpu_sort(x, model)
    ref, ost = O.nnsort(x, model)
    assert_same_bits(out, ref)
    assert st["rounds"] == ost["rounds"] and st["collided"] == ost["collided"]


def test_sort_edge_keys_and_tau_zero():
    x = np.concatenate([W.edge_keys(seed=s) for s in range(20)])
    model = random_model(32, 4, lo=-3.0, inv=1 / 6.0)
    for eps, tau in ((1, 0), (3, 0), (8, 10)):
        out, st = gpu_sort(x, model, eps=eps, tau=tau)
        ref, ost = O.nnsort(x, model, eps=eps, tau=tau)
        assert_same_bits(out, ref)
        assert st["collided"] == ost["collided"] and st["unmapped"] > 0


# ---------------------------------------------------------------------------
# closed-form slots through nnsort_sort_with_slots
# ---------------------------------------------------------------------------
def gpu_sort_slots(x, slots, **kw):
    sp = nn.sort_params(**kw)
    out, st = nn.nnsort_sort_with_slots(torch.from_numpy(slots.astype(np.int64)).to(DEV), to_dev(x), sp=sp)
    torch.cuda.synchronize()
    return to_host(out, x.dtype), st


def test_constant_slot_worst_case():
    """Every key in one slot: the densest range goes through the residue path
    and each round stores one key (|c_r| = n - r)."""
    x = W.uniform(300_000, seed=1)
    slots = np.full(x.size, 12345, np.uint32)
    out, st = gpu_sort_slots(x, slots, eps=5, tau=0)
    assert_same_bits(out, np.sort(x))
    assert st["collided"] == [x.size - r for r in range(1, 6)]
    assert st["big_buckets"] == 1


def test_perfect_rank_and_reversed_slots():
    x = W.uniform(400_000, seed=2)
    rank = np.empty(x.size, np.int64)
    rank[np.argsort(x)] = np.arange(x.size)
    for F in (rank / x.size, (x.size - 1 - rank) / x.size):
        slots = O.slots_from_F(F, 1.25 * x.size)
        out, st = gpu_sort_slots(x, slots, tau=0)
        ref, ost = O.nnsort(x, {"H": 1, "lo": 0, "inv_range": 1, "theta": np.zeros(6, np.float32)}, slots=slots,
                            tau=0)
        assert_same_bits(out, ref)
        # nothing collides, so count(w) = 0 <= tau ends the loop after round 1
        assert st["collided"] == ost["collided"] == [0]


def test_duplicate_groups_closed_form():
    rng = np.random.default_rng(5)
    vals = rng.permutation(40_000).astype(np.float64)
    g = rng.integers(1, 9, vals.size)
    x = rng.permutation(np.repeat(vals, g))
    vrank = np.searchsorted(np.sort(vals), x)
    slots = O.slots_from_F(vrank / vals.size, 1.25 * x.size)
    out, st = gpu_sort_slots(x, slots, eps=4, tau=0)
    assert_same_bits(out, np.sort(x))
    k = np.bincount(slots.astype(np.int64))
    assert st["collided"] == [int(np.maximum(0, k - r).sum()) for r in range(1, 5)]


def test_bad_slot_rejected():
    x = W.uniform(5000, seed=3)
    slots = np.zeros(x.size, np.uint32)
    slots[7] = 10 ** 6   # beyond S
    with pytest.raises(nn.NNSortError):
        gpu_sort_slots(x, slots, tau=0)


# ---------------------------------------------------------------------------
# BF16 form
# ---------------------------------------------------------------------------
def _mag_bf16(model, x):
    H = model["H"]
    th = model["theta"].astype(np.float64)
    w1, b1 = th[:H], th[H:2 * H]
    W2 = np.array([O.round_bf16(v) for v in th[2 * H:2 * H + H * H]]).reshape(H, H)
    b2, w3, b3 = th[2 * H + H * H:3 * H + H * H], th[3 * H + H * H:4 * H + H * H], th[-1]
    a1 = np.abs(w1)[None, :] * np.abs(x)[:, None] + np.abs(b1)[None, :]
    a2 = np.abs(b2)[None, :] + a1 @ np.abs(W2).T
    return np.abs(b3) + a2 @ np.abs(w3)


@pytest.mark.parametrize("H", [32, 64])
def test_bf16_F_within_bound(H):
    """F of the BF16 form vs the FP64 evaluation of the same model with W2
    rounded to bf16: the three-term split is exact, so the difference is FP32
    accumulation only, |dF| <= 2 gamma_{3H+8} * (sum of |terms|)."""
    x = W.gauss_mix(100_000, seed=4)
    model = O.fit(x, H=H, sample_frac=0.05, batch=4096, steps=3)
    sp = nn.sort_params(form=nn.FORM_BF16, bf16_terms=3)
    _, F = nn.nnsort_predict(nn.model_from_dict(model), to_dev(x), sp)
    xh, ok = O.translate(x, model["lo"], model["inv_range"])
    ref = O.eval_F(xh, model, O.FORM_BF16W)
    u = 2.0 ** -24
    k = 3 * H + 8
    bound = 2 * k * u / (1 - k * u) * _mag_bf16(model, xh)
    d = np.abs(F.cpu().numpy() - ref)
    assert np.all(d[ok] <= bound[ok] + 1e-300), float(np.max(d[ok] / bound[ok]))


def test_bf16_scaled_operands_change_no_bit():
    """The BF16 form runs on power-of-two-scaled operands (relu as a clamp to
    [0, 1]) when every scaled operand is exact, and on the unscaled ones with
    an explicit relu otherwise.  Scaling commutes with rounding, so both give
    the same F bit for bit.  Model 2 differs from model 1 only in a hidden-2
    row whose output weight is 0 (it adds an exact 0 to F) and whose tiny
    W2 entry cannot be scaled exactly, which forces the unscaled kernel."""
    x = W.gauss_mix(200_000, seed=8)
    H = 64
    m1 = O.fit(x, H=H, sample_frac=0.01, steps=0)
    th = m1["theta"].copy()
    iW2, iw3 = 2 * H, 3 * H + H * H
    th[iw3 + H - 1] = 0.0
    m1 = dict(m1, theta=th)
    th2 = th.copy()
    th2[iW2 + (H - 1) * H + 0] = 1e-37
    th2[iW2 + (H - 1) * H + 1] = 1.0
    m2 = dict(m1, theta=th2)
    sp = nn.sort_params(form=nn.FORM_BF16, bf16_terms=3)
    xd = to_dev(x)
    _, F1 = nn.nnsort_predict(nn.model_from_dict(m1), xd, sp)
    _, F2 = nn.nnsort_predict(nn.model_from_dict(m2), xd, sp)
    assert_same_bits(F1.cpu().numpy(), F2.cpu().numpy())


@pytest.mark.parametrize("name,H", [("gauss_mix", 64), ("lognormal", 32)])
def test_bf16_slots_track_fp32_on_ramp_model(name, H):
    """On a ramp model (W2 = -I is exact in bf16, output weights all different)
    the three-term BF16 form must give the FP32 form's slots up to rounding:
    nearly all equal, none more than one slot away, and the same round counts
    to within 0.1% of n."""
    n = 1_000_000
    x = W.make(name, n)
    model = O.fit(x, H=H, sample_frac=0.01, steps=0)
    m = nn.model_from_dict(model)
    xd = to_dev(x)
    s32, _ = nn.nnsort_predict(m, xd, nn.sort_params(form=nn.FORM_FP32))
    s16, _ = nn.nnsort_predict(m, xd, nn.sort_params(form=nn.FORM_BF16, bf16_terms=3))
    a = s32.cpu().numpy().astype(np.int64)
    b = s16.cpu().numpy().astype(np.int64)
    assert np.mean(a == b) > 0.999
    # W2 = -I is exact in bf16 and the split activations are exact, so the two
    # forms differ only in how the output sum is rounded (Dot2 in FP32 against
    # FP64 accumulation): a slot can move only across a rounding boundary
    assert np.max(np.abs(a - b)) <= 1
    _, st32 = nn.nnsort_sort_with_model(m, xd, sp=nn.sort_params(form=nn.FORM_FP32))
    _, st16 = nn.nnsort_sort_with_model(m, xd, sp=nn.sort_params(form=nn.FORM_BF16))
    for c32, c16 in zip(st32["collided"], st16["collided"]):
        assert abs(c32 - c16) <= n // 1000


@pytest.mark.parametrize("terms", [1, 2, 3])
def test_bf16_sort_exact_and_counts(terms):
    x = W.gauss_mix(400_000, seed=6)
    model = O.fit(x, H=64, sample_frac=0.01, batch=4096, steps=3)
    m = nn.model_from_dict(model)
    sp = nn.sort_params(form=nn.FORM_BF16, bf16_terms=terms, tau=0, stats_level=1)
    xd = to_dev(x)
    out, st = nn.nnsort_sort_with_model(m, xd, sp=sp)
    assert_same_bits(to_host(out, x.dtype), O.sort_reference(x))
    slots, _ = nn.nnsort_predict(m, xd, sp)
    s = slots.cpu().numpy().astype(np.int64)
    k = np.bincount(s[s != 0xFFFFFFFF])
    assert st["collided"] == [int(np.maximum(0, k - r).sum()) for r in range(1, 4)]


@pytest.mark.parametrize("n", [2, 63, 64, 65, 2047, 2048, 2049, 6143, 6145])
def test_bf16_sort_tile_edges(n):
    """The BF16 map kernel counts the first partition pass's digits per
    2048-key tile itself: sizes around a 64-key block and a tile, with the
    round-count shortcut off (tau 0), sort exactly with the oracle's counts."""
    x = W.gauss_mix(n, seed=40 + n % 7)
    model = O.fit(W.gauss_mix(20_000, seed=5), H=64, sample_frac=0.05, batch=512, steps=2)
    m = nn.model_from_dict(model)
    sp = nn.sort_params(form=nn.FORM_BF16, tau=0, stats_level=1)
    xd = to_dev(x)
    out, st = nn.nnsort_sort_with_model(m, xd, sp=sp)
    assert_same_bits(to_host(out, x.dtype), O.sort_reference(x))
    slots, _ = nn.nnsort_predict(m, xd, sp)
    s = slots.cpu().numpy().astype(np.int64)
    k = np.bincount(s[s != 0xFFFFFFFF])
    want = [int(np.maximum(0, k - r).sum()) for r in range(1, 4)]
    # with tau 0 the rounds stop after the first one that leaves no conflict
    rounds = next((i + 1 for i, c in enumerate(want) if c == 0), 3)
    assert st["rounds"] == rounds and st["collided"] == want[:rounds]


# ---------------------------------------------------------------------------
# determinism, radix sort, fit, gradients, errors
# ---------------------------------------------------------------------------
def test_repeat_runs_identical():
    x = W.lognormal(600_000, seed=12)
    model = O.fit(x, H=32, sample_frac=0.01, batch=4096, steps=3)
    a, sa = gpu_sort(x, model)
    b, sb = gpu_sort(x, model)
    assert_same_bits(a, b)
    for k in ("collided", "placed", "residue", "boundary_keys"):
        assert sa[k] == sb[k]


def test_concurrent_sorts_from_two_threads():
    """Two host threads sort different inputs at once, each on its own stream
    and workspace, several times over: every output is exact and the counts
    are those of a sort run alone (each thread reads its counters back through
    its own pinned buffer)."""
    import threading
    xs = [W.lognormal(700_001, seed=31), W.gauss_mix(500_003, seed=32)]
    models = [O.fit(x, H=32 if i == 0 else 64, sample_frac=0.01, batch=4096, steps=3) for i, x in enumerate(xs)]
    alone = [gpu_sort(x, m, form=nn.FORM_BF16) for x, m in zip(xs, models)]
    sp = nn.sort_params(form=nn.FORM_BF16, stats_level=1)
    keys = [to_dev(x) for x in xs]
    outs = [torch.empty_like(k) for k in keys]
    wss = [nn.alloc_workspace(nn.workspace_size(k.numel(), nn.F64, sp), keys[0].device) for k in keys]
    ms = [nn.model_from_dict(m) for m in models]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    stats = [[], []]
    errors = []

    def run(i):
        try:
            for _ in range(6):
                _, st = nn.nnsort_sort_with_model(ms[i], keys[i], out=outs[i], sp=sp, ws=wss[i], stream=streams[i])
                stats[i].append(st)
        except Exception as e:  # reported in the main thread
            errors.append(e)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, x in enumerate(xs):
        assert_same_bits(to_host(outs[i], x.dtype), O.sort_reference(x))
        assert_same_bits(to_host(outs[i], x.dtype), alone[i][0])
        for st in stats[i]:
            for k in ("rounds", "collided", "placed", "residue"):
                assert st[k] == alone[i][1][k], (i, k)


@pytest.mark.parametrize("name,n", [("uniform", 1), ("lognormal", 4095), ("gauss_mix", 4097),
                                    ("zipf_u64", 1_000_003), ("uniform", 2_000_000)])
def test_radix_sort(name, n):
    x = W.make(name, n)
    out = nn.nnsort_radix_sort(to_dev(x))
    assert_same_bits(to_host(out, x.dtype), O.sort_reference(x))


def test_radix_sort_edge_keys():
    x = np.concatenate([W.edge_keys(seed=s) for s in range(50)])
    out = nn.nnsort_radix_sort(to_dev(x))
    assert_same_bits(to_host(out, x.dtype), O.sort_reference(x))


@pytest.mark.parametrize("init,H", [(1, 32), (0, 16), (1, 64)])
def test_fit_init_matches_oracle(init, H):
    """Same Philox sample and initialisation: identical weights at step 0."""
    x = W.lognormal(200_000, seed=5)
    fp = nn.fit_params(hidden=H, sample_frac=0.05, steps=0, init=init, seed=77)
    m = nn.nnsort_fit(to_dev(x), fp)
    got = nn.model_to_dict(m)
    ref = O.fit(x, H=H, sample_frac=0.05, steps=0, init=init, seed=77)
    assert got["lo"] == ref["lo"] and got["inv_range"] == ref["inv_range"]
    assert np.array_equal(got["theta"], ref["theta"])


@pytest.mark.parametrize("name", ["zipf_u64", "gauss_mix"])
def test_fit_init_greedy_knots_large_sample(name):
    """Greedy knots over a 10^5-point sample (the scan spread over many
    workgroups; zipf has long runs of equal keys, hence zero-width pieces):
    identical weights at step 0."""
    x = W.make(name, 1_000_000)
    fp = nn.fit_params(hidden=64, sample_frac=0.1, steps=0, init=1, seed=5)
    got = nn.model_to_dict(nn.nnsort_fit(to_dev(x), fp))
    ref = O.fit(x, H=64, sample_frac=0.1, steps=0, init=1, seed=5)
    assert got["lo"] == ref["lo"] and got["inv_range"] == ref["inv_range"]
    assert np.array_equal(got["theta"], ref["theta"])


def test_fit_loss_tracks_oracle():
    x = W.uniform(100_000, seed=8)
    fp = nn.fit_params(hidden=16, sample_frac=0.2, batch=2048, steps=30, init=0, lr=1e-2, seed=3)
    m, hist = nn.nnsort_fit(to_dev(x), fp, history=True)
    ref, rhist = O.fit(x, H=16, sample_frac=0.2, batch=2048, steps=30, init=0, lr=1e-2, seed=3,
                       return_history=True)
    assert abs(hist[0] - rhist[0]) <= 1e-5 * max(1.0, rhist[0])
    assert hist[-1] < 0.5 * hist[0]
    assert abs(hist[-1] - rhist[-1]) <= 0.05 * rhist[-1] + 1e-6


def test_default_fit_recipe_matches_oracle():
    """The default fit (H 64, 1% sample, 200 Adam steps on batches of 65,536,
    ramp start, keep the lowest batch loss unless it is more disordered than
    the start) on the device and in the oracle: the batch loss of every step
    within FP32 evaluation error of the oracle's FP64 loss, the same lo and
    inv_range, and the two chosen models' slots within one slot of each other
    on a sample of keys."""
    x = W.gauss_mix(1_000_000, seed=13)
    _, fp = nn.default_params()
    fp.hidden = 64
    m, hist = nn.nnsort_fit(to_dev(x), fp, history=True)
    ref, rhist = O.fit(x, H=64, sample_frac=fp.sample_frac, batch=fp.batch, steps=fp.steps, lr=fp.lr,
                       seed=fp.seed, init=fp.init, loss=fp.loss, return_history=True)
    assert len(hist) == len(rhist) == 200
    h, r = np.array(hist), np.array(rhist)
    assert np.all(np.abs(h - r) <= 1e-3 * r + 1e-12), float(np.max(np.abs(h - r) / r))
    got = nn.model_to_dict(m)
    assert got["lo"] == ref["lo"] and got["inv_range"] == ref["inv_range"]
    xs = x[np.random.default_rng(3).choice(x.size, 100_000, replace=False)]
    M = 1.25 * x.size
    xh, ok = O.translate(xs, got["lo"], got["inv_range"])
    a = O.slots_from_F(O.eval_F(xh, got, O.FORM_FP32C), M).astype(np.int64)
    b = O.slots_from_F(O.eval_F(xh, ref, O.FORM_FP32C), M).astype(np.int64)
    assert np.max(np.abs(a - b)[ok]) <= 1


@pytest.mark.parametrize("H,loss", [(8, 0), (32, 0), (64, 0), (32, 1)])
def test_gradient_vs_fp64_reference(H, loss):
    rng = np.random.default_rng(H)
    model = random_model(H, 10 + H)
    th = torch.from_numpy(model["theta"]).to(DEV)
    B = 3000
    x = rng.random(B)
    y = rng.random(B)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.from_numpy(y.astype(np.float32)).to(DEV)
    saved = torch.empty(B * 2 * H, dtype=torch.float32, device=DEV)
    F = nn.nnsort_mlp_forward(H, th, xd, saved)
    L, gF = nn.nnsort_loss_grad(F, yd, loss=loss, delta=0.3)
    g = nn.nnsort_mlp_backward(H, th, xd, saved, gF).cpu().numpy().astype(np.float64)
    Lr, gr = O.loss_grad(model["theta"].astype(np.float64), H, x, y.astype(np.float32).astype(np.float64), loss,
                         0.3)
    assert abs(float(L.item()) - Lr) <= 1e-5 * max(1.0, Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)


@pytest.mark.parametrize("H,loss,B", [(32, 0, 3000), (64, 0, 3000), (64, 1, 4096), (64, 0, 65536),
                                       (64, 0, 200_003), (32, 1, 100_001)])
def test_fit_step_gradient_vs_fp64_reference(H, loss, B):
    """The fit's own step for widths 32 and 64 (one fused kernel on the FP32
    matrix cores): the batch it draws from the sample (Philox, stream 3) is
    the oracle's, and its loss and gradient match the oracle's FP64 ones on
    that batch.  Batches past 65,536 entries give each wave several tiles in
    turn (the next tile's entries are fetched while one is processed), with a
    ragged last round."""
    rng = np.random.default_rng(H + B)
    model = random_model(H, 20 + H)
    th = torch.from_numpy(model["theta"]).to(DEV)
    k = 5000
    x = np.sort(rng.random(k))
    y = ((np.arange(k) + 0.5) / k).astype(np.float32)
    seed, step = 17, 5
    L, g = nn.nnsort_fit_gradient(H, th, torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV), B, seed, step,
                                  loss=loss, delta=0.05)
    g = g.cpu().numpy().astype(np.float64)
    bi = O.batch_indices(seed, step, k, B)
    Lr, gr = O.loss_grad(model["theta"].astype(np.float64), H, x[bi], y[bi].astype(np.float64), loss, 0.05)
    assert abs(float(L.item()) - Lr) <= 1e-5 * max(1.0, Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr), np.linalg.norm(g - gr) / np.linalg.norm(gr)


@pytest.mark.parametrize("H", [32, 64])
def test_fit_mfma_loss_tracks_oracle(H):
    """A fit that moves (uniform start, lr 1e-2, 30 steps) through the fused
    step: the first batch loss matches the oracle's to FP32 rounding, the loss
    halves, and the last loss stays close to the oracle's FP64 fit."""
    x = W.uniform(100_000, seed=8)
    fp = nn.fit_params(hidden=H, sample_frac=0.2, batch=2048, steps=30, init=0, lr=1e-2, seed=3)
    m, hist = nn.nnsort_fit(to_dev(x), fp, history=True)
    ref, rhist = O.fit(x, H=H, sample_frac=0.2, batch=2048, steps=30, init=0, lr=1e-2, seed=3,
                       return_history=True)
    assert abs(hist[0] - rhist[0]) <= 1e-5 * max(1.0, rhist[0])
    assert hist[-1] < 0.5 * hist[0]
    assert abs(hist[-1] - rhist[-1]) <= 0.05 * rhist[-1] + 1e-6


def test_gradient_vs_finite_differences_through_autograd():
    """torch.autograd through NNSortMLPFn; compared with central differences of
    the FP64 loss of the oracle on parameters away from ReLU kinks."""
    H = 16
    rng = np.random.default_rng(1)
    model = random_model(H, 31)
    x = rng.random(512)
    y = rng.random(512)
    th = torch.from_numpy(model["theta"]).to(DEV).requires_grad_(True)
    F = nn.mlp(torch.from_numpy(x).to(DEV), th, H)
    L = ((F.double() - torch.from_numpy(y).to(DEV)) ** 2).mean()
    L.backward()
    g = th.grad.cpu().numpy().astype(np.float64)
    t64 = model["theta"].astype(np.float64)
    checked = 0
    for p in range(t64.size):
        h = 1e-6 * max(1.0, abs(t64[p]))
        tp, tm = t64.copy(), t64.copy()
        tp[p] += h
        tm[p] -= h
        L0 = O.loss_value(t64, H, x, y)
        Lp, Lm = O.loss_value(tp, H, x, y), O.loss_value(tm, H, x, y)
        if abs((Lp - L0) - (L0 - Lm)) > 1e-4 * max(abs(Lp - L0), 1e-12):
            continue
        cd = (Lp - Lm) / (2 * h)
        assert abs(cd - g[p]) <= 1e-4 * max(1e-3, abs(cd)) + 1e-6, (p, cd, g[p])
        checked += 1
    assert checked > 0.7 * t64.size


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(2)
    P = 1000
    th = rng.standard_normal(P).astype(np.float32)
    g = rng.standard_normal(P).astype(np.float32)
    d = {k: torch.from_numpy(v.copy()).to(DEV) for k, v in (("th", th), ("g", g))}
    m1 = torch.zeros(P, dtype=torch.float32, device=DEV)
    m2 = torch.zeros(P, dtype=torch.float32, device=DEV)
    t64, m64, v64 = th.astype(np.float64), np.zeros(P), np.zeros(P)
    for t in range(1, 4):
        nn.nnsort_adam_step(d["th"], d["g"], m1, m2, t, lr=1e-3)
        O.adam_step(t64, g.astype(np.float64), m64, v64, t, lr=1e-3)
    assert np.allclose(d["th"].cpu().numpy(), t64, rtol=0, atol=1e-6)


def test_errors_reported():
    x = to_dev(W.uniform(5000, seed=1))
    m = nn.model_from_dict(random_model(32, 1))
    with pytest.raises(nn.NNSortError):
        nn.nnsort_sort_with_model(m, x, out=x)            # in place is rejected
    with pytest.raises(nn.NNSortError):
        nn.nnsort_sort_with_model(m, x, ws=nn.alloc_workspace(1024))
    with pytest.raises(nn.NNSortError):
        nn.nnsort_sort_with_model(m, x, sp=nn.sort_params(eps=9))


# ---------------------------------------------------------------------------
# the procedure's parameters (m, eps, tau), and a model that does not fit the
# data (Sec. 4, Exp-3 and Exp-4)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,eps,tau", [(1.0, 1, 1024), (1.0, 3, 0), (1.5, 2, 1024), (2.0, 5, 1024),
                                       (1.25, 1, 0), (3.0, 8, 100_000)])
def test_sort_parameters_match_oracle(m, eps, tau):
    x = W.lognormal(300_000, seed=21)
    model = O.fit(x, H=32, sample_frac=0.01, batch=4096, steps=5)
    out, st = gpu_sort(x, model, m=m, eps=eps, tau=tau)
    ref, ost = O.nnsort(x, model, m=m, eps=eps, tau=tau)
    assert_same_bits(out, ref)
    for k in ("rounds", "collided", "placed", "residue"):
        assert st[k] == ost[k], (k, st[k], ost[k])


@pytest.mark.parametrize("noise", [0.0, 0.1, 0.5])
def test_model_fitted_on_other_data(noise):
    """A model fitted on uniform keys sorts uniform + normal mixes exactly;
    only the conflict counts grow with the mismatch."""
    fit_x = W.uniform(200_000, seed=3)
    model = O.fit(fit_x, H=32, sample_frac=0.05, batch=4096, steps=5)
    x = W.noisy_uniform(250_000, noise, seed=9)
    out, st = gpu_sort(x, model)
    ref, ost = O.nnsort(x, model)
    assert_same_bits(out, ref)
    for k in ("rounds", "collided", "placed", "residue"):
        assert st[k] == ost[k], (k, st[k], ost[k])


def test_models_alternating_on_one_thread():
    """The library prepares each model's device form on the host and keeps the
    last one per thread, reusing it when the next model has the same bytes.
    Sorts that alternate between two models, and one whose weight is changed
    in place in the same C struct, must each see their own model: every
    call's round counts equal the oracle's for the model of that call."""
    x = W.gauss_mix(150_003, seed=4)
    mA = O.fit(x, H=32, sample_frac=0.02, batch=4096, steps=3)
    mB = O.fit(x, H=32, sample_frac=0.05, batch=4096, steps=3, seed=7)
    refs = {}
    for name, md in (("A", mA), ("B", mB)):
        ref, ost = O.nnsort(x, md)
        refs[name] = (ref, ost)
    assert refs["A"][1]["collided"] != refs["B"][1]["collided"], "the two models must differ in their counts"
    keys = to_dev(x)
    sp = nn.sort_params(stats_level=1)
    cA, cB = nn.model_from_dict(mA), nn.model_from_dict(mB)
    for name, cm in (("A", cA), ("B", cB), ("A", cA), ("B", cB)):
        out, st = nn.nnsort_sort_with_model(cm, keys, sp=sp)
        torch.cuda.synchronize()
        ref, ost = refs[name]
        assert_same_bits(to_host(out, x.dtype), ref)
        assert st["collided"] == ost["collided"], (name, st["collided"], ost["collided"])
    # one weight changed in place: same struct, new bytes
    mC = dict(mA, theta=mA["theta"].copy())
    mC["theta"][5] = np.float32(mC["theta"][5] * 1.5)  # w1 of hidden unit 5
    cA.w1[5] = float(mC["theta"][5])
    ref, ost = O.nnsort(x, mC)
    out, st = nn.nnsort_sort_with_model(cA, keys, sp=sp)
    torch.cuda.synchronize()
    assert_same_bits(to_host(out, x.dtype), ref)
    assert st["collided"] == ost["collided"], (st["collided"], ost["collided"])


@pytest.mark.parametrize("batch,delta", [(128, 0.01), (4096, 0.05)])
def test_huber_fit_tracks_oracle(batch, delta):
    """The paper's training recipe (Sec. 4.1, Eq. (loss)): Huber loss, small
    batches.  Same Philox sample, initial weights and batches on both sides:
    the first loss agrees to FP32 rounding, both fits lower the loss, and the
    final losses stay close."""
    x = W.uniform(100_000, seed=8)
    kw = dict(sample_frac=0.2, batch=batch, steps=40, init=0, lr=1e-2, seed=3, loss=1, delta=delta)
    fp = nn.fit_params(hidden=16, sample_frac=kw["sample_frac"], batch=batch, steps=kw["steps"], init=0,
                       lr=kw["lr"], seed=3, loss=1, huber_delta=delta)
    m, hist = nn.nnsort_fit(to_dev(x), fp, history=True)
    ref, rhist = O.fit(x, H=16, return_history=True, **kw)
    assert abs(hist[0] - rhist[0]) <= 1e-5 * max(1.0, rhist[0])
    assert hist[-1] < 0.7 * hist[0] and rhist[-1] < 0.7 * rhist[0]
    assert abs(hist[-1] - rhist[-1]) <= 0.1 * rhist[-1] + 1e-7


# ---------------------------------------------------------------------------
# a model with a non-finite parameter maps no key
# ---------------------------------------------------------------------------
def _nonfinite_models(H=32):
    base = random_model(H, 31)
    out = []
    for where, val in (("w1", np.nan), ("W2", np.nan), ("w3", np.inf), ("b3", -np.inf)):
        th = base["theta"].copy()
        idx = {"w1": 3, "W2": 2 * H + 5 * H + 7, "w3": 3 * H + H * H + 2, "b3": -1}[where]
        th[idx] = val
        out.append((where, dict(base, theta=th)))
    out.append(("lo", dict(base, lo=np.nan)))
    return out


@pytest.mark.parametrize("form", [nn.FORM_FP32, nn.FORM_BF16, nn.FORM_PWL])
def test_nonfinite_model_sends_every_key_to_the_residue(form):
    """Every key of a sort with a non-finite model takes the conventional
    path: no key is placed, every round's conflict array holds all n keys, the
    output is still the exact sorted array, and the slot map reports no slot
    and F = NaN for every key (the oracle's rule for such models)."""
    x = W.gauss_mix(70_001, seed=9)
    xd = to_dev(x)
    for where, model in _nonfinite_models():
        m = nn.model_from_dict(model)
        sp = nn.sort_params(form=form, stats_level=2)
        out, st = nn.nnsort_sort_with_model(m, xd, sp=sp)
        assert_same_bits(to_host(out, x.dtype), O.sort_reference(x))
        ref, ost = O.nnsort(x, model)
        assert st["unmapped"] == x.size, where
        assert st["collided"] == ost["collided"] == [x.size] * 3, where
        assert st["placed"] == [0, 0, 0], where
        slots, F = nn.nnsort_predict(m, xd, sp)
        assert np.all(slots.cpu().numpy() == 0xFFFFFFFF), where
        assert np.all(np.isnan(F.cpu().numpy())), where
