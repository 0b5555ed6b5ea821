"""Every branch of the range polish and of the boundary fix-up, driven through
caller-given slots (the sorting phase of Sec. 2 takes any slot per key; the
output is the sorted input whatever the slots are, and the round counts depend
on the slots only).  Each case compares the output bit for bit and the round
counts with the oracle on the same slots, checks a precondition on the slots
(on the host) that puts the intended branch in play, and reads the stats that
show the branch ran:
  - slots jittered by one: descents inside ranges (tile repair) and overlaps
    between neighbouring ranges (zone merges);
  - slots shuffled inside each range: the whole-range re-sort;
  - slot groups larger than the group-rank limit;
  - ranges of up to half the LDS capacity, of up to all of it, and denser
    ones (residue path) side by side;
  - slots scrambled across ranges: the full-sort fallback;
  - ranges whose key sets are out of value order, and keys without a slot
    that are not the extremes: overlaps the neighbour merges cannot settle;
  - NaNs, infinities, signed zeros and subnormals in dense and small ranges;
  - the model path with dense ranges and keys without a slot sharing the
    residue path.
"""
import numpy as np
import pytest

import oracle as O
import paper_1907_08817_amd as nn
from paper_1907_08817_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
UNM = 0xFFFFFFFF
RANGE_SLOTS = 2048          # slots per range
HALF, CAP = 2048, 4096      # LDS capacities of the two polish variants
DUMMY = {"H": 1, "lo": 0.0, "inv_range": 1.0, "theta": np.zeros(O.num_params(1), np.float32)}


def to_dev(x):
    return torch.from_numpy(x.copy() if x.dtype == np.float64 else x.view(np.int64).copy()).to(DEV)


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def ranks(x):
    """Position of each key in the sorted input (totalOrder, ties by index)."""
    r = np.empty(x.size, np.int64)
    r[np.argsort(O.order_keys(x), kind="stable")] = np.arange(x.size)
    return r


def rank_slots(x, m=1.25):
    return O.slots_from_F(ranks(x) / x.size, m * x.size).astype(np.int64)


def range_counts(s):
    s = np.asarray(s, np.int64)
    return np.bincount(s[s != UNM] >> 11)


def sort_slots(x, s, **kw):
    """GPU sort from slots s, checked against the oracle on the same slots;
    returns the GPU stats."""
    s = np.asarray(s, np.int64)
    sp = nn.sort_params(**kw)
    out, st = nn.nnsort_sort_with_slots(torch.from_numpy(s).to(DEV), to_dev(x), sp=sp)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref, ost = O.nnsort(x, DUMMY, slots=s.astype(np.uint32), **kw)
    bad = np.nonzero(bits(got) != bits(ref))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    for k in ("rounds", "collided", "placed", "residue"):
        assert st[k] == ost[k], (k, st[k], ost[k])
    return st


# ---------------------------------------------------------------------------
# polish inside a range
# ---------------------------------------------------------------------------
def test_jitter_of_one_slot():
    x = W.uniform(400_000, seed=21)
    S = O.num_slots(x.size)
    s = np.clip(rank_slots(x) + np.random.default_rng(1).integers(-1, 2, x.size), 0, S - 1)
    assert range_counts(s).max() <= HALF
    st = sort_slots(x, s)
    assert st["fallback"] == 0 and st["boundary_keys"] > 0
    assert st["range_resorts"] == 0      # tile merges settle displacements of a few keys


def test_shuffle_inside_ranges():
    x = W.lognormal(300_000, seed=22)
    S = O.num_slots(x.size)
    s = rank_slots(x)
    s = np.minimum((s & ~(RANGE_SLOTS - 1)) | np.random.default_rng(2).integers(0, RANGE_SLOTS, x.size), S - 1)
    cnt = range_counts(s)
    assert cnt.max() <= HALF
    st = sort_slots(x, s, eps=4)
    # key sets of the ranges are still in value order: no boundary work
    assert st["fallback"] == 0 and st["boundary_keys"] == 0
    assert st["range_resorts"] >= np.count_nonzero(cnt > 64) - 1


@pytest.mark.parametrize("group", [32, 33, 200, 2000])
def test_large_slot_groups(group):
    x = W.gauss_mix(200_000, seed=23)
    s = rank_slots(x)
    r = ranks(x)
    rng = np.random.default_rng(group)
    for r0 in rng.choice(x.size - group, 20, replace=False):
        sel = (r >= r0) & (r < r0 + group)
        s[sel] = s[r == r0][0]
    st = sort_slots(x, s, eps=5, tau=0)
    assert st["fallback"] == 0


# ---------------------------------------------------------------------------
# the two LDS variants and the residue path side by side
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("jitter", [0, 1])
def test_density_mix(jitter):
    x = W.gauss_mix(600_000, seed=24)
    n = x.size
    r = ranks(x).astype(np.float64)
    a, b = n // 3, 2 * n // 3
    # keys per slot: 0.8 (ranges of ~1640 keys), 1.7 (~3480), 2.5 (~5120)
    g = np.where(r < a, 1.25 * r, np.where(r < b, 1.25 * a + (r - a) / 1.7, 1.25 * a + (b - a) / 1.7 + (r - b) / 2.5))
    s = np.floor(g).astype(np.int64)
    if jitter:
        s = np.clip(s + np.random.default_rng(3).integers(-1, 2, n), 0, O.num_slots(n) - 1)
    cnt = range_counts(s)
    assert (cnt <= HALF).sum() > 10 and ((cnt > HALF) & (cnt <= CAP)).sum() > 10 and (cnt > CAP).sum() > 10
    st = sort_slots(x, s)
    assert st["big_buckets"] == int((cnt > CAP).sum())
    assert st["big_bucket_keys"] == int(cnt[cnt > CAP].sum())
    assert st["fallback"] == 0
    if jitter:
        assert st["boundary_keys"] > 0


# ---------------------------------------------------------------------------
# overlaps the neighbour merges cannot settle
# ---------------------------------------------------------------------------
def test_scramble_across_ranges():
    x = W.uniform(200_000, seed=25)
    S = O.num_slots(x.size)
    s = np.clip(rank_slots(x) + np.random.default_rng(4).integers(-3000, 3001, x.size), 0, S - 1)
    st = sort_slots(x, s)
    assert st["fallback"] == 1


def test_ranges_out_of_value_order():
    """Ranges 0..3 hold the value blocks 3, 1, 4, 2 (of 2000 keys each).  The
    ranges two apart are in order, each neighbour pair either overlaps wholly
    or not at all, and the two zone merges give blocks 1 3 and 2 4 side by
    side: out of order at their junction."""
    x = W.uniform(8000, seed=26)
    r = ranks(x)
    blk = r // 2000                               # value block 0..3
    where = np.array([1, 3, 0, 2])[blk]           # range holding each block
    s = where * RANGE_SLOTS + (r % 2000)
    assert s.max() < O.num_slots(x.size)
    st = sort_slots(x, s)
    assert st["fallback"] == 2


@pytest.mark.parametrize("extremes", [True, False])
def test_finite_keys_without_slot(extremes):
    """Keys without a slot go to the ends of the output: below every mapped
    key if negative, above if not.  When they are the extremes (as for the
    keys a model cannot map) that is their place; otherwise the junctions
    show it and the output is sorted whole."""
    x = W.gauss_mix(200_000, seed=27) - 0.5
    s = rank_slots(x)
    r = ranks(x)
    if extremes:
        s[(r < 700) | (r >= x.size - 300)] = UNM
    else:
        s[np.random.default_rng(5).choice(x.size, 1000, replace=False)] = UNM
    st = sort_slots(x, s)
    assert st["unmapped"] == 1000
    assert st["fallback"] == (0 if extremes else 2)


# ---------------------------------------------------------------------------
# non-finite keys, signed zeros and subnormals
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("layout", ["dense_middle", "dense_ends", "jitter"])
def test_edge_keys_in_every_path(layout):
    x = np.concatenate([W.edge_keys(seed=s) for s in range(40)])
    n = x.size
    r = ranks(x)
    e = 4500
    if layout == "dense_middle":
        s = np.where(r < 1500, r, np.where(r < n - 1500, RANGE_SLOTS + (r - 1500) * 2047 // (n - 3000),
                                           2 * RANGE_SLOTS + r - (n - 1500)))
    else:
        s = np.where(r < e, r * 2047 // e, np.where(r < n - e, RANGE_SLOTS + (r - e),
                                                    2 * RANGE_SLOTS + (r - (n - e)) * 2047 // e))
        if layout == "jitter":
            s = np.clip(s + np.random.default_rng(6).integers(-1, 2, n), 0, None)
    assert s.max() < O.num_slots(n)
    cnt = range_counts(s)
    assert (cnt > CAP).any()
    st = sort_slots(x, s)
    assert st["big_buckets"] == int((cnt > CAP).sum())


def test_model_dense_ranges_and_unmapped_keys():
    """F = relu(relu(xhat)) on xhat = (x + 1) / 2: keys below -1 all take slot
    0 and keys above 1 the last slot (two dense ranges); NaNs and infinities
    have no slot.  Both kinds meet in the residue path."""
    x = np.concatenate([np.random.default_rng(7).standard_normal(200_000)] +
                       [W.edge_keys(seed=s) for s in range(10)])
    th = np.zeros(O.num_params(1), np.float32)
    th[0], th[2], th[4] = 1.0, 1.0, 1.0           # w1, W2, w3
    model = {"H": 1, "lo": -1.0, "inv_range": 0.5, "theta": th}
    sp = nn.sort_params(stats_level=1)
    out, st = nn.nnsort_sort_with_model(nn.model_from_dict(model), to_dev(x), sp=sp)
    torch.cuda.synchronize()
    ref, ost = O.nnsort(x, model)
    assert np.array_equal(bits(out.cpu().numpy()), bits(ref))
    for k in ("rounds", "collided", "placed", "residue"):
        assert st[k] == ost[k], (k, st[k], ost[k])
    assert st["big_buckets"] >= 2 and st["unmapped"] > 0


# ---------------------------------------------------------------------------
# dense ranges: lengths at the merge-run boundaries, and a range too long for
# the range-by-range merge (then all of the residue goes through one radix sort)
# ---------------------------------------------------------------------------
def slots_for_range_sizes(x, sizes, seed):
    """Range b (in value order) gets sizes[b] keys at random slots of that
    range; the rest of the keys spread one per slot after them."""
    r = ranks(x)
    rng = np.random.default_rng(seed)
    edges = np.concatenate([[0], np.cumsum(sizes)])
    s = np.empty(x.size, np.int64)
    for b in range(len(sizes)):
        sel = (r >= edges[b]) & (r < edges[b + 1])
        s[sel] = b * RANGE_SLOTS + rng.integers(0, RANGE_SLOTS, int(sel.sum()))
    rest = r >= edges[-1]
    s[rest] = len(sizes) * RANGE_SLOTS + (r[rest] - edges[-1])
    assert s.max() < O.num_slots(x.size)
    return s


@pytest.mark.parametrize("sizes", [[4097, 8192, 8193, 12288, 16385, 65537], [5000] * 7 + [40_000, 100],
                                   [16383, 16384, 24577, 32769, 49152, 131073]])
def test_dense_ranges_at_run_boundaries(sizes):
    x = W.gauss_mix(400_000, seed=28)
    s = slots_for_range_sizes(x, sizes, seed=len(sizes))
    cnt = range_counts(s)
    st = sort_slots(x, s)
    assert st["big_buckets"] == int((cnt > CAP).sum())
    assert st["big_bucket_keys"] == int(cnt[cnt > CAP].sum())
    assert st["fallback"] == 0


def test_dense_range_too_long_for_merging():
    """One range of 1.2M keys (beyond 4096 * 2^8): the residue is sorted by
    one radix pass sequence over all of it, beside two ordinary dense ranges."""
    x = np.concatenate([W.uniform(1_400_000, seed=29), W.edge_keys(seed=29)])
    s = slots_for_range_sizes(x, [6000, 1_200_000, 9000], seed=3)
    st = sort_slots(x, s)
    assert st["big_buckets"] == 3 and st["big_bucket_keys"] == 1_215_000
    assert st["fallback"] == 0


def test_dense_range_longest_merged():
    """One range of exactly 4096 * 2^8 keys: 8 merge rounds, the most the
    range-by-range path takes."""
    x = W.uniform(1_100_000, seed=30)
    s = slots_for_range_sizes(x, [1_048_576, 7000], seed=4)
    st = sort_slots(x, s)
    assert st["big_buckets"] == 2 and st["big_bucket_keys"] == 1_055_576
    assert st["fallback"] == 0


# More than 4M dense keys: the chunk sort leaves runs of two chunks (8192
# keys), so the merge rounds start there and reach 8192 * 2^8 keys.
def test_many_dense_keys_wide_runs():
    """Ranges of 1.7M, 2^20 + 1 (an odd chunk count) and 1.5M keys."""
    x = W.uniform(4_400_000, seed=31)
    s = slots_for_range_sizes(x, [1_700_000, 1_048_577, 1_500_000, 9000], seed=5)
    st = sort_slots(x, s)
    assert st["big_buckets"] == 4 and st["big_bucket_keys"] == 4_257_577
    assert st["fallback"] == 0


def test_many_dense_keys_range_too_long_for_wide_runs():
    """With wide runs a range of 2.2M keys (beyond 8192 * 2^8) sends the
    residue to one radix pass sequence."""
    x = W.uniform(4_500_000, seed=32)
    s = slots_for_range_sizes(x, [2_200_000, 2_100_000, 5000], seed=6)
    st = sort_slots(x, s)
    assert st["big_buckets"] == 3 and st["big_bucket_keys"] == 4_305_000
    assert st["fallback"] == 0


def test_many_dense_ranges_counted_several_chunks_per_workgroup():
    """3,000 dense ranges of 4,097 to 6,000 keys (15.2M keys): with more than
    4,096 chunks of 4,096 dense keys, each workgroup of the slot count takes
    several consecutive chunks, and most of them cross from one range into the
    next; the round counts must still equal the oracle's."""
    x = W.uniform(15_500_000, seed=33)
    rng = np.random.default_rng(7)
    sizes = rng.integers(4097, 6001, 3000)
    edges = np.concatenate([[0], np.cumsum(sizes)])
    r = ranks(x)
    b = np.searchsorted(edges, r, side="right") - 1
    dense = b < sizes.size
    s = np.empty(x.size, np.int64)
    s[dense] = b[dense] * RANGE_SLOTS + rng.integers(0, RANGE_SLOTS, int(dense.sum()))
    s[~dense] = sizes.size * RANGE_SLOTS + (r[~dense] - edges[-1])
    assert s.max() < O.num_slots(x.size)
    assert int(sizes.sum()) // 4096 + sizes.size >= 2 * 2048  # at least two chunks per workgroup
    st = sort_slots(x, s)
    assert st["big_buckets"] == sizes.size and st["big_bucket_keys"] == int(sizes.sum())
    assert st["fallback"] == 0
