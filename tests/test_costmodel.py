"""The operation-count model (Sec. 3, Model Analysis): the package's closed
form (C1 n^2 + C2 n log n + C3 n) against the oracle's iteration-by-iteration
count (s(n) + p(n) from sizes), and both against hand-derived values of
special cases.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1907_08817_amd import costmodel as C
from paper_1907_08817_amd import workloads as W


def close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1.0)


# ---------------------------------------------------------------------------
# special cases, by hand
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("theta", [1.0, 32.0, 129.0])
def test_no_conflicts_ordered(theta):
    """f places every key in order in one iteration: each key goes through f
    once and is appended once."""
    n = 10_000
    assert close(C.operations(n, [0.0], [0.0], theta), (theta + 1) * n)
    assert close(O.cost_operations(n, [0], [n], [0], theta), (theta + 1) * n)


def test_no_conflicts_some_out_of_order():
    """A share e of the keys is out of order: each costs n / 2 to insert."""
    n, e, theta = 4000, 0.25, 32.0
    want = e * n * n / 2 + (1 - e) * n + theta * n
    assert close(C.operations(n, [0.0], [e], theta), want)
    assert close(O.cost_operations(n, [0], [n], [int(e * n)], theta), want)


def test_everything_collides():
    """The constant model: one pass through f, every key to the conflict
    array, sorted conventionally (n log2 n) and appended."""
    n, theta = 1 << 16, 32.0
    want = n * 16 + (theta + 1) * n
    assert close(C.operations(n, [1.0], [0.0], theta), want)
    assert close(O.cost_operations(n, [n], [0], [0], theta), want)


def test_exp5_setting_coefficients():
    """Exp-5: t = 5, theta = 32, sigma_i = e_i = 10% in every iteration.
    Geometric sums: C1 = (0.1 * 0.9 / 2) (1 - 0.01^5) / (1 - 0.01),
    C2 = 0.1^5, C3 = (32 + 0.9 * 0.9 + 0.1) (1 - 0.1^5) / 0.9 + C2 log2 C2."""
    c = C.coefficients([0.1] * 5, [0.1] * 5, 32.0)
    assert close(c.C1, 0.0454545454545, rel=1e-11)
    assert close(c.C2, 1e-5)
    assert close(c.C3, 36.566301 + 1e-5 * math.log2(1e-5), rel=1e-12)
    # 5%: C1 = (0.05 * 0.95 / 2) (1 - 0.0025^5) / (1 - 0.0025)
    c = C.coefficients([0.05] * 5, [0.05] * 5, 32.0)
    assert close(c.C1, 0.02375 / 0.9975, rel=1e-11)


def test_one_key():
    assert C.operations(1, [0.5], [0.5], 32.0) == 1.0
    assert O.cost_operations(1, [0], [1], [0], 32.0) == 1.0


def test_rates_from_counts():
    sigma, e = C.rates_from_counts(1000, [300, 60, 0], [700, 240, 60], [7, 24, 0])
    assert sigma == [0.3, 0.2, 0.0]
    assert e == [0.01, 0.1, 0.0]
    with pytest.raises(ValueError):
        C.coefficients([0.1], [0.1, 0.2], 32.0)
    with pytest.raises(ValueError):
        C.coefficients([1.5], [0.0], 32.0)


# ---------------------------------------------------------------------------
# the two forms agree
# ---------------------------------------------------------------------------
def random_counts(rng, n, t):
    collided, placed, extracted = [], [], []
    w = n
    for _ in range(t):
        c = int(rng.integers(0, w + 1))
        p = w - c
        collided.append(c)
        placed.append(p)
        extracted.append(int(rng.integers(0, p + 1)))
        w = c
    return collided, placed, extracted


def test_forms_agree_on_random_counts():
    rng = np.random.default_rng(0)
    for _ in range(200):
        n = int(rng.integers(2, 10 ** 9))
        t = int(rng.integers(1, 9))
        col, pl, ex = random_counts(rng, n, t)
        theta = float(rng.uniform(1, 300))
        sigma, e = C.rates_from_counts(n, col, pl, ex)
        assert close(C.operations(n, sigma, e, theta), O.cost_operations(n, col, pl, ex, theta), rel=1e-9)


@pytest.mark.parametrize("name,H,eps", [("gauss_mix", 32, 3), ("lognormal", 32, 5), ("zipf_u64", 16, 2)])
def test_forms_agree_on_oracle_runs(name, H, eps):
    x = W.make(name, 100_000)
    model = O.fit(x, H=H, sample_frac=0.05, batch=4096, steps=3)
    _, st = O.nnsort(x, model, eps=eps, tau=0)
    assert [p + c for p, c in zip(st["placed"], st["collided"])] == [x.size] + st["collided"][:-1]
    sigma, e = C.rates_from_counts(x.size, st["collided"], st["placed"], st["extracted"])
    theta = 2 * H + 1
    a = C.operations(x.size, sigma, e, theta)
    b = O.cost_operations(x.size, st["collided"], st["placed"], st["extracted"], theta)
    assert close(a, b, rel=1e-12)
    assert a >= theta * x.size  # every key goes through f at least once
