"""The operation-count model of NN-sort (Sec. 3, Model Analysis, Eq.
(operations)):

    T(n, e, sigma, t, theta) = C1 n^2 + C2 n log n + C3 n        (n > 1)
    C1 = 1/2 sum_i e_i (1 - sigma_i) (prod_{j<i} sigma_j)^2
    C2 = prod_{j<=t} sigma_j
    C3 = sum_i [theta prod_{j<i} sigma_j + (1 - e_i)(1 - alpha_i) prod_{j<i} sigma_j
                + prod_{j<=i} sigma_j] + C2 log C2

with, per iteration i = 1..t, sigma_i the conflict rate (the share of that
iteration's input that lost its slot), e_i the share of the keys stored in o_i
that are out of order, and theta the operations per key through f.

Readings where the text is ambiguous or at odds with itself:
  - alpha_i is not defined; the polish analysis derives that term as
    (1 - e_i)(1 - sigma_i), so alpha_i = sigma_i;
  - the model-feeding term is printed as theta sum_{j<=i} sigma_j n, but
    iteration i feeds its input, prod_{j<i} sigma_j n keys (sigma_0 = 1), which
    is what is counted here;
  - log is log2 (the n log n of a comparison sort), and 0 log 0 = 0.

The model counts operations of the paper's CPU procedure (an out-of-order
key costs half the merged array to insert); it is a statement about that
procedure, not about the time of this GPU implementation, whose polish orders
each slot range in LDS.  sweep.py prints the two side by side.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass
class Coefficients:
    C1: float
    C2: float
    C3: float


def _check(sigma, e):
    if len(sigma) != len(e) or not sigma:
        raise ValueError("sigma and e need one entry per iteration (t >= 1)")
    for v in list(sigma) + list(e):
        if not 0.0 <= v <= 1.0:
            raise ValueError("rates lie in [0, 1]")


def coefficients(sigma, e, theta: float) -> Coefficients:
    """C1, C2, C3 of Eq. (operations) for iterations i = 1..t."""
    _check(sigma, e)
    c1 = c3 = 0.0
    before = 1.0  # prod_{j<i} sigma_j
    for s, ei in zip(sigma, e):
        c1 += 0.5 * ei * (1.0 - s) * before * before
        c3 += theta * before + (1.0 - ei) * (1.0 - s) * before + before * s
        before *= s
    c2 = before
    c3 += c2 * math.log2(c2) if c2 > 0.0 else 0.0
    return Coefficients(c1, c2, c3)


def operations(n: int, sigma, e, theta: float) -> float:
    """T(n, e, sigma, t, theta); 1 for n = 1."""
    if n <= 1:
        return 1.0
    c = coefficients(sigma, e, theta)
    return c.C1 * n * n + c.C2 * n * math.log2(n) + c.C3 * n


def comparison_sort_operations(n: int) -> float:
    """The n log2 n baseline the model is compared against (Exp-5)."""
    return n * math.log2(n) if n > 1 else 1.0


def rates_from_counts(n: int, collided, placed, extracted):
    """sigma_i and e_i from one run's counts: |c_i| after round i, keys
    stored in o_i, and out-of-order keys of o_i.  sigma_i = |c_i| / |c_{i-1}|
    (|c_0| = n); e_i = extracted_i / placed_i (0 when o_i is empty)."""
    sigma, e = [], []
    prev = n
    for c, p, x in zip(collided, placed, extracted):
        sigma.append(c / prev if prev else 0.0)
        e.append(x / p if p else 0.0)
        prev = c
    return sigma, e
