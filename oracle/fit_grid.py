"""Does Adam improve the fitted CDF model for sorting?  A grid of oracle fits.

TEST INFRASTRUCTURE (analysis of the oracle's fit; never imported by the
library).  For each workload, learning rate, loss and step scaling it runs
the oracle's fit loop (FP64 forward/backward, Adam with bias correction) from
the ramp start for 200 steps on batches of 65,536, and reports the round-1
conflict fraction |c_1| / n of the FP64 model on all n keys (m = 1.25):
  - at the start, after the step with the lowest batch loss, at the end, and
    the lowest seen every 25 steps along the way;
  - beside the first, lowest and last batch loss.

Step scalings (the update of parameter p is lr * s_p * mhat_p / (sqrt(vhat_p)
+ eps), Adam on the rescaled parameter theta_p / s_p):
  plain     s_p = 1 (Adam as published, Kingma and Ba);
  relative  s_p = |theta_p at the start| (zero-start parameters stay 0);
  leverage  s_p = 1 / RMS over the sample of dF/dtheta_p at the start (zero-start
            parameters stay 0), so that a step moves F by about lr whatever the
            parameter.

    python -m oracle.fit_grid [n] > grid.md
"""
from __future__ import annotations

import math
import sys
import time

import numpy as np

import oracle as O
from paper_1907_08817_amd import workloads as W

H, FRAC, BATCH, STEPS, SEED, M = 64, 0.01, 65536, 200, 0, 1.25


def conflicts1(x, th, lo, inv):
    xh, ok = O.translate(x, lo, inv)
    F = O.eval_F(xh[ok], {"H": H, "theta": th.astype(np.float32)}, O.FORM_FP64)
    k = np.bincount(O.slots_from_F(F, M * x.size).astype(np.int64))
    return float(np.maximum(k - 1, 0).sum() + (~ok).sum()) / x.size


def jac_rms(th, x):
    """RMS over x of dF/dtheta, by the chain rule on the FP64 graph."""
    w1, b1 = th[:H], th[H:2 * H]
    W2 = th[2 * H:2 * H + H * H].reshape(H, H)
    b2, w3 = th[2 * H + H * H:3 * H + H * H], th[3 * H + H * H:4 * H + H * H]
    z1 = np.outer(x, w1) + b1
    a1 = z1 > 0
    h1 = np.where(a1, z1, 0.0)
    z2 = h1 @ W2.T + b2
    a2 = z2 > 0
    h2 = np.where(a2, z2, 0.0)
    d2 = a2 * w3
    d1 = (d2 @ W2) * a1
    sq = np.zeros(th.size)
    sq[:H] = (d1 ** 2 * x[:, None] ** 2).mean(0)
    sq[H:2 * H] = (d1 ** 2).mean(0)
    sq[2 * H:2 * H + H * H] = ((d2 ** 2).T @ (h1 ** 2) / x.size).ravel()
    sq[2 * H + H * H:3 * H + H * H] = (d2 ** 2).mean(0)
    sq[3 * H + H * H:4 * H + H * H] = (h2 ** 2).mean(0)
    sq[-1] = 1.0
    return np.sqrt(sq)


def run(x, lr, loss, scaling):
    _, lo, inv, xh, y = O.fit_sample(x, FRAC, SEED)
    th0 = O.init_theta(H, 1, SEED, xh)
    if scaling == "plain":
        s = np.ones_like(th0)
    elif scaling == "relative":
        s = np.abs(th0)
    else:
        lev = jac_rms(th0, xh)
        s = np.where((th0 != 0) & (lev > 0), 1.0 / np.maximum(lev, 1e-300), 0.0)
    th = th0.copy()
    m1, m2 = np.zeros_like(th), np.zeros_like(th)
    best, best_loss, hist, traj = th.copy(), math.inf, [], []
    for t in range(1, STEPS + 1):
        bi = O.batch_indices(SEED, t, xh.size, BATCH)
        L, g = O.loss_grad(th, H, xh[bi], y[bi], loss, 0.01)
        hist.append(L)
        if L < best_loss:
            best, best_loss = th.copy(), L
        phi = np.zeros_like(th)
        O.adam_step(phi, np.ascontiguousarray(g * s), m1, m2, t, lr)
        th = (th + s * phi).astype(np.float32).astype(np.float64)
        if t % 25 == 0:
            traj.append(conflicts1(x, th, lo, inv) if np.all(np.isfinite(th)) else 1.0)
    c0 = conflicts1(x, th0, lo, inv)
    cb = conflicts1(x, best, lo, inv)
    ce = conflicts1(x, th, lo, inv) if np.all(np.isfinite(th)) else 1.0
    return c0, cb, ce, min(traj), hist[0], min(hist), hist[-1]


def main():
    n = int(float(sys.argv[1])) if len(sys.argv) > 1 else 10 ** 7
    print(f"n = {n} keys per workload, H {H}, {FRAC:.0%} sample, batch {BATCH}, {STEPS} steps, seed {SEED}; "
          "c1 = round-1 conflict fraction of the FP64 model on all n keys\n")
    print("| workload | loss | scaling | lr | c1 start | c1 best-loss | c1 end | lowest c1 seen | "
          "loss first | loss lowest | loss last |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for name in ("gauss_mix", "piecewise_uniform"):
        x = W.make(name, n)
        for loss in (0, 1):
            for scaling in ("plain", "relative", "leverage"):
                for lr in (1e-3, 1e-5, 1e-7):
                    t = time.time()
                    r = run(x, lr, loss, scaling)
                    print(f"| {name} | {'MSE' if loss == 0 else 'Huber 0.01'} | {scaling} | {lr:g} | "
                          f"{r[0]:.5f} | {r[1]:.5f} | {r[2]:.5f} | {r[3]:.5f} | {r[4]:.3g} | {r[5]:.3g} | "
                          f"{r[6]:.3g} |", flush=True)
                    print(f"<!-- {time.time() - t:.0f} s -->", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
