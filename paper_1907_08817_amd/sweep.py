"""Parameter and distribution-shift sweeps of the GPU NN-sort.

    python -m paper_1907_08817_amd.sweep params [--workload NAME] [--n N]
    python -m paper_1907_08817_amd.sweep shift  [--n N]
    python -m paper_1907_08817_amd.sweep fit    [--workload NAME] [--n N]
    python -m paper_1907_08817_amd.sweep cost   [--workload NAME] [--n N]

params: one device-fitted model, then sorts with eps = 1..5 (eps = 1 is a
single mapping round, the SageDB-style one-pass use of the model), m in
{1.0, 1.25, 1.5, 2.0}, tau in {0, 1024, 1e6} and, for the BF16 form, 1..3 bf16
terms per activation; per setting the rounds run,
the conflict array after each round as a fraction of n, and the time of each
phase (Sec. 4, Exp-4: the number of iterations; Sec. 3: the relaxation factor
m trades slots for conflicts).

shift: a model fitted on uniform keys sorts uniform keys with a growing
fraction replaced by normal keys (Sec. 4, Exp-3), beside the GPU radix sort of
the same keys.

fit: the device fit under three recipes -- MSE with batches of 65,536 (the
default), and the paper's Huber loss (Sec. 4.1, Eq. (loss)) with batches of
65,536 and of 128 -- with the fit time, the batch loss before the first and
after the last step, and the sort that the fitted model gives.

cost: the operation-count model of Sec. 3 (costmodel.py) fed with measured
rates -- sigma_i from the sort's round counts and e from f's inversions (the
share of keys whose slot is below the running maximum of the slots of all
smaller keys, read off the sorted output; 0 exactly when f is monotone on the
keys, and then every e_i is 0) -- with theta = f's flops per key, for eps =
1..5, beside the measured sort time and the n log2 n of a comparison sort;
then the model's curve for Exp-5 (t = 5, theta = 32, sigma_i = e_i = 10% and
5%) over n.

Each setting prints one JSON line.  Times are medians of --reps sorts, from
HIP events on the call's stream, with keys resident in device memory.
"""
from __future__ import annotations

import argparse
import json
import statistics
import time

import numpy as np

from . import costmodel as CM
from . import workloads as W
from . import (F64, U64, FORM_BF16, FORM_FP32, alloc_workspace, fit_params, nnsort_fit, nnsort_predict,
               nnsort_radix_sort, nnsort_sort_with_model, sort_params, workspace_size, _lib)


def _timed(fn, reps, torch):
    ts, out = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(ts), out


def _phases(st):
    return {k: round(v, 3) for k, v in st.items() if k.startswith("t_")}


def sweep_params(args, torch, dev):
    name, n, H, form, frac = W.CONFIGS[args.workload]
    n = args.n or n
    x = W.make(name, n)
    is_f64 = x.dtype == np.float64
    keys = torch.from_numpy(x if is_f64 else x.view(np.int64)).to(dev)
    dt = F64 if is_f64 else U64
    fc = FORM_BF16 if form == "bf16" else FORM_FP32
    big = sort_params(m=3.0, form=fc)
    ws = alloc_workspace(workspace_size(n, dt, big, fit_params(hidden=H, sample_frac=frac)), dev)
    model = nnsort_fit(keys, fit_params(hidden=H, sample_frac=frac), ws=ws)
    out = torch.empty_like(keys)
    grid = [(e, 1.25, 1024) for e in range(1, 6)] + [(3, m, 1024) for m in (1.0, 1.5, 2.0)] + \
           [(3, 1.25, t) for t in (0, 1_000_000)]
    for eps, m, tau in grid:
        sp = sort_params(form=fc, eps=eps, m=m, tau=tau, stats_level=1)
        nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws)
        ms, (_, st) = _timed(lambda: nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws), args.reps, torch)
        print(json.dumps({"sweep": "params", "workload": args.workload, "n": n, "eps": eps, "m": m, "tau": tau,
                          "rounds": st["rounds"], "conflict_frac": [round(c / n, 5) for c in st["collided"][:st["rounds"]]],
                          "residue_frac": round(st["residue"] / n, 5), "ms": round(ms, 3),
                          "gkeys_s": round(n / ms / 1e6, 3), "phases": _phases(st)}), flush=True)
    if fc != FORM_BF16:
        return
    # the number of bf16 terms each hidden activation is split into: 1 is a
    # plain bf16 activation, 3 carries all 24 bits of the FP32 value
    for terms in (1, 2, 3):
        sp = sort_params(form=fc, bf16_terms=terms, stats_level=2)
        _, st2 = nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws)
        sp = sort_params(form=fc, bf16_terms=terms, stats_level=1)
        ms, (_, st) = _timed(lambda: nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws), args.reps, torch)
        print(json.dumps({"sweep": "params", "workload": args.workload, "n": n, "bf16_terms": terms,
                          "pos_err": float(f"{st2['pos_err']:.5g}"), "rounds": st["rounds"],
                          "conflict_frac": [round(c / n, 5) for c in st["collided"][:st["rounds"]]],
                          "residue_frac": round(st["residue"] / n, 5), "fallback": st["fallback"],
                          "ms": round(ms, 3), "gkeys_s": round(n / ms / 1e6, 3), "phases": _phases(st)}),
              flush=True)


def sweep_shift(args, torch, dev):
    n = args.n or 100_000_000
    fx = W.uniform(n, seed=0)
    fkeys = torch.from_numpy(fx).to(dev)
    fp = fit_params(hidden=32, sample_frac=0.01)
    sp = sort_params(form=FORM_FP32, stats_level=1)
    ws = alloc_workspace(workspace_size(n, F64, sp, fp), dev)
    model = nnsort_fit(fkeys, fp, ws=ws)
    del fkeys
    rws = alloc_workspace(_lib().nnsort_radix_workspace_size(n), dev)
    for noise in (0.0, 0.05, 0.1, 0.2, 0.3, 0.4, 0.5):
        x = W.noisy_uniform(n, noise, seed=5)
        keys = torch.from_numpy(x).to(dev)
        out = torch.empty_like(keys)
        nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws)
        ms, (_, st) = _timed(lambda: nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws), args.reps, torch)
        rms, _ = _timed(lambda: nnsort_radix_sort(keys, out=out, ws=rws), args.reps, torch)
        print(json.dumps({"sweep": "shift", "n": n, "noise": noise, "rounds": st["rounds"],
                          "conflict_frac": [round(c / n, 5) for c in st["collided"][:st["rounds"]]],
                          "residue_frac": round(st["residue"] / n, 5), "ms": round(ms, 3),
                          "gkeys_s": round(n / ms / 1e6, 3), "radix_ms": round(rms, 3),
                          "radix_gkeys_s": round(n / rms / 1e6, 3), "phases": _phases(st)}), flush=True)
        del keys, out


def sweep_fit(args, torch, dev):
    name, n, H, form, frac = W.CONFIGS[args.workload]
    n = args.n or n
    x = W.make(name, n)
    is_f64 = x.dtype == np.float64
    keys = torch.from_numpy(x if is_f64 else x.view(np.int64)).to(dev)
    dt = F64 if is_f64 else U64
    fc = FORM_BF16 if form == "bf16" else FORM_FP32
    sp = sort_params(form=fc, stats_level=1)
    ws = alloc_workspace(workspace_size(n, dt, sp, fit_params(hidden=H, sample_frac=frac)), dev)
    out = torch.empty_like(keys)
    for loss, delta, batch in ((0, 1.0, 65536), (1, 0.01, 65536), (1, 0.01, 128)):
        fp = fit_params(hidden=H, sample_frac=frac, loss=loss, huber_delta=delta, batch=batch)
        nnsort_fit(keys, fp, ws=ws)  # the first call in the process also loads the fit's kernels
        fit_ms, (model, hist) = _timed(lambda: nnsort_fit(keys, fp, ws=ws, history=True), 1, torch)
        nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws)
        ms, (_, st) = _timed(lambda: nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws), args.reps, torch)
        print(json.dumps({"sweep": "fit", "workload": args.workload, "n": n, "loss": "huber" if loss else "mse",
                          "delta": delta, "batch": batch, "steps": fp.steps, "fit_ms": round(fit_ms, 2),
                          "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
                          "conflict_frac": [round(c / n, 5) for c in st["collided"][:st["rounds"]]],
                          "residue_frac": round(st["residue"] / n, 5), "dense_range_keys": st["big_bucket_keys"],
                          "ms": round(ms, 3), "gkeys_s": round(n / ms / 1e6, 3)}), flush=True)


def sweep_cost(args, torch, dev):
    name, n, H, form, frac = W.CONFIGS[args.workload]
    n = args.n or n
    x = W.make(name, n)
    is_f64 = x.dtype == np.float64
    keys = torch.from_numpy(x if is_f64 else x.view(np.int64)).to(dev)
    dt = F64 if is_f64 else U64
    fc = FORM_BF16 if form == "bf16" else FORM_FP32
    fp = fit_params(hidden=H, sample_frac=frac)
    sp = sort_params(form=fc, eps=5, tau=0, stats_level=1)
    ws = alloc_workspace(workspace_size(n, dt, sp, fp), dev)
    model = nnsort_fit(keys, fp, ws=ws)
    out = torch.empty_like(keys)
    nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws)
    slots, _ = nnsort_predict(model, out, sp, want_F=False)
    s = slots.cpu().numpy().astype(np.int64)
    s = s[s != 0xFFFFFFFF]
    e_hat = float(np.count_nonzero(s < np.maximum.accumulate(s))) / max(n, 1)
    theta = 2 * H * H + 4 * H + 1
    del slots, s
    for eps in range(1, 6):
        sp = sort_params(form=fc, eps=eps, tau=0, stats_level=1)
        nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws)
        ms, (_, st) = _timed(lambda: nnsort_sort_with_model(model, keys, out=out, sp=sp, ws=ws), args.reps, torch)
        sigma, _ = CM.rates_from_counts(n, st["collided"][:st["rounds"]], st["placed"][:st["rounds"]],
                                        [0] * st["rounds"])
        e = [e_hat] * len(sigma)
        T = CM.operations(n, sigma, e, theta)
        c = CM.coefficients(sigma, e, theta)
        print(json.dumps({"sweep": "cost", "workload": args.workload, "n": n, "eps": eps, "theta": theta,
                          "sigma": [round(v, 5) for v in sigma], "e": e_hat,
                          "C1": c.C1, "C2": c.C2, "C3": round(c.C3, 3), "T_ops": T,
                          "T_over_nlog2n": round(T / CM.comparison_sort_operations(n), 3),
                          "ms": round(ms, 3), "ps_per_op": round(ms * 1e9 / T, 4)}), flush=True)
    for rate in (0.10, 0.05):
        curve = {}
        for k in range(3, 10):
            nn_ = 10 ** k
            curve[f"1e{k}"] = round(CM.operations(nn_, [rate] * 5, [rate] * 5, 32.0) /
                                    CM.comparison_sort_operations(nn_), 4)
        print(json.dumps({"sweep": "cost_exp5", "t": 5, "theta": 32, "sigma=e": rate, "T_over_nlog2n": curve}),
              flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["params", "shift", "fit", "cost"])
    ap.add_argument("--workload", default="gauss_mix_1e8_bf16_h64")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch
    dev = torch.device("cuda:0")
    {"params": sweep_params, "shift": sweep_shift, "fit": sweep_fit, "cost": sweep_cost}[args.what](args, torch, dev)


if __name__ == "__main__":
    main()
