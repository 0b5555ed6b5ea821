"""Benchmark: sorted Gkeys/s of NN-sort on one MI355X.

Workload (default): 1e8 float64 keys from a skewed mixture of 8 Gaussians
(weights Dirichlet(0.3), means U[-1e6, 1e6], sigma log-uniform in [1, 1e4])
with 1% duplicated keys; model 1 -> 64 -> 64 -> 1 fitted on the device from a
1% sample (200 Adam steps) before timing, as the paper excludes training from
the sort time (the first fit call and a second, steady-state one are timed
and reported); inference in the BF16 form (hidden layer on bf16 matrix cores,
FP32 accumulation).  A step is one full sort of the resident keys: map,
rounds, polish, residue sort and merge.

Beside the headline it reports the FP32 and piecewise-linear forms on the same
weights, a full-n GPU radix sort, the fit time, the CPU oracle on a bounded
sample of the same workload, and 1-thread and multi-threaded host sorts of
that sample.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HEADLINE_METRIC = "sorted Gkeys/s at 1e8 f64 keys, BF16-MFMA vs FP32 NN-sort; % HBM roofline"
DEFAULT_WORKLOAD = "gauss_mix_1e8_bf16_h64"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0      # dense bf16 MFMA
FP32_VALU_PEAK_TFLOPS = 157.3  # vector FP32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--n", type=int, default=0, help="override the key count (testing only)")
    ap.add_argument("--form", choices=["config", "bf16", "fp32", "pwl"], default="config",
                    help="map form; 'config' takes the workload's (bf16 for the headline workload)")
    ap.add_argument("--bf16-terms", type=int, default=3)
    ap.add_argument("--no-context", action="store_true", help="skip FP32/radix/CPU context legs")
    ap.add_argument("--cpu-sample", type=int, default=20_000_000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter calibration)")
    return ap.parse_args()


def src_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_counters(kernel: str, sha: str, keys: int) -> dict:
    """The committed counter record of `kernel` (HBM bytes and VALU
    instructions per launch), or {} when absent, taken on a different kernel
    source or on a launch of a different size."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return {}
    e = d.get(kernel)
    if not e or e.get("source_sha256") != sha or e.get("keys_per_launch") != keys:
        return {}
    return e


# VALU issue: a wave64 vector instruction occupies its SIMD for 4 cycles
# (16 lanes per cycle, FP32 and FP64 alike); 256 CUs x 4 SIMDs at 2.4 GHz.
SIMDS, CLOCK_HZ, CYCLES_PER_VALU = 1024, 2.4e9, 4


def valu_issue(counters: dict, launch_ms: float):
    """Time the kernel's counted VALU instructions need at full issue rate,
    and its share of the measured launch time."""
    insts = counters.get("valu_insts_per_launch")
    if not insts:
        return None
    ms = insts * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ) * 1e3
    return {"valu_insts": insts, "issue_ms": round(ms, 4), "frac": round(ms / launch_ms, 4)}


def host_parallel_sort(xs: np.ndarray, threads: int) -> np.ndarray:
    """A conventional multi-threaded host sort, for context: each of `threads`
    chunks is sorted by one worker and cut at splitters drawn from a sorted
    sample; each bucket then merges its sorted pieces (numpy's stable sort
    finds the runs).  numpy releases the GIL inside sort and searchsorted."""
    from concurrent.futures import ThreadPoolExecutor
    if threads < 2 or xs.size < 1 << 16:
        return np.sort(xs)
    rng = np.random.default_rng(0)
    sample = np.sort(xs[rng.integers(0, xs.size, 64 * threads)])
    split = sample[64::64]
    chunks = np.array_split(xs, threads)
    with ThreadPoolExecutor(threads) as pool:
        srt = list(pool.map(np.sort, chunks))
        cuts = [np.concatenate(([0], np.searchsorted(c, split), [c.size])) for c in srt]
        sizes = [sum(int(cuts[c][b + 1] - cuts[c][b]) for c in range(threads)) for b in range(threads)]
        offs = np.concatenate(([0], np.cumsum(sizes)))
        out = np.empty_like(xs)

        def bucket(b):
            piece = np.concatenate([srt[c][cuts[c][b]:cuts[c][b + 1]] for c in range(threads)])
            out[offs[b]:offs[b + 1]] = np.sort(piece, kind="stable")

        list(pool.map(bucket, range(threads)))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sharded path is not built",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1907_08817_amd as nn
    from paper_1907_08817_amd import workloads as W

    name, n_cfg, H, form, frac = W.CONFIGS[args.workload]
    if args.form != "config":
        form = args.form
    n = args.n or n_cfg
    t0 = time.time()
    x = W.make(name, n)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(x if x.dtype == np.float64 else x.view(np.int64)).to(dev)
    out = torch.empty_like(keys)
    dt = nn.F64 if x.dtype == np.float64 else nn.U64

    form_code = {"bf16": nn.FORM_BF16, "fp32": nn.FORM_FP32, "pwl": nn.FORM_PWL}[form]
    sp = nn.sort_params(form=form_code, bf16_terms=args.bf16_terms, stats_level=1)
    fp = nn.fit_params(hidden=H, sample_frac=frac)
    ws = nn.alloc_workspace(nn.workspace_size(n, dt, sp, fp), dev)

    # device fit, excluded from the sort time and reported separately: the
    # first call in the process (which also loads the fit's kernels) and a
    # second one, the steady-state time that value_with_fit uses
    fit_calls_ms = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model = nn.nnsort_fit(keys, fp, ws=ws)
        torch.cuda.synchronize()
        fit_calls_ms.append((time.perf_counter() - t0) * 1e3)
    fit_first_ms, fit_ms = fit_calls_ms

    def run_sort(params):
        return nn.nnsort_sort_with_model(model, keys, out=out, sp=params, ws=ws)

    for _ in range(args.warmup):
        run_sort(sp)
    torch.cuda.synchronize()
    infer_ms, stats = [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, stats = run_sort(sp)
        infer_ms.append(stats["t_infer_ms"])
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3) / 1e9

    # correctness spot check of the timed output (non-decreasing order keys)
    o = out.view(torch.int64)
    top = torch.tensor(-(2 ** 63), dtype=torch.int64, device=dev)
    if dt == nn.F64:
        k = torch.where(o < 0, (~o) ^ top, o)  # totalOrder key with its top bit flipped (signed order)
    else:
        k = o ^ top
    sorted_ok = bool((k[1:] >= k[:-1]).all().item())
    # model quality, outside the timed region (a context leg: its extra map
    # launch writes F instead of slots): mean |F(key) n - rank| / n over the
    # sorted output, with F from the timed form's map kernel
    pos_err = {}
    if not args.no_context:
        _, st2 = run_sort(nn.sort_params(form=form_code, bf16_terms=args.bf16_terms, stats_level=2))
        pos_err["form"] = st2["pos_err"]

    # conflicts of the fit's starting model (no Adam step), beside those of
    # the fitted one that the timed sorts used
    fp0 = nn.fit_params(hidden=H, sample_frac=frac, steps=0)
    model0 = nn.nnsort_fit(keys, fp0, ws=ws)
    _, st0 = nn.nnsort_sort_with_model(model0, keys, out=out, sp=sp, ws=ws)
    init_collided = [round(v / n, 5) for v in st0["collided"]]

    # roofline of the dominant kernel: the model map (inference + hand-off).
    # BF16 form: the hidden-to-hidden product is the matrix cores' work,
    # 2 H^2 flop per key (algorithmic); the bf16x3 split issues it three times
    k1_ms = float(np.mean(infer_ms))
    flop_per_key = 2 * H * H if form == "bf16" else 2 * (2 * H + H * H)
    achieved_tflops = flop_per_key * n / (k1_ms * 1e-3) / 1e12
    if form == "pwl":
        # HBM-bound: 8 bytes read and a 4-byte slot written per key; the map
        # time includes the two launches that compile the pieces
        kname = "k_infer_pwl"
        ctr = load_counters(kname, src_sha(["paper_1907_08817_amd/csrc/infer_pwl.hip",
                                            "paper_1907_08817_amd/csrc/infer_common.h"]), n)
        achieved_gbs = 12 * n / (k1_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 5),
                    "traffic": ctr.get("bytes_per_launch"), "bytes_per_key": 12, "keys_per_launch": n,
                    "avg_launch_ms": round(k1_ms, 4), "valu_issue": valu_issue(ctr, k1_ms)}
    else:
        kname = f"k_infer_bf16<{64 if H > 32 else 32},{args.bf16_terms}>" if form == "bf16" else \
            f"k_infer_fp32<{64 if H > 32 else 32}>"
        ksha = src_sha(["paper_1907_08817_amd/csrc/infer_bf16.hip" if form == "bf16" else
                        "paper_1907_08817_amd/csrc/infer.hip", "paper_1907_08817_amd/csrc/infer_common.h"])
        ctr = load_counters(kname, ksha, n)
        peak = BF16_PEAK_TFLOPS if form == "bf16" else FP32_VALU_PEAK_TFLOPS
        # the matrix-core roofline the metric names, and beside it the vector
        # issue bound that actually limits this kernel (from the committed
        # instruction count and the live launch time)
        roofline = {"bound": "mfma" if form == "bf16" else "alu", "kernel": kname,
                    "achieved": round(achieved_tflops, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved_tflops / peak, 5), "traffic": ctr.get("bytes_per_launch"),
                    "flop_per_key": flop_per_key, "keys_per_launch": n, "avg_launch_ms": round(k1_ms, 4),
                    "valu_issue": valu_issue(ctr, k1_ms)}
        if form == "bf16":
            issued = args.bf16_terms * flop_per_key
            roofline["issued_flop_per_key"] = issued
            roofline["issued_frac"] = round(issued * n / (k1_ms * 1e-3) / 1e12 / peak, 5)

    # whole-sort algorithmic HBM bytes: keys read, placed keys written/read,
    # conflict (key, slot) pairs written/read, residue radix passes, output
    c = stats["collided"]
    ct = stats["residue"]
    placed = n - ct
    alg_bytes = 8 * n + 16 * placed + 24 * sum(c) + 16 * 8 * ct + 8 * ct + 8 * n
    e2e = {"alg_bytes_per_key": round(alg_bytes / n, 2),
           "achieved_GBs": round(alg_bytes / (ms_per_step * 1e-3) / 1e9, 1),
           "frac_of_8TBs": round(alg_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if not args.copy_calibration:
        # the same bytes against what a plain device copy of the keys reaches
        # on this machine (read + write counted), outside the timed region
        a = torch.empty_like(keys)
        a.copy_(keys)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            a.copy_(keys)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2 * 8 * n * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        e2e["copy_GBs"] = round(copy_gbs, 1)
        e2e["frac_of_copy"] = round(alg_bytes / (ms_per_step * 1e-3) / 1e9 / copy_gbs, 4)
        del a

    context = {}
    if not args.no_context:
        # FP32 form on the same weights
        sp32 = nn.sort_params(form=nn.FORM_FP32, stats_level=1)
        run_sort(sp32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(2, args.steps // 3)
        for _ in range(reps):
            _, st32 = run_sort(sp32)
        torch.cuda.synchronize()
        fp32_ms = (time.perf_counter() - t0) * 1e3 / reps
        context["fp32_form_gkeys"] = round(n / (fp32_ms * 1e-3) / 1e9, 3)
        context["fp32_form_ms"] = round(fp32_ms, 3)
        context["fp32_infer_ms"] = round(st32["t_infer_ms"], 3)
        context[f"{form}_vs_fp32"] = round(fp32_ms / ms_per_step, 3)
        _, st32 = run_sort(nn.sort_params(form=nn.FORM_FP32, stats_level=2))
        pos_err["fp32_form"] = st32["pos_err"]
    if not args.no_context and form != "pwl":
        # piecewise-linear form on the same weights
        sppw = nn.sort_params(form=nn.FORM_PWL, stats_level=1)
        run_sort(sppw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, stpw = run_sort(sppw)
        torch.cuda.synchronize()
        pw_ms = (time.perf_counter() - t0) * 1e3 / reps
        context["pwl_form_gkeys"] = round(n / (pw_ms * 1e-3) / 1e9, 3)
        context["pwl_form_ms"] = round(pw_ms, 3)
        context["pwl_infer_ms"] = round(stpw["t_infer_ms"], 3)
        context["pwl_collided_frac"] = [round(v / n, 5) for v in stpw["collided"]]
        _, stpw = run_sort(nn.sort_params(form=nn.FORM_PWL, stats_level=2))
        pos_err["pwl_form"] = stpw["pos_err"]
    if not args.no_context:
        # full-n GPU LSD radix sort
        rws = nn.alloc_workspace(nn._lib().nnsort_radix_workspace_size(n), dev)
        nn.nnsort_radix_sort(keys, out=out, ws=rws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            nn.nnsort_radix_sort(keys, out=out, ws=rws)
        torch.cuda.synchronize()
        rad_ms = (time.perf_counter() - t0) * 1e3 / reps
        context["radix_gkeys"] = round(n / (rad_ms * 1e-3) / 1e9, 3)
        del rws
    if args.copy_calibration:
        a = torch.empty(n, dtype=torch.float64, device=dev)
        a.copy_(keys)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_context and args.cpu_sample > 0:
        import oracle
        m = min(args.cpu_sample, n)
        xs = x[:m]
        mdict = nn.model_to_dict(model)
        formc = {"bf16": oracle.FORM_BF16W, "fp32": oracle.FORM_FP32C, "pwl": oracle.FORM_FP64}[form]
        evaluator = {"bf16": "FP64 evaluator with W2 rounded to bf16", "fp32": "canonical FP32 evaluator",
                     "pwl": "FP64 evaluator"}[form]
        t0 = time.perf_counter()
        oracle.nnsort(xs, mdict, form=formc)
        cpu_s = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # a conventional host sort of the same sample (numpy's introsort, one
        # thread), with the host's CPU model
        t0 = time.perf_counter()
        ref = np.sort(xs, kind="quicksort")
        context["host_sort_gkeys"] = round(m / (time.perf_counter() - t0) / 1e9, 5)
        context["host_sort"] = "numpy quicksort (introsort), 1 thread, same sample"
        t0 = time.perf_counter()
        par = host_parallel_sort(xs, cores)
        context["host_par_sort_gkeys"] = round(m / (time.perf_counter() - t0) / 1e9, 5)
        context["host_par_sort"] = (f"sample sort over {cores} threads (numpy sort per chunk and bucket), "
                                    f"same sample, output equal to the 1-thread sort: "
                                    f"{bool(np.array_equal(par, ref, equal_nan=True))}")
        try:
            context["host_cpu"] = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                                       if l.startswith("model name"))
        except (OSError, StopIteration):
            context["host_cpu"] = None
        cpu = {"value": round(m / cpu_s / 1e9, 6), "unit": "Gkeys/s", "cores": cores, "kind": "oracle",
               "sample": f"first {m} keys of the same workload, same model, {evaluator}; {cpu_s:.1f} s"}

    res = {
        "metric": HEADLINE_METRIC if (args.workload == DEFAULT_WORKLOAD and n == n_cfg and form == "bf16")
        else f"sorted Gkeys/s at {n:.0e} {'f64' if dt == nn.F64 else 'u64'} keys, {form} NN-sort ({args.workload})",
        "value": round(value, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp32": "fp32", "pwl": "f64"}[form],
        "data": "synthetic",
        "config": {"workload": args.workload, "distribution": name, "n": n,
                   "keys": "f64" if dt == nn.F64 else "u64", "hidden": H,
                   "form": {"bf16": f"bf16x{args.bf16_terms}", "fp32": "fp32", "pwl": "piecewise-linear f64"}[form],
                   "m": 1.25, "eps": 3, "tau": 1024, "fit": f"device, {frac:g} sample, 200 Adam steps, "
                                                          "outside the timed region"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "sorted_ok": sorted_ok,
        "fit_ms": round(fit_ms, 2),
        "fit_first_call_ms": round(fit_first_ms, 2),
        "value_with_fit": round(n / ((ms_per_step + fit_ms) * 1e-3) / 1e9, 4),
        "e2e_hbm": e2e,
        "rounds": stats["rounds"],
        "collided_frac": [round(v / n, 5) for v in c],
        "init_collided_frac": init_collided,
        "residue_frac": round(ct / n, 5),
        "pos_err": {k: float(f"{v:.5g}") for k, v in pos_err.items()},
        "boundary_keys": stats["boundary_keys"],
        "fallback": stats["fallback"], "range_resorts": stats["range_resorts"],
        "big_bucket_keys": stats["big_bucket_keys"],
        "phase_ms": {k: round(stats[k], 3) for k in ("t_infer_ms", "t_place_ms", "t_polish_ms",
                                                       "t_residue_ms", "t_merge_ms", "t_total_ms")},
        "context": context,
        "datagen_s": round(gen_s, 1),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
