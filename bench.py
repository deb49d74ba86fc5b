"""Benchmark: Gibbs sweeps of BPMF on one MI355X.

A step is one full sweep of the hot path over the workload: every row given
W, every column given the new X, the Normal-Wishart draws, the tau draw and
the sample store.  Default workload: the ratings-shaped single block
N = 70,000, D = 10,700, K = 10, 10M observed entries (9M train), Zipf(1.2)
degrees (synthetic, seeded).  The headline arm runs in BF16 state precision,
batched; the plain FP32 arm is timed beside it and both chains' test RMSE
after burn-in are reported.

Prints one JSON line.  `--gpus N` with N > 1 is not supported (one GPU).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "row-updates/s and ratings/s per Gibbs sweep, batched BF16 vs plain FP32, equal RMSE"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--config", type=int, default=2)
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--no-rmse", action="store_true", help="skip the equal-RMSE chains")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    return p.parse_args()


def algorithmic_bytes(kind, M, n, K, state_bytes, kept):
    """Bytes one update launch must move: per entry a column index and a value
    (8 B) plus the K-element factor row it gathers; per entity its pointer
    pair and its written state row (and sample row when the sweep is kept)."""
    b = M * (8 + K * state_bytes) + n * (8 + K * state_bytes)
    if kept:
        b += n * K * 4
    return b


def run_arm(d, cfg, precision, batched, steps, warmup, rmse, seed):
    """Time `steps` sweeps after `warmup` (every timed sweep stores a sample),
    then, in a second context, run the configuration's chain (sweeps, burn-in)
    and compute the test RMSE of the posterior-mean prediction."""
    import torch
    from paper_1703_00734_amd import BMF

    def ctx(burnin, kept):
        return BMF(d["N"], d["D"], d["K"], d["row"], d["col"], d["val"], I=cfg["I"], J=cfg["J"],
                   order=cfg["order"], seed=seed, burnin=burnin, thin=1, max_kept=kept,
                   precision=precision, batched=batched)

    g = ctx(warmup, steps)
    stream = torch.cuda.current_stream()
    g.gibbs_sweep(warmup)
    torch.cuda.synchronize()
    g.enable_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    g.gibbs_sweep(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    g.enable_timing(False)
    ktimes = g.kernel_times()
    row_updates, ratings = g.stage_work()
    out = dict(ms_per_step=ms, wall_ms_per_step=1000 * wall / steps, ktimes=ktimes,
               row_updates=row_updates, ratings=ratings, stats=g.stats())
    g.close()
    if rmse:
        sweeps, burnin = cfg["sweeps"], cfg["burnin"]
        h = ctx(burnin, sweeps - burnin)
        h.gibbs_sweep(sweeps)
        p = h.predict(d["test_row"], d["test_col"])
        out["rmse"] = float(np.sqrt(np.mean((p - d["test_val"]) ** 2)))
        out["rmse_sweeps"] = sweeps
        out["rmse_burnin"] = burnin
        h.close()
    return out


def cpu_baseline(d, cfg, seconds, seed):
    """The FP64 oracle's sweeps on the host cores for a bounded time."""
    from oracle.bpmf import Oracle
    o = Oracle(d["N"], d["D"], d["K"], d["row"], d["col"], d["val"], I=cfg["I"], J=cfg["J"],
               order=cfg["order"], seed=seed)
    o.begin_stage(1)
    blocks = o.stage_blocks(1)
    M = sum(b["M"] for b in blocks)
    n = sum(b["R"] + b["C"] for b in blocks)
    o.sweep(1)                                 # warm-up
    t0 = time.perf_counter()
    k = 0
    while True:
        o.sweep(1)
        k += 1
        el = time.perf_counter() - t0
        if el >= seconds or k >= 1000:
            break
    cores = len(os.sched_getaffinity(0))
    return dict(value=M * k / el, unit="ratings/s", cores=cores, kind="oracle",
                row_updates_per_s=n * k / el,
                sample="%d full FP64 oracle sweeps of stage 1 (%d blocks) of the same workload, "
                       "%.1f s, OpenMP over rows" % (k, len(blocks), el))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = dict(synth.CONFIGS[a.config])
    d = synth.config(a.config, seed=a.seed)
    K = d["K"]
    main_prec = "bf16" if cfg["precision"] in ("fp32", "bf16") else cfg["precision"]
    arms = {}
    arms["batched_" + main_prec] = run_arm(d, cfg, main_prec, True, a.steps, a.warmup,
                                           not a.no_rmse, 101)
    print("arm batched %s: %.4f ms/step" % (main_prec, arms["batched_" + main_prec]["ms_per_step"]),
          file=sys.stderr, flush=True)
    if main_prec != "fp64":
        arms["plain_fp32"] = run_arm(d, cfg, "fp32", False, a.steps, a.warmup, not a.no_rmse, 101)
        print("arm plain fp32: %.4f ms/step" % arms["plain_fp32"]["ms_per_step"], file=sys.stderr,
              flush=True)
    m = arms["batched_" + main_prec]
    ms = m["ms_per_step"]
    value = m["ratings"] / (ms / 1000.0)
    # dominant kernel of the timed region
    kt = {k: v for k, v in m["ktimes"].items() if v[0] > 0}
    dom = max(kt, key=lambda k: kt[k][1])
    launches, tot_ms = kt[dom]
    state_bytes = {"fp64": 8, "fp32": 4, "bf16": 2}[main_prec]
    roof = None
    if dom in ("update_rows", "update_cols"):
        M = m["ratings"]
        n = d["N"] if dom == "update_rows" else d["D"]
        # one launch per pass in batched mode; every timed sweep stores a sample
        per_launch = algorithmic_bytes(dom, M, n, K, state_bytes, True)
        avg_ms = tot_ms / launches
        ach = per_launch / (avg_ms / 1000.0) / 1e9
        roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=None, avg_launch_ms=avg_ms,
                    algorithmic_bytes_per_launch=per_launch)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ratings/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {"workload": "ratings-shaped single block N=%d D=%d K=%d, %d train entries, "
                               "Zipf(1.2) degrees, %dx%d partition" % (d["N"], d["D"], K,
                                                                    d["row"].size, cfg["I"],
                                                                    cfg["J"]),
                   "N": d["N"], "D": d["D"], "K": K, "train_nnz": int(d["row"].size),
                   "partition": "%dx%d" % (cfg["I"], cfg["J"])},
        "row_updates_per_s": m["row_updates"] / (ms / 1000.0),
        "roofline": roof,
        "kernel_ms_per_step": {k: v[1] / a.steps for k, v in kt.items()},
        "arms": {k: {"ms_per_step": v["ms_per_step"],
                     "ratings_per_s": v["ratings"] / (v["ms_per_step"] / 1000.0),
                     "row_updates_per_s": v["row_updates"] / (v["ms_per_step"] / 1000.0),
                     "test_rmse": v.get("rmse"), "fallback_rows": v["stats"]["fallback_rows"]}
                 for k, v in arms.items()},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(d, cfg, a.cpu_seconds, 101)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
