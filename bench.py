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
import hashlib
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
# entities with at most this many entries under a propagated prior take the
# low-rank kernel (the library's own threshold)
LOWRANK_NNZ = 8


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
    p.add_argument("--batched-only", action="store_true",
                   help="skip the plain FP32 arm (for profiler runs)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run 5 device-to-device copies of MIB MiB (to scale the HBM "
                        "traffic counters), then exit")
    return p.parse_args()


def algorithmic_bytes(kind, M, n, K, state_bytes, kept, n_prop=0, n_empty=0, n_lowrank=0):
    """Bytes one update pass must move: per entry a column index and a value
    (8 B) plus the K-element factor row it gathers; per entity its pointer
    pair and its written state row (and sample row when the sweep is kept);
    per entity under a propagated prior (PP stages 2-3) that is factored its
    packed FP64 prior, K(K+1)/2 precision entries and K of the
    precision-weighted mean; per entity with no entries under a propagated
    prior whose factor was computed at stage begin (n_empty) the FP32 factor,
    K(K+1)/2 entries, and the K FP64 entries of the mean; per entity with a
    few entries under such a prior (n_lowrank) the factor, the mean and the
    precision-weighted mean."""
    b = M * (8 + K * state_bytes) + n * (8 + K * state_bytes)
    if kept:
        b += n * K * 4
    b += n_prop * (K * (K + 1) // 2 + K) * 8
    b += n_empty * (K * (K + 1) // 2 * 4 + K * 8)
    b += n_lowrank * (K * (K + 1) // 2 * 4 + 2 * K * 8)
    return b


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1703_00734_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kclass, config, precision):
    """HBM bytes per launch of an update pass, from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE counter passes summarised under profiles/ (each counter scaled by
    what it reads for a device copy of known size).  None when no summary covers
    this pass, or when the kernel sources have changed since the counters were
    taken."""
    want = kernel_sources_hash()
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    for f in sorted(os.listdir(d)):
        if not f.endswith(".md"):
            continue
        with open(os.path.join(d, f)) as fh:
            for line in fh:
                if not line.startswith("traffic-record: "):
                    continue
                r = json.loads(line[len("traffic-record: "):])
                if (r["kclass"] == kclass and r["config"] == config and r["precision"] == precision
                        and r["sources"] == want):
                    return r["hbm_bytes_per_launch"]
    return None


def stages_of(cfg):
    I, J = cfg["I"], cfg["J"]
    st = [1]
    if I > 1 or J > 1:
        st.append(2)
    if I > 1 and J > 1:
        st.append(3)
    return st


def run_arm(d, cfg, precision, batched, steps, warmup, rmse, seed):
    """For every PP stage of the configuration: `warmup` sweeps, then `steps`
    timed sweeps as launched in production (graph replays when batched), then
    as many sweeps launched eagerly with HIP events around every kernel.  Every
    sweep stores a sample (so the next stage has its moment-matched priors).
    Then, in a second context, the configuration's own chain (sweeps per stage,
    burn-in) and the test RMSE of its posterior-mean prediction."""
    import torch
    from paper_1703_00734_amd import BMF

    def ctx(burnin, kept):
        return BMF(d["N"], d["D"], d["K"], d["row"], d["col"], d["val"], I=cfg["I"], J=cfg["J"],
                   order=cfg["order"], seed=seed, burnin=burnin, thin=1, max_kept=kept,
                   precision=precision, batched=batched)

    stream = torch.cuda.current_stream()
    # moment matching needs more kept samples than the rank: stages that feed a
    # next stage top up their samples with untimed sweeps
    need = 2 * d["K"] + 2
    extra = max(0, need - (warmup + 2 * steps))
    g = ctx(0, warmup + 2 * steps + extra)
    per_stage = {}
    stages = stages_of(cfg)
    for s in stages:
        g.pp_stage(s, 0)
        g.gibbs_sweep(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        g.gibbs_sweep(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / steps
        before = g.kernel_times()            # totals so far (earlier stages)
        g.enable_timing(True)
        g.gibbs_sweep(steps)
        torch.cuda.synchronize()
        g.enable_timing(False)
        after = g.kernel_times()
        ktimes = {k: (after[k][0] - before.get(k, (0, 0.0))[0], after[k][1] - before.get(k, (0, 0.0))[1])
                  for k in after}
        row_updates, ratings = g.stage_work()
        # entities with no entries (or at most LOWRANK_NNZ) under a propagated
        # prior: the prior-factor paths take them in FP32/BF16 passes with K > 16
        empty, lowrank = [0, 0], [0, 0]
        if precision != "fp64" and d["K"] > 16 and cfg["I"] * cfg["J"] > 1:
            for b in range(g.nblocks()):
                info = g.block_info(b)
                if info["stage"] != s:
                    continue
                bi, bj = divmod(b, cfg["J"])
                for side, prop in ((0, bj > 0), (1, bi > 0)):
                    if prop:
                        deg = np.diff(g.block_csr(b, side)[0])
                        empty[side] += int(np.count_nonzero(deg == 0))
                        lowrank[side] += int(np.count_nonzero((deg >= 1) & (deg <= LOWRANK_NNZ)))
        print("bench: stage %d timed, %.4f ms per sweep" % (s, ms), file=sys.stderr, flush=True)
        if s != stages[-1] and extra:
            g.gibbs_sweep(extra)
            torch.cuda.synchronize()
        per_stage[s] = dict(ms_per_step=ms, wall_ms_per_step=1000 * wall / steps,
                            ktimes=ktimes, row_updates=row_updates, ratings=ratings,
                            schedule=g.schedule(), empty_prop=empty, lowrank_prop=lowrank)
    out = dict(per_stage=per_stage, stats=g.stats())
    g.close()
    if rmse:
        sweeps, burnin = cfg["sweeps"], cfg["burnin"]
        h = ctx(burnin, sweeps - burnin)
        t0 = time.perf_counter()
        for s in stages_of(cfg):
            h.pp_stage(s, sweeps)
            torch.cuda.synchronize()
            print("bench: chain stage %d done" % s, file=sys.stderr, flush=True)
        p = h.predict(d["test_row"], d["test_col"])
        torch.cuda.synchronize()
        out["chain_wall_s"] = time.perf_counter() - t0
        out["rmse"] = float(np.sqrt(np.mean((p - d["test_val"]) ** 2)))
        out["rmse_sweeps"] = sweeps
        out["rmse_burnin"] = burnin
        h.close()
    return out


def rows_cols_of_stage(d, cfg, s, propagated=False):
    """Rows and columns updated per sweep by the blocks of stage s (with
    propagated=True: only those under a propagated prior, the rows of blocks
    off the first block column and the columns of blocks off the first block
    row)."""
    N, D, I, J = d["N"], d["D"], cfg["I"], cfg["J"]
    bs_r, bs_c = -(-N // I), -(-D // J)
    R = [min(bs_r, N - i * bs_r) for i in range(I)]
    C = [min(bs_c, D - j * bs_c) for j in range(J)]
    rows = cols = 0
    for i in range(I):
        for j in range(J):
            st = 1 if (i == 0 and j == 0) else (2 if (i == 0 or j == 0) else 3)
            if st == s:
                if not propagated or j > 0:
                    rows += R[i]
                if not propagated or i > 0:
                    cols += C[j]
    return rows, cols


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
    if a.copy_calibration > 0:
        n = a.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 5}))
        return
    cfg = dict(synth.CONFIGS[a.config])
    say = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
    say("drawing workload %d" % a.config)
    d = synth.config(a.config, seed=a.seed, progress=say)
    K = d["K"]
    main_prec = "bf16" if cfg["precision"] in ("fp32", "bf16") else cfg["precision"]
    arms = {}
    arms["batched_" + main_prec] = run_arm(d, cfg, main_prec, True, a.steps, a.warmup,
                                           not a.no_rmse, 101)
    print("arm batched %s done" % main_prec, file=sys.stderr, flush=True)
    if main_prec != "fp64" and not a.batched_only:
        arms["plain_fp32"] = run_arm(d, cfg, "fp32", False, a.steps, a.warmup, not a.no_rmse, 101)
        print("arm plain fp32 done", file=sys.stderr, flush=True)
    stages = stages_of(cfg)
    head = stages[-1]                          # the largest, most parallel stage
    m = arms["batched_" + main_prec]["per_stage"][head]
    ms = m["ms_per_step"]
    value = m["ratings"] / (ms / 1000.0)
    # dominant kernel of the per-kernel region of the headline stage
    kt = {k: v for k, v in m["ktimes"].items() if v[0] > 0}
    dom = max(kt, key=lambda k: kt[k][1])
    launches, tot_ms = kt[dom]
    state_bytes = {"fp64": 8, "fp32": 4, "bf16": 2}[main_prec]
    roof = None
    if dom in ("update_rows", "update_cols"):
        M = m["ratings"]
        # entities of the pass: rows (or columns) of every block of the stage
        side = 0 if dom == "update_rows" else 1
        n = rows_cols_of_stage(d, cfg, head)[side]
        n_empty = m["empty_prop"][side]
        n_lowrank = m["lowrank_prop"][side]
        n_prop = rows_cols_of_stage(d, cfg, head, propagated=True)[side] - n_empty - n_lowrank
        # a pass is one launch (K <= 16) or a few: heavy entities, light ones
        # (K > 16), segment Grams apart; the rate is the pass's bytes over the
        # pass's summed launch time
        per_pass = algorithmic_bytes(dom, M, n, K, state_bytes, True, n_prop, n_empty, n_lowrank)
        passes = a.steps
        # the partial Grams of heavy entities (both passes) count against this pass
        seg_ms = kt.get("gram_segments", (0, 0.0))[1]
        avg_ms = (tot_ms + seg_ms) / passes
        ach = per_pass / (avg_ms / 1000.0) / 1e9
        roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS,
                    traffic=measured_traffic(dom, a.config, main_prec), avg_launch_ms=avg_ms,
                    launches_per_pass=launches / passes,
                    algorithmic_bytes_per_launch=per_pass)
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
        "config": {"workload": "%s N=%d D=%d K=%d, %d train entries, Zipf(1.2) degrees, %dx%d "
                               "partition, %s order; step = one sweep of PP stage %d"
                               % ("ratings-shaped" if cfg["kind"] == "ratings" else cfg["kind"],
                                  d["N"], d["D"], K, d["row"].size, cfg["I"], cfg["J"],
                                  cfg["order"], head),
                   "N": d["N"], "D": d["D"], "K": K, "train_nnz": int(d["row"].size),
                   "partition": "%dx%d" % (cfg["I"], cfg["J"]), "stage": head},
        "row_updates_per_s": m["row_updates"] / (ms / 1000.0),
        "roofline": roof,
        "kernel_ms_per_step": {k: v[1] / a.steps for k, v in kt.items()},
        "timing": "ms_per_step: HIP events around the timed sweeps (graph replays in the batched "
                  "arm); kernel times and roofline: a second region of as many sweeps launched "
                  "eagerly with HIP events around every kernel",
        "arms": {},
    }
    for k, v in arms.items():
        arm = {"test_rmse": v.get("rmse"), "chain_wall_s": v.get("chain_wall_s"),
               "fallback_rows": v["stats"]["fallback_rows"], "stages": {}}
        for s_, ps in v["per_stage"].items():
            arm["stages"][str(s_)] = {
                "ms_per_step": ps["ms_per_step"],
                "ratings_per_s": ps["ratings"] / (ps["ms_per_step"] / 1000.0),
                "row_updates_per_s": ps["row_updates"] / (ps["ms_per_step"] / 1000.0),
                "schedule": ps["schedule"]}
        out["arms"][k] = arm
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(d, cfg, a.cpu_seconds, 101)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
