"""Benchmark: Gibbs sweeps of BPMF under posterior propagation on one MI355X.

Default workload: the ratings-shaped 480,000 x 17,800 matrix, K = 32, 100M
observed entries (90M train), Zipf(1.2) degrees with a heavy head, partitioned
8 x 8 in decreasing order of observations (synthetic, seeded).  A step is one
sweep of each of the three PP stages: all 64 blocks once (every row given W,
every column given the new X, the Normal-Wishart draws of the non-propagated
sides, the tau draw and the sample store), so the whole job's throughput is
the training entries of all blocks over the summed per-sweep times of the
stages (stages run in order: each needs the previous one's moment-matched
priors).  The headline arm keeps the chain state in BF16 and runs every stage
batched (one launch per pass over all of the stage's blocks, each sweep
replayed from a captured HIP graph); the plain FP32 arm (FP32 state, one launch
sequence per block, no graph) is timed beside it, and both arms' test RMSE
after their full chains (three chain seeds) are reported.

Prints one JSON line.  `--gpus N` with N > 1 is not supported (one GPU).
"""
import argparse
import hashlib
import itertools
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
CHAIN_SEEDS = (101, 102, 103)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--config", type=int, default=5)
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--no-rmse", action="store_true", help="skip the equal-RMSE chains")
    p.add_argument("--chains", type=int, default=3, help="chain seeds per arm for the RMSE")
    p.add_argument("--cpu-seconds", type=float, default=24.0,
                   help="oracle time budget with all host threads (the 1-thread run gets half)")
    p.add_argument("--batched-only", action="store_true",
                   help="skip the plain FP32 arm (for profiler runs)")
    p.add_argument("--trace", default="",
                   help="write a per-sweep JSONL trace (train RMSE, tau, counters) of the first "
                        "headline chain to this path")
    p.add_argument("--paper-sim", action="store_true",
                   help="instead of the headline: the paper's simulated workload (Sec. 5.3) with its "
                        "1200/800/2 schedule at partitions 1x1 .. 30x30, both orders, both missingness "
                        "scenarios; prints one JSON line of test RMSE and chain times beside Table 4")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run 5 device-to-device copies of MIB MiB (to scale the HBM "
                        "traffic counters), then exit")
    return p.parse_args()


def say(m):
    print("bench: " + m, file=sys.stderr, flush=True)


def algorithmic_bytes(M, n, K, state_bytes, kept, n_prior=0, n_factor=0):
    """Bytes one update pass must move: per entry a column index and a value
    (8 B) plus the K-element factor row it gathers; per entity its pointer
    pair and its written state row (and sample row when the sweep is kept).
    Propagated priors (PP stages 2-3) are charged once per distinct
    propagated row, however many sibling blocks hold a copy of it: n_prior
    rows whose packed FP64 prior (K(K+1)/2 precision entries and K of the
    precision-weighted mean) some copy's factorisation reads, and n_factor
    rows whose stored FP32 prior factor (K(K+1)/2 entries) and FP64 mean and
    precision-weighted mean (2K entries) the copies with at most eight
    entries read."""
    b = M * (8 + K * state_bytes) + n * (8 + K * state_bytes)
    if kept:
        b += n * K * 4
    b += n_prior * (K * (K + 1) // 2 + K) * 8
    b += n_factor * (K * (K + 1) // 2 * 4 + 2 * K * 8)
    return b


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1703_00734_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kclass, config, stage, precision):
    """HBM bytes per pass of an update pass, from the rocprofv3 FETCH_SIZE and
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
                if (r["kclass"] == kclass and r["config"] == config and r.get("stage", 1) == stage
                        and r["precision"] == precision and r["sources"] == want):
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


def _ctx(d, cfg, precision, batched, seed, burnin, kept):
    from paper_1703_00734_amd import BMF
    return BMF(d["N"], d["D"], d["K"], d["row"], d["col"], d["val"], I=cfg["I"], J=cfg["J"],
               order=cfg["order"], seed=seed, burnin=burnin, thin=1, max_kept=kept,
               precision=precision, batched=batched)


def time_stages(d, cfg, precision, batched, steps, warmup):
    """For every PP stage: `warmup` sweeps, then `steps` timed sweeps as
    launched in production (graph replays when batched), then as many sweeps
    launched eagerly with HIP events around every kernel.  Every sweep stores a
    sample (so the next stage has its moment-matched priors)."""
    import torch
    stream = torch.cuda.current_stream()
    # moment matching needs more kept samples than the rank: stages that feed a
    # next stage top up their samples with untimed sweeps
    need = 2 * d["K"] + 2
    extra = max(0, need - (warmup + 2 * steps))
    t_init = time.perf_counter()
    g = _ctx(d, cfg, precision, batched, CHAIN_SEEDS[0], 0, warmup + 2 * steps + extra)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t_init       # validation, ordering, partition, CSR/CSC, upload
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
        # propagated rows, once each across the sibling blocks that hold a
        # copy: those some copy factorises (reading the packed FP64 prior) and
        # those some copy with at most LOWRANK_NNZ entries takes on the
        # prior-factor path (FP32/BF16 passes with K > 16)
        fast = precision != "fp64" and d["K"] > 16
        copies, prop, pfac = [0, 0], [0, 0], [0, 0]
        ents = [0, 0]
        parts = [{}, {}]
        for b in range(g.nblocks()):
            info = g.block_info(b)
            if info["stage"] != s:
                continue
            bi, bj = divmod(b, cfg["J"])
            ents[0] += info["R"]
            ents[1] += info["C"]
            for side, is_prop, part in ((0, bj > 0, bi), (1, bi > 0, bj)):
                if is_prop:
                    parts[side].setdefault(part, []).append(np.diff(g.block_csr(b, side)[0]))
        for side in (0, 1):
            for degs in parts[side].values():
                dm = np.stack(degs)
                copies[side] += dm.size
                if fast:
                    prop[side] += int(np.count_nonzero((dm > LOWRANK_NNZ).any(axis=0)))
                    pfac[side] += int(np.count_nonzero((dm <= LOWRANK_NNZ).any(axis=0)))
                else:
                    prop[side] += dm.shape[1]
        say("stage %d timed, %.4f ms per sweep" % (s, ms))
        if s != stages[-1] and extra:
            g.gibbs_sweep(extra)
            torch.cuda.synchronize()
        per_stage[s] = dict(ms_per_step=ms, wall_ms_per_step=1000 * wall / steps,
                            ktimes=ktimes, row_updates=row_updates, ratings=ratings,
                            schedule=g.schedule(), prop_copies=copies, prior_rows=prop,
                            factor_rows=pfac, ents=ents)
    out = dict(per_stage=per_stage, stats=g.stats(), init_s=init_s)
    g.close()
    return out


def run_chains(d, cfg, precision, batched, nchains, trace=""):
    """The configuration's own chain (sweeps per stage, burn-in) for each chain
    seed, and the test RMSE of its posterior-mean prediction (Sec. 5.2)."""
    import torch
    sweeps, burnin = cfg["sweeps"], cfg["burnin"]
    out = []
    for q, seed in enumerate(CHAIN_SEEDS[:nchains]):
        h = _ctx(d, cfg, precision, batched, seed, burnin, sweeps - burnin)
        tf = open(trace, "w") if (trace and q == 0) else None
        t0 = time.perf_counter()
        for s in stages_of(cfg):
            # stage begin (the previous stage's moment matching and prior
            # factors, this stage's initial state) with per-kernel timing;
            # the sweeps run as captured graphs without it
            h.enable_timing(True)
            h.pp_stage(s, 0)
            h.enable_timing(False)
            if tf is None:
                h.gibbs_sweep(sweeps)
            else:
                M = h.stage_work()[1]
                for t in range(sweeps):
                    h.gibbs_sweep(1)
                    st = h.stats()
                    tf.write(json.dumps({"stage": s, "sweep": t, "train_rmse": float(np.sqrt(st["train_sse"] / M)),
                                         "tau_block0": h.get_tau(min(b for b in range(h.nblocks())
                                                                     if h.block_info(b)["stage"] == s)),
                                         "fallback_rows": st["fallback_rows"],
                                         "nonpd_rows": st["nonpd_rows"]}) + "\n")
            torch.cuda.synchronize()
        h.enable_timing(True)
        h.aggregate()                      # the last stage's moment matching, then Algorithm 2
        h.enable_timing(False)
        p = h.predict(d["test_row"], d["test_col"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = h.stats()
        kt = h.kernel_times()
        out.append(dict(seed=seed, rmse=float(np.sqrt(np.mean((p - d["test_val"]) ** 2))), chain_wall_s=wall,
                        mm_ridged=st["mm_ridged"], agg_corrections=st["agg_corrections"],
                        fallback_rows=st["fallback_rows"],
                        stage_end_ms={k: kt[k][1] for k in ("moment_match", "aggregate", "init") if k in kt}))
        if tf is not None:
            tf.close()
        h.close()
        say("%s chain seed %d: rmse %.6f, %.2f s" % (precision, seed, out[-1]["rmse"], wall))
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, cfg, seconds, seed):
    """The FP64 oracle's sweeps on the host cores, bounded in time.  Every PP
    stage is sampled: its blocks are swept in order (each block's full sweep:
    rows, columns, hyperparameter and tau draws) until the stage's share of the
    time budget is used, at least one block per stage.  The propagated priors
    of stages 2 and 3 are placeholders (identity precision, zero mean): the
    oracle's arithmetic per sweep does not depend on their values.  Its whole-job
    rate is the training entries of all blocks over the sum of the per-stage
    sweep times this gives (the same definition as the GPU value).  With all
    host threads, then with one thread on stage 3 alone."""
    from oracle.bpmf import Oracle
    t0 = time.perf_counter()
    o = Oracle(d["N"], d["D"], d["K"], d["row"], d["col"], d["val"], I=cfg["I"], J=cfg["J"],
               order=cfg["order"], seed=seed)
    K = d["K"]
    say("oracle built in %.1f s" % (time.perf_counter() - t0))

    eye = {}

    def placeholder(n):
        # one identity-precision array per size, shared by the blocks that bind it
        if n not in eye:
            eye[n] = (np.zeros((n, K)), np.ascontiguousarray(np.broadcast_to(np.eye(K), (n, K, K))))
        return eye[n]

    def sample(stage, budget, nthreads):
        o.nthreads = nthreads
        if stage > 1:
            for blk in o.blocks:
                if blk["stage"] < stage and blk["b"] not in o.mm:
                    (xm, xl), (wm, wl) = placeholder(blk["R"]), placeholder(blk["C"])
                    o.mm[blk["b"]] = dict(x_mu=xm, x_Lam=xl, w_mu=wm, w_Lam=wl, ridged=0)
        o.begin_stage(stage)
        blocks = o.stage_blocks(stage)
        M = n = nb = 0
        t1 = time.perf_counter()
        for blk in blocks:
            o.sweep_block(blk)
            M += blk["M"]
            n += blk["R"] + blk["C"]
            nb += 1
            if time.perf_counter() - t1 >= budget:
                break
        el = time.perf_counter() - t1
        return dict(stage=stage, blocks=nb, of=len(blocks), ratings=M, row_updates=n, seconds=el,
                    ratings_per_s=M / el, row_updates_per_s=n / el,
                    stage_ratings=sum(b["M"] for b in blocks),
                    stage_row_updates=sum(b["R"] + b["C"] for b in blocks))

    cores = len(os.sched_getaffinity(0))
    stages = stages_of(cfg)
    all_thr = [sample(s, seconds / len(stages), 0) for s in stages]
    t_step = sum(r["stage_ratings"] / r["ratings_per_s"] for r in all_thr)
    M_tot = sum(r["stage_ratings"] for r in all_thr)
    RU_tot = sum(r["stage_row_updates"] for r in all_thr)
    one = sample(stages[-1], seconds / 2, 1)
    desc = "; ".join("stage %d: %d of %d blocks, %d entries, %.1f s" % (r["stage"], r["blocks"], r["of"],
                                                                        r["ratings"], r["seconds"])
                     for r in all_thr)
    return dict(value=M_tot / t_step, unit="ratings/s", cores=cores, kind="oracle",
                row_updates_per_s=RU_tot / t_step, cpu_model=cpu_model(),
                sample="FP64 oracle (C, OpenMP over rows, %d threads) full block sweeps per PP stage of "
                       "the same workload (%s), placeholder propagated priors; whole-job rate = all "
                       "training entries over the summed per-stage sweep times" % (cores, desc),
                per_stage=all_thr,
                single_thread=dict(value=one["ratings_per_s"], unit="ratings/s", cores=1,
                                   row_updates_per_s=one["row_updates_per_s"],
                                   sample="stage %d only: %d of %d blocks, %d entries, %.1f s"
                                          % (one["stage"], one["blocks"], one["of"], one["ratings"],
                                             one["seconds"])))


def pass_rooflines(d, cfg, arm, steps, state_bytes, config_id, precision):
    """Achieved algorithmic bandwidth of every update pass (stage, rows or
    columns) of the per-kernel region: the pass's bytes over its summed
    launch time per sweep (the segment Grams of heavy entities, which serve
    both passes, are charged to each pass, so the rate is a lower bound)."""
    K = d["K"]
    out = []
    for s, m in arm["per_stage"].items():
        kt = m["ktimes"]
        seg_ms = kt.get("gram_segments", (0, 0.0))[1]
        for side, kcls in ((0, "update_rows"), (1, "update_cols")):
            if kcls not in kt or kt[kcls][0] == 0:
                continue
            launches, tot_ms = kt[kcls]
            n = m["ents"][side]
            nbytes = algorithmic_bytes(m["ratings"], n, K, state_bytes, True, m["prior_rows"][side],
                                       m["factor_rows"][side])
            avg_ms = (tot_ms + seg_ms) / steps
            ach = nbytes / (avg_ms / 1000.0) / 1e9
            traffic = measured_traffic(kcls, config_id, s, precision)
            r = dict(kernel="%s (stage %d pass)" % (kcls, s), stage=s, bound="hbm", achieved=ach,
                     peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS, traffic=traffic,
                     avg_launch_ms=avg_ms, launches_per_pass=launches / steps,
                     algorithmic_bytes_per_launch=nbytes, pass_ms_share=avg_ms / m["ms_per_step"])
            if traffic:
                r["traffic_frac"] = traffic / (avg_ms / 1000.0) / 1e9 / HBM_PEAK_GBS
            out.append(r)
    return out


TABLE4_SIM = {1: (1.008, 1.008), 3: (1.008, 1.008), 5: (1.008, 1.008), 10: (1.009, 1.009), 30: (1.018, 1.020)}
TABLE4_SIM_SECONDS_1X1 = 118124.0      # the paper's 1x1 run (R, one node), decreasing order


def paper_sim():
    """Test RMSE and wall-clock of full PP chains on the paper's simulated data
    (K = 5, tau = 1 fixed, 1200 sweeps, 800 burn-in, thin 2), batched BF16,
    under each approximation (moment matching, dominant mode, mixture)."""
    import torch
    import synth
    from paper_1703_00734_amd import BMF
    out = {"metric": "test RMSE and chain wall-clock, paper's simulated workload", "runs": []}
    data = {m: synth.simulated(1, m) for m in ("mar", "structured")}
    for missing, IJ, order, approx in itertools.product(("mar", "structured"), (1, 3, 5, 10, 30),
                                                        ("decreasing", "random"), ("mm", "dm", "gmm")):
        d = data[missing]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = BMF(d["N"], d["D"], 5, d["row"], d["col"], d["val"], I=IJ, J=IJ, order=order,
                sample_tau=False, tau_fixed=1.0, seed=101, burnin=800, thin=2, max_kept=200,
                precision="bf16", batched=True, approx=approx)
        stage_s = {}
        for s in (1, 2, 3):
            ts = time.perf_counter()
            g.pp_stage(s, 1200)
            torch.cuda.synchronize()
            stage_s[s] = time.perf_counter() - ts
        ta = time.perf_counter()
        g.aggregate()
        torch.cuda.synchronize()
        agg_s = time.perf_counter() - ta
        wall = time.perf_counter() - t0
        p = g.predict(d["test_row"], d["test_col"])
        g.close()
        rmse = float(np.sqrt(np.mean((p.astype(np.float64) - d["test_val"]) ** 2)))
        r = dict(missing=missing, partition="%dx%d" % (IJ, IJ), order=order, approx=approx, rmse=rmse,
                 chain_wall_s=wall, stage_s=stage_s, aggregate_s=agg_s, train_entries=int(d["row"].size))
        if missing == "mar":
            r["paper_rmse"] = TABLE4_SIM[IJ][0 if order == "decreasing" else 1]
        out["runs"].append(r)
        say("sim %s %dx%d %s %s: rmse %.5f, %.2f s" % (missing, IJ, IJ, order, approx, rmse, wall))
    out["paper_1x1_seconds"] = TABLE4_SIM_SECONDS_1X1
    print(json.dumps(out))


def main():
    a = parse()
    if a.paper_sim:
        paper_sim()
        return
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
    say("drawing workload %d" % a.config)
    d = synth.config(a.config, seed=a.seed, progress=say)
    K = d["K"]
    main_prec = "bf16" if cfg["precision"] in ("fp32", "bf16") else cfg["precision"]
    state_bytes = {"fp64": 8, "fp32": 4, "bf16": 2}[main_prec]
    stages = stages_of(cfg)
    arms = {"batched_" + main_prec: time_stages(d, cfg, main_prec, True, a.steps, a.warmup)}
    say("arm batched %s timed" % main_prec)
    if main_prec != "fp64" and not a.batched_only:
        arms["plain_fp32"] = time_stages(d, cfg, "fp32", False, a.steps, a.warmup)
        say("arm plain fp32 timed")
    head = arms["batched_" + main_prec]
    ms = sum(head["per_stage"][s]["ms_per_step"] for s in stages)
    ratings = sum(head["per_stage"][s]["ratings"] for s in stages)
    row_updates = sum(head["per_stage"][s]["row_updates"] for s in stages)
    roofs = pass_rooflines(d, cfg, head, a.steps, state_bytes, a.config, main_prec)
    roof = max(roofs, key=lambda r: r["avg_launch_ms"]) if roofs else None
    if roof is not None:
        roof = {k: v for k, v in roof.items() if k != "pass_ms_share"}
    kernel_ms = {}
    for s in stages:
        for k, v in head["per_stage"][s]["ktimes"].items():
            if v[0] > 0:
                kernel_ms["stage%d.%s" % (s, k)] = v[1] / a.steps
    partition = "%dx%d" % (cfg["I"], cfg["J"])
    out = {
        "metric": METRIC,
        "value": ratings / (ms / 1000.0),
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
        "config": {"workload": "%s N=%d D=%d K=%d, %d train entries, Zipf(1.2) degrees, %s partition, %s "
                               "order; step = one sweep of each PP stage (%s)"
                               % ("ratings-shaped" if cfg["kind"] == "ratings" else cfg["kind"],
                                  d["N"], d["D"], K, d["row"].size, partition, cfg["order"],
                                  ", ".join("stage %d" % s for s in stages)),
                   "N": d["N"], "D": d["D"], "K": K, "train_nnz": int(d["row"].size),
                   "partition": partition, "stages": stages},
        "row_updates_per_s": row_updates / (ms / 1000.0),
        "roofline": roof,
        "roofline_passes": roofs,
        "kernel_ms_per_step": kernel_ms,
        "timing": "ms_per_step: per stage, HIP events around `steps` timed sweeps (graph replays in the "
                  "batched arm), summed over the stages; kernel times and roofline: a second region of as "
                  "many sweeps per stage launched eagerly with HIP events around every kernel",
        "arms": {},
    }
    for k, v in arms.items():
        t_arm = sum(v["per_stage"][s]["ms_per_step"] for s in stages)
        arm = {"ms_per_step": t_arm, "ratings_per_s": ratings / (t_arm / 1000.0),
               "row_updates_per_s": row_updates / (t_arm / 1000.0),
               "fallback_rows": v["stats"]["fallback_rows"], "init_s": v["init_s"], "stages": {}}
        for s_, ps in v["per_stage"].items():
            arm["stages"][str(s_)] = {
                "ms_per_step": ps["ms_per_step"], "ratings": ps["ratings"], "row_updates": ps["row_updates"],
                "ratings_per_s": ps["ratings"] / (ps["ms_per_step"] / 1000.0),
                "row_updates_per_s": ps["row_updates"] / (ps["ms_per_step"] / 1000.0),
                "schedule": ps["schedule"]}
        out["arms"][k] = arm
    if "plain_fp32" in arms:
        out["speedup_vs_plain_fp32"] = out["arms"]["plain_fp32"]["ms_per_step"] / ms
    if not a.no_rmse:
        rm = {}
        for k in arms:
            prec = main_prec if k.startswith("batched") else "fp32"
            rm[k] = run_chains(d, cfg, prec, k.startswith("batched"), a.chains,
                               a.trace if k.startswith("batched") else "")
            out["arms"][k]["chains"] = rm[k]
            out["arms"][k]["test_rmse"] = float(np.mean([c["rmse"] for c in rm[k]]))
        if "plain_fp32" in rm:
            r0 = out["arms"]["batched_" + main_prec]["test_rmse"]
            r1 = out["arms"]["plain_fp32"]["test_rmse"]
            out["equal_rmse"] = {"relative_difference": abs(r0 - r1) / r1, "bound": 0.005,
                                 "holds": abs(r0 - r1) / r1 <= 0.005,
                                 "chains_per_arm": a.chains}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(d, cfg, a.cpu_seconds, CHAIN_SEEDS[0])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
