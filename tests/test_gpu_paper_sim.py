"""The paper's simulated workload on the GPU path (needs an MI355X).

Sec. 5.3's simulated data (6040 x 3706, K = 5, standard-normal factors and
noise, tau = 1 fixed, 80 % of the cells missing at random and used as the test
set) with the paper's schedule (1200 sweeps, 800 burn-in, every second sweep
kept: 200 samples per stage; Sec. 5.2), partitions 1x1 to 30x30 in random and
decreasing order, through the batched BF16 path: the test RMSE of the
posterior-mean prediction lies within 0.01 of the published value (Table 4,
averaged there over 5 data sets) at 1x1 to 10x10.  At 1x1 and 3x3 the FP64
oracle runs the same chain on the host cores, and both GPU arms (batched BF16,
plain FP32 per block) land within 0.5 % of its RMSE.

At 30x30 the stage-1 block is 202 x 124 with about 5,000 entries, and moment
matching propagates whatever that short-data chain visits in its kept window:
over ten chain seeds of the paper's schedule, four (random order) and five
(decreasing order) end within 0.01 of Table 4 and the others between 1.29 and
1.69 (the frame of the stage-1 block moves during the kept sweeps, and the
broadened priors let the stage-2 blocks settle in frames that disagree).  The
oracle shows the same for the same chain (sim30_oracle_rmse.txt, written by
make_sim30_oracle.py): a 30x30 test checks the FP64 GPU chain against the
oracle's RMSE and correction count for two such chains.  The mixture
approximation reproduces Table 4 at 30x30 (mean over 5 simulated data sets,
as the paper averages 5 runs on 5 data sets).
"""
import os

import numpy as np
import pytest

import synth
from paper_1703_00734_amd import BMF

pytestmark = pytest.mark.gpu

PARTS = [1, 3, 5, 10]
SWEEPS, BURNIN, THIN = 1200, 800, 2


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def sim():
    return synth.simulated(1, "mar")


def _table4(golden_dir):
    out = {}
    for l in open(os.path.join(golden_dir, "table4_simulated_rmse.txt")):
        if l.startswith("#") or not l.strip():
            continue
        p, dec, rnd = l.split()
        out[int(p)] = {"decreasing": float(dec), "random": float(rnd)}
    return out


def _gpu_run(d, IJ, order, precision="bf16", batched=True, seed=101, approx="mm"):
    g = BMF(d["N"], d["D"], 5, d["row"], d["col"], d["val"], I=IJ, J=IJ, order=order, sample_tau=False,
            tau_fixed=1.0, seed=seed, burnin=BURNIN, thin=THIN, max_kept=(SWEEPS - BURNIN) // THIN,
            precision=precision, batched=batched, approx=approx)
    for s in (1, 2, 3):
        g.pp_stage(s, SWEEPS)
    p = g.predict(d["test_row"], d["test_col"])
    st = g.stats()
    g.close()
    assert st["nonpd_rows"] == 0 and st["mm_ridged"] == 0
    return float(np.sqrt(np.mean((p.astype(np.float64) - d["test_val"]) ** 2))), st


def _gpu_rmse(d, IJ, order, precision="bf16", batched=True):
    return _gpu_run(d, IJ, order, precision, batched)[0]


@pytest.mark.parametrize("order", ["random", "decreasing"])
@pytest.mark.parametrize("IJ", PARTS)
def test_paper_schedule_rmse_in_table4_band(sim, golden_dir, IJ, order):
    want = _table4(golden_dir)[IJ][order]
    rmse = _gpu_rmse(sim, IJ, order)
    print("%dx%d %s: gpu rmse %.5f, paper %.3f" % (IJ, IJ, order, rmse, want), flush=True)
    assert abs(rmse - want) <= 0.01


@pytest.mark.parametrize("order", ["random", "decreasing"])
def test_30x30_mixture_approximation_in_table4_band(golden_dir, order):
    """At 30x30 the mixture approximation (lambda-means, three components, the
    component of largest responsibility as each row's prior; Sec. 5.1) keeps
    the frames of the stage-1 chain apart instead of averaging over them.  As in
    the paper (5 independent simulated data sets, results averaged over the 5
    runs; Sec. 5.3 and Sec. 5.2), one chain on each of 5 data sets: their mean
    test RMSE lies within 0.01 of Table 4."""
    want = _table4(golden_dir)[30][order]
    got = []
    for dseed in (1, 2, 3, 4, 5):
        d = synth.simulated(dseed, "mar")
        got.append(_gpu_run(d, 30, order, approx="gmm")[0])
        print("30x30 %s data set %d: gpu gmm rmse %.5f, paper %.3f" % (order, dseed, got[-1], want), flush=True)
    print("mean %.5f" % np.mean(got), flush=True)
    assert abs(np.mean(got) - want) <= 0.01


@pytest.mark.parametrize("IJ", [1, 3])
def test_gpu_rmse_within_half_percent_of_oracle(sim, IJ):
    from oracle.bpmf import Oracle
    d = sim
    o = Oracle(d["N"], d["D"], 5, d["row"], d["col"], d["val"], I=IJ, J=IJ, order="random",
               sample_tau=False, tau_fixed=1.0, seed=101, burnin=BURNIN, thin=THIN)
    o.run_pp(SWEEPS)
    o.aggregate()
    p = o.predict(d["test_row"], d["test_col"])
    want = float(np.sqrt(np.mean((p - d["test_val"]) ** 2)))
    for precision, batched in (("bf16", True), ("fp32", False)):
        got = _gpu_rmse(d, IJ, "random", precision, batched)
        print("%dx%d: oracle rmse %.5f, gpu %s %.5f" % (IJ, IJ, want, precision, got), flush=True)
        assert abs(got - want) <= 0.005 * want


def test_30x30_paper_schedule_equals_oracle(sim, golden_dir):
    """30x30, random order, the paper's schedule, FP64 on the GPU: the RMSE and the
    number of Algorithm 2 eigenvalue corrections of the oracle's chain for the
    same seed (identical noise), for one chain seed whose propagated priors
    broaden (RMSE far outside Table 4's 1.020) and one that stays within 0.01."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "sim30_oracle_rmse.txt")) if not l.startswith("#")]
    want = _table4(golden_dir)[30]["random"]
    for seed, rmse_o, corr_o in rows:
        rmse, st = _gpu_run(sim, 30, "random", "fp64", True, int(seed))
        print("30x30 random seed %s: gpu fp64 rmse %.6f (corrections %d), oracle %s (%s), paper %.3f"
              % (seed, rmse, st["agg_corrections"], rmse_o, corr_o, want), flush=True)
        assert abs(rmse - float(rmse_o)) <= 1e-5 * float(rmse_o)
        assert st["agg_corrections"] == int(corr_o)


def test_structured_missingness_equals_oracle():
    """The second simulated scenario of Sec. 5.3 (structured missingness: cell
    (n, d) observed with probability w_n w_d, weights equally spaced from 0.9
    down to 0.005, so that the densest rows and columns come first), at one
    fifth of the paper's rows and columns, partitioned 3 x 3 in decreasing
    order of observations (the paper's remedy for non-random missingness,
    Sec. 6) with a shortened schedule (400 sweeps, 200 burn-in, every second
    kept).  The paper gives this scenario only as a figure, so the check is
    against the oracle's chain with the same seed: the FP64 GPU chain's test
    RMSE equals it to 1e-5, and both GPU arms (batched BF16, plain FP32 per
    block) land within 0.5 % of it."""
    from oracle.bpmf import Oracle
    d = synth.simulated(2, "structured", N=1208, D=741)
    sweeps, burnin, thin = 400, 200, 2

    def gpu(precision, batched):
        g = BMF(d["N"], d["D"], 5, d["row"], d["col"], d["val"], I=3, J=3, order="decreasing", sample_tau=False,
                tau_fixed=1.0, seed=101, burnin=burnin, thin=thin, max_kept=(sweeps - burnin) // thin,
                precision=precision, batched=batched)
        for s in (1, 2, 3):
            g.pp_stage(s, sweeps)
        p = g.predict(d["test_row"], d["test_col"])
        g.close()
        return float(np.sqrt(np.mean((p.astype(np.float64) - d["test_val"]) ** 2)))

    o = Oracle(d["N"], d["D"], 5, d["row"], d["col"], d["val"], I=3, J=3, order="decreasing",
               sample_tau=False, tau_fixed=1.0, seed=101, burnin=burnin, thin=thin)
    o.run_pp(sweeps)
    o.aggregate()
    p = o.predict(d["test_row"], d["test_col"])
    want = float(np.sqrt(np.mean((p - d["test_val"]) ** 2)))
    got64 = gpu("fp64", True)
    print("structured 3x3 decreasing: oracle rmse %.6f, gpu fp64 %.6f" % (want, got64), flush=True)
    assert abs(got64 - want) <= 1e-5 * want
    for precision, batched in (("bf16", True), ("fp32", False)):
        got = gpu(precision, batched)
        print("structured 3x3 decreasing: gpu %s %.6f" % (precision, got), flush=True)
        assert abs(got - want) <= 0.005 * want
