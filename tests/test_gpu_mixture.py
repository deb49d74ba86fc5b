"""Dominant-mode and mixture approximations on the GPU against the oracle
(needs an MI355X).

Sec. 4.1 and Sec. 5.1: each row's kept samples are clustered by lambda-means;
the dominant-mode fit moment-matches the largest cluster, the mixture keeps the
three largest clusters as weighted components, a row under a mixture prior
takes the component of largest responsibility at its current value every
sweep, and aggregation uses the pooled mixture moments (Sec. 4.2, eq.
marginal_mixture).  The labels are compared bit for bit (both sides take every
decision in FP64 with the same operations in the same order), the fits to FP64
rounding, FP64 chains of all three stages to the oracle's with identical
noise, and FP32/BF16 chains by their test RMSE.
"""
import numpy as np
import pytest

from gpu_helpers import pair, small_data
from oracle import native
from oracle.bpmf import LMEANS_CMAX, LMEANS_MAXIT
from oracle.native import ptr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _labels_oracle(smp, scale):
    S, R, K = smp.shape
    lab = np.zeros((R, S), dtype=np.int32)
    ncl = np.zeros(R, dtype=np.int32)
    native.lib().orc_lmeans(R, K, S, ptr(np.ascontiguousarray(smp)), scale, LMEANS_CMAX, LMEANS_MAXIT,
                            ptr(lab), ptr(ncl))
    return lab


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("precision,K,approx", [("fp64", 4, "dm"), ("fp64", 6, "gmm"), ("fp32", 12, "gmm"),
                                                ("bf16", 20, "gmm"), ("bf16", 32, "dm"), ("fp32", 32, "gmm")])
def test_clusters_and_fits_match_oracle(precision, K, approx):
    """Stage 1 of a 2 x 2 partition: the library's lambda-means labels of its own
    kept samples equal the oracle's bit for bit, and its dominant-mode or
    mixture fit (weights, means, precisions, log-determinants, pooled moments)
    matches the oracle's fit of the same samples."""
    d = small_data(K, seed=5, N=300, D=200, nnz=9000, empty_rows=3)
    S, scale = 40, 1.5
    print("case", precision, K, approx, flush=True)
    g, o = pair(d, K, precision, I=2, J=2, order="random", burnin=5, max_kept=S, approx=approx,
                lambda_scale=scale)
    g.pp_stage(1, 5 + S)
    smps = [np.stack([g.get_sample(0, side, q) for q in range(S)]) for side in (0, 1)]
    g.pp_stage(2, 0)                       # finalises stage 1
    multi = 0
    for side in (0, 1):
        smp = smps[side]
        lab = g.get_clusters(0, side, S)
        np.testing.assert_array_equal(lab, _labels_oracle(smp, scale))
        multi += int((lab.max(1) > 0).sum())
        fit = o.cluster_fit(np.ascontiguousarray(smp))
        mu, Lam = g.get_mm(0, side)
        assert _rel(mu, fit["mu"]) < 1e-9
        assert _rel(Lam, fit["Lam"]) < 1e-7
        if approx == "gmm":
            for c in range(3):
                comp = g.get_component(0, side, c)
                np.testing.assert_array_equal(comp["pi"], fit["pi"][:, c])
                on = fit["pi"][:, c] > 0
                assert _rel(comp["mu"][on], fit["cmu"][on, c]) < 1e-9
                assert _rel(comp["Lam"][on], fit["cLam"][on, c]) < 1e-7
                np.testing.assert_allclose(comp["logdet"][on], fit["logdet"][on, c], rtol=1e-9, atol=1e-9)
        else:
            comp = g.get_component(0, side, 0)
            np.testing.assert_allclose(comp["logdet"], np.linalg.slogdet(fit["Lam"])[1], rtol=1e-9, atol=1e-9)
    print("rows with more than one cluster:", multi, flush=True)
    assert multi > 0
    g.close()


@pytest.mark.parametrize("approx,IJ,order,K,sweeps", [("dm", (2, 2), "random", 6, 12),
                                                      ("gmm", (2, 2), "random", 6, 12),
                                                      ("gmm", (3, 2), "decreasing", 5, 12),
                                                      ("dm", (2, 3), "random", 17, 40),
                                                      ("gmm", (2, 2), "random", 17, 40)])
def test_fp64_pp_stages_track_oracle(approx, IJ, order, K, sweeps):
    """Stages 1-3 in FP64 with identical noise: every block's labels equal the
    oracle's, its fits agree, the mixture picks (which decide each row's
    prior every sweep) keep the chains together, and Algorithm 2 with its
    eigenvalue corrections gives the oracle's predictions."""
    d = small_data(K, seed=7, N=300, D=200, nnz=12000, empty_rows=0)
    I, J = IJ
    print("case", approx, IJ, order, K, sweeps, flush=True)
    g, o = pair(d, K, "fp64", I=I, J=J, order=order, burnin=2, thin=1, max_kept=sweeps, approx=approx,
                lambda_scale=1.5)
    for s in (1, 2, 3):
        g.pp_stage(s, sweeps)
        if o.stage_blocks(s):
            o.run_stage(s, sweeps)
    S = sweeps - 2
    pg = g.predict(d["test_row"], d["test_col"])      # finalises the last stage
    for b in range(I * J):
        for side, key in ((0, "x"), (1, "w")):
            np.testing.assert_array_equal(g.get_clusters(b, side, S), o.mm[b][key + "_labels"])
            mg, Lg = g.get_mm(b, side)
            np.testing.assert_allclose(mg, o.mm[b][key + "_mu"], rtol=1e-6, atol=1e-7)
            np.testing.assert_allclose(Lg, o.mm[b][key + "_Lam"], rtol=1e-4, atol=1e-4)
    o.aggregate()
    po = o.predict(d["test_row"], d["test_col"])
    print("aggregation corrections: gpu", g.stats()["agg_corrections"], "oracle", o.corrections)
    assert g.stats()["agg_corrections"] == o.corrections
    np.testing.assert_allclose(pg, po, rtol=1e-5, atol=1e-5)
    g.close()


@pytest.mark.parametrize("precision,approx", [("bf16", "gmm"), ("fp32", "dm"), ("bf16", "dm")])
def test_pp_chain_rmse_matches_oracle(precision, approx):
    """A 2 x 2 PP chain under the dominant-mode or mixture approximation: test
    RMSE within 0.5 % of the oracle's chains (mean of 3 seeds)."""
    import synth
    K = 10
    d = synth.make("ratings", 3000, 1500, K, 300000, 0.8, 6)
    rg, ro = [], []
    for seed in (201, 202, 203):
        g, o = pair(d, K, precision, I=2, J=2, order="random", seed=seed, burnin=15, max_kept=25, approx=approx)
        for s in (1, 2, 3):
            g.pp_stage(s, 40)
            o.run_stage(s, 40)
        pg = g.predict(d["test_row"], d["test_col"])
        o.aggregate()
        po = o.predict(d["test_row"], d["test_col"])
        rg.append(np.sqrt(np.mean((pg - d["test_val"]) ** 2)))
        ro.append(np.sqrt(np.mean((po - d["test_val"]) ** 2)))
        assert g.stats()["nonpd_rows"] == 0
        g.close()
    print(approx, precision, "pp rmse gpu", rg, "oracle", ro)
    assert abs(np.mean(rg) - np.mean(ro)) <= 0.005 * np.mean(ro)


def test_checkpoint_resume_under_mixture_priors(tmp_path):
    """A mixture-propagated stage stopped after a checkpoint and resumed in a
    fresh context gives the uninterrupted chain's prediction bit for bit (a
    fixed lane-group size: the autotuner's timed choice may differ between
    runs, and with it the order of the FP32 sums)."""
    K = 6
    d = small_data(K, seed=9, N=200, D=150, nnz=6000, empty_rows=0)
    g, _ = pair(d, K, "fp32", I=2, J=2, order="random", seed=3, burnin=2, max_kept=10, approx="gmm",
                lambda_scale=1.5, lane_nnz=16)
    for s in (1, 2, 3):
        g.pp_stage(s, 12)
    want = g.predict(d["test_row"], d["test_col"])
    g.close()
    g, _ = pair(d, K, "fp32", I=2, J=2, order="random", seed=3, burnin=2, max_kept=10, approx="gmm",
                lambda_scale=1.5, lane_nnz=16)
    g.pp_stage(1, 12)
    g.pp_stage(2, 12)
    g.pp_stage(3, 5)
    path = str(tmp_path / "gmm.ckpt")
    g.save_state(path)
    g.close()
    h, _ = pair(d, K, "fp32", I=2, J=2, order="random", seed=3, burnin=2, max_kept=10, approx="gmm",
                lambda_scale=1.5, lane_nnz=16)
    h.load_state(path)
    h.gibbs_sweep(7)
    got = h.predict(d["test_row"], d["test_col"])
    h.close()
    np.testing.assert_array_equal(got, want)
