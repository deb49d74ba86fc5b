"""Invariants of the method checked on the GPU path through the C ABI.

* A one-block partition makes PP's first stage plain BPMF (Theorem 1): a chain
  run as bmf_pp_stage(1) equals the same chain run by bmf_gibbs_sweep, state
  and predictions bit for bit, in every precision, and the aggregated
  posterior mean (Algorithm 2 with no siblings) is the mean of the kept
  samples.
* Every conditional precision the sampler forms is positive definite: no row
  fails its FP64 Cholesky in a PP chain whose propagated priors come from few
  kept samples (ridged moment matching), and the FP32 pivot test sends rows to
  the FP64 redo rather than dropping them.
"""
import numpy as np
import pytest

from gpu_helpers import pair, small_data

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision,K", [("fp64", 10), ("fp32", 10), ("bf16", 10), ("bf16", 32)])
def test_one_block_pp_stage_is_plain_bpmf(precision, K):
    print("case 1x1", precision, K, flush=True)
    d = small_data(K, seed=30 + K)
    a, _ = pair(d, K, precision, burnin=4, max_kept=8, lane_nnz=16)
    b, _ = pair(d, K, precision, burnin=4, max_kept=8, lane_nnz=16)
    a.pp_stage(1, 12)
    b.gibbs_sweep(12)
    sa, sb = a.get_state(0), b.get_state(0)
    for key in ("X", "W", "tau"):
        assert np.array_equal(sa[key], sb[key]), key
    pa = a.predict(d["test_row"], d["test_col"])
    pb = b.predict(d["test_row"], d["test_col"])
    assert np.array_equal(pa, pb)
    # Algorithm 2 without siblings: the kept-sample mean (given order: local ids
    # are the original ids)
    for side in (0, 1):
        mean = np.mean([a.get_sample(0, side, q) for q in range(8)], axis=0)
        np.testing.assert_allclose(a.get_aggregate(side), mean, rtol=1e-12, atol=1e-13)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_conditional_precisions_stay_positive_definite(precision):
    K = 24
    d = small_data(K, seed=9, N=500, D=260, nnz=6000, kind="uniform")
    g, _ = pair(d, K, precision, I=2, J=2, order="random", max_kept=6, pivot_theta=0.5)
    for s in (1, 2, 3):
        g.pp_stage(s, 6)                      # 6 <= K kept samples: ridged priors
    st = g.stats()
    print(precision, st, flush=True)
    assert st["mm_ridged"] > 0
    assert st["nonpd_rows"] == 0
    if precision != "fp64":
        assert st["fallback_rows"] > 0        # the strict pivot test sends rows to the FP64 redo
    p = g.predict(d["test_row"], d["test_col"])
    assert np.all(np.isfinite(p))
    g.close()


@pytest.mark.parametrize("precision,K", [("fp32", 10), ("bf16", 10), ("fp32", 32)])
def test_per_block_sweeps_equal_batched_with_fp64_redo(precision, K):
    """The plain per-block launches and the batched graph give the same chain
    bit for bit through all three stages, also when many rows take the FP64
    redo (propagated priors from fewer kept samples than K are ridged and
    badly conditioned): each block's redo takes only its own pass's rows."""
    print("case per-block redo", precision, K, flush=True)
    d = small_data(K, seed=40 + K, N=700, D=330, nnz=24000)
    runs = []
    for batched in (True, False):
        g, _ = pair(d, K, precision, I=2, J=3, order="decreasing", batched=batched, burnin=2,
                    max_kept=6, lane_nnz=16)
        for s in (1, 2, 3):
            g.pp_stage(s, 8)
        st = g.stats()
        assert st["fallback_rows"] > 0 and st["nonpd_rows"] == 0
        runs.append((g.predict(d["test_row"], d["test_col"]), g.get_state(4), st))
        g.close()
    (pa, sa, ta), (pb, sb, tb) = runs
    assert np.array_equal(pa, pb)
    for key in ("X", "W", "tau"):
        assert np.array_equal(sa[key], sb[key]), key
    assert ta["fallback_rows"] == tb["fallback_rows"]
