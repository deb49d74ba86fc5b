"""GPU parity at the benchmark workloads' full sizes (needs an MI355X).

One batched BF16 sweep of the first stage's block, replayed from the captured
graph with the schedule the autotuner picks at stage begin (the launch
configuration bench.py times), from a state loaded identically into the
library and the oracle: every row and column the sweep draws, and the
Normal-Wishart and tau draws that close it, against the oracle's conditional
draws with the same Philox noise.
"""
import numpy as np
import pytest

from gpu_helpers import load_state, pair, random_state, round_state

pytestmark = pytest.mark.gpu

# the state is stored in BF16: the oracle's FP64 draw is compared after the same
# rounding, so a row may differ by the BF16 rounding of both draws (2^-8
# relative per entry) on top of the BF16-Gram error of one step (3e-3)
TOL_STATE = 1.2e-2


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(x_gpu, x_or):
    """||dx_n|| / max(||x_n||, a tenth of the median row norm) per row."""
    nrm = np.linalg.norm(x_or, axis=1)
    den = np.maximum(nrm, 0.1 * np.median(nrm))
    return np.linalg.norm(x_gpu - x_or, axis=1) / den


@pytest.mark.parametrize("cid", [2, 3, 4])
def test_full_size_sweep_matches_oracle(cid):
    import synth
    cfg = synth.CONFIGS[cid]
    print("case: full-size workload", cid, flush=True)
    d = synth.config(cid, seed=1)
    K = d["K"]
    g, o = pair(d, K, "bf16", I=cfg["I"], J=cfg["J"], order=cfg["order"], seed=101, max_kept=1)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    assert g.block_info(0)["stage"] == 1
    st = random_state(np.random.default_rng(70 + cid), blk["R"], blk["C"], K)
    load_state(g, o, 0, st)
    print("schedule", g.schedule(), "rows", blk["R"], "cols", blk["C"], flush=True)
    g.gibbs_sweep(1)                         # sweep 0, batched and graph-captured
    s = g.get_state(0)
    # rows from the loaded state
    o.update_rows(blk, 0)
    rel = _rel(s["X"], round_state(blk["X"], "bf16"))
    print("rows: max rel", rel.max(), "p99.9", np.quantile(rel, 0.999), flush=True)
    assert rel.max() <= TOL_STATE
    # columns from the library's new rows (the values its column pass read)
    blk["X"] = s["X"].copy()
    o.update_cols(blk, 0)
    rel = _rel(s["W"], round_state(blk["W"], "bf16"))
    print("cols: max rel", rel.max(), "p99.9", np.quantile(rel, 0.999), flush=True)
    assert rel.max() <= TOL_STATE
    # Normal-Wishart draws from the library's state, then tau
    blk["W"] = s["W"].copy()
    o.hyper_draw(blk, "x", 0)
    o.hyper_draw(blk, "w", 0)
    for key in ("hx", "hw"):
        np.testing.assert_allclose(s[key][0], blk[key][0], rtol=1e-6, atol=1e-9 * np.abs(blk[key][0]).max())
        np.testing.assert_allclose(s[key][1], blk[key][1], rtol=1e-6, atol=1e-9)
    o.tau_draw(blk, 0)
    np.testing.assert_allclose(s["tau"], blk["tau"], rtol=1e-4)
    stats = g.stats()
    assert stats["nonpd_rows"] == 0
    g.close()


def test_full_size_stage3_sweep_matches_oracle():
    """The 480k x 17.8k, K = 32 workload on its 8 x 8 partition: stages 1 and 2
    run with 2K + 2 kept samples, then one batched, graph-replayed sweep of
    stage 3, which takes every update kernel: the prior-factor path (rows
    without entries), the low-rank path (one to eight entries), the
    two-per-wavefront kernel and the MFMA wavefront kernel.  Block (7, 7), of
    the sparsest rows and columns (decreasing order), is checked against the
    oracle's conditional draws under the library's own moment-matched priors
    (rows: block (7, 0)'s, columns: block (0, 7)'s), from a state loaded into
    both, with the same noise."""
    import synth
    cfg = synth.CONFIGS[5]
    print("case: full-size workload 5, stage 3", flush=True)
    d = synth.config(5, seed=1, progress=lambda m: print("data:", m, flush=True))
    K = d["K"]
    S = 2 * K + 2
    g, o = pair(d, K, "bf16", I=cfg["I"], J=cfg["J"], order=cfg["order"], seed=101, max_kept=S)
    print("library and oracle built", flush=True)
    g.pp_stage(1, S)
    g.pp_stage(2, S)
    g.pp_stage(3, 0)
    print("stages 1 and 2 done", flush=True)
    I, J = cfg["I"], cfg["J"]
    b = (I - 1) * J + (J - 1)
    assert g.block_info(b)["stage"] == 3
    mx, Lx = g.get_mm((I - 1) * J + 0, 0)
    mw, Lw = g.get_mm(0 * J + (J - 1), 1)
    blk = o.blocks[b]
    blk["x_prior"] = (Lx, mx)
    blk["w_prior"] = (Lw, mw)
    deg = np.diff(blk["csr_ptr"])
    print("rows", blk["R"], "cols", blk["C"], "empty rows", int((deg == 0).sum()), "rows with 1-8 entries",
          int(((deg >= 1) & (deg <= 8)).sum()), flush=True)
    assert (deg == 0).sum() > 1000 and ((deg >= 1) & (deg <= 8)).sum() > 1000
    st = random_state(np.random.default_rng(75), blk["R"], blk["C"], K)
    load_state(g, o, b, st)
    g.gibbs_sweep(1)                         # sweep 0 of stage 3, batched and graph-captured
    s = g.get_state(b)
    o.update_rows(blk, 0)
    rel = _rel(s["X"], round_state(blk["X"], "bf16"))
    print("rows: max rel", rel.max(), "p99.9", np.quantile(rel, 0.999), flush=True)
    assert rel.max() <= TOL_STATE
    blk["X"] = s["X"].copy()
    o.update_cols(blk, 0)
    rel = _rel(s["W"], round_state(blk["W"], "bf16"))
    print("cols: max rel", rel.max(), "p99.9", np.quantile(rel, 0.999), flush=True)
    assert rel.max() <= TOL_STATE
    blk["W"] = s["W"].copy()
    o.tau_draw(blk, 0)
    np.testing.assert_allclose(s["tau"], blk["tau"], rtol=1e-4)
    assert g.stats()["nonpd_rows"] == 0
    g.close()
