"""Abort, checkpoint and resume through the C ABI (needs an MI355X).

The progress callback stops a PP chain before a chosen sweep (BMF_EABORT); the
state is saved to a file, loaded into a fresh context, and the chain is
finished there.  Every draw is addressed by its Philox counter and every
reduction has a fixed order, so the resumed chain must equal the uninterrupted
one bit for bit: states, moment-matched priors, counters and predictions.
"""
import numpy as np
import pytest

from gpu_helpers import pair, small_data
from paper_1703_00734_amd import BMFError

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ctx(d, K, precision, batched):
    g, _ = pair(d, K, precision, I=2, J=3, order="decreasing", batched=batched, burnin=4,
                max_kept=10, lane_nnz=16)
    return g


def _finish(g, d):
    out = {"pred": g.predict(d["test_row"], d["test_col"]), "stats": g.stats()}
    for b in range(g.nblocks()):
        if g.block_info(b)["stage"] == 3:
            s = g.get_state(b)
            out[b] = (s["X"], s["W"], s["tau"])
    out["mm"] = g.get_mm(4, 0)
    return out


@pytest.mark.parametrize("precision,K", [("fp64", 6), ("fp32", 10), ("bf16", 10), ("bf16", 24),
                                         ("fp32", 32)])
@pytest.mark.parametrize("stop", [(2, 5), (3, 0), (3, 9)])
def test_abort_save_load_resume_is_bit_identical(tmp_path, precision, K, stop):
    print("case checkpoint", precision, K, stop, flush=True)
    d = small_data(K, seed=20 + K, N=700, D=330, nnz=24000)
    S = 14
    ref = _ctx(d, K, precision, True)
    for s in (1, 2, 3):
        ref.pp_stage(s, S)
    want = _finish(ref, d)
    ref.close()

    g = _ctx(d, K, precision, True)
    g.set_progress(lambda stage, sweep: (stage, sweep) == stop)
    stage_stop, sweep_stop = stop
    for s in (1, 2, 3):
        if s < stage_stop:
            g.pp_stage(s, S)
        else:
            with pytest.raises(BMFError) as e:
                g.pp_stage(s, S)
            assert e.value.status == "BMF_EABORT"
            break
    path = str(tmp_path / "chain.ckpt")
    g.save_state(path)
    g.close()

    # resume in a fresh context (per-block launches: the launch form does not
    # change the values)
    h = _ctx(d, K, precision, precision != "fp32")
    h.load_state(path)
    h.gibbs_sweep(S - sweep_stop)
    for s in range(stage_stop + 1, 4):
        h.pp_stage(s, S)
    got = _finish(h, d)
    h.close()
    assert np.array_equal(want["pred"], got["pred"])
    for key in want:
        if isinstance(key, int):
            for a, b in zip(want[key], got[key]):
                assert np.array_equal(a, b), key
    assert np.array_equal(want["mm"][0], got["mm"][0]) and np.array_equal(want["mm"][1], got["mm"][1])
    for k in ("nonpd_rows", "mm_ridged", "agg_corrections", "train_sse"):
        assert want["stats"][k] == got["stats"][k], k


def test_checkpoint_refused_by_another_configuration(tmp_path):
    K = 6
    d = small_data(K, seed=3)
    g = _ctx(d, K, "fp32", True)
    g.pp_stage(1, 3)
    path = str(tmp_path / "a.ckpt")
    g.save_state(path)
    g.close()
    other = dict(d)
    other["val"] = d["val"] + np.float32(1.0)                 # same shapes, other values
    h = _ctx(other, K, "fp32", True)
    with pytest.raises(BMFError) as e:
        h.load_state(path)
    assert e.value.status == "BMF_EINVAL" and "training data" in str(e.value)
    h.close()
    h = _ctx(d, K, "fp64", True)
    with pytest.raises(BMFError) as e:
        h.load_state(path)
    assert e.value.status == "BMF_EINVAL"
    h.close()
    with open(path, "r+b") as f:                               # truncated file
        f.truncate(4096)
    h = _ctx(d, K, "fp32", True)
    with pytest.raises(BMFError) as e:
        h.load_state(path)
    assert e.value.status == "BMF_EINVAL"
    h.close()


def test_train_sse_matches_residuals():
    """bmf_get_stats' train_sse equals the residual sum of squares of the state
    the last sweep left (fixed tau: the statistic is still evaluated)."""
    K = 10
    d = small_data(K, seed=5)
    for sample_tau in (True, False):
        g, o = pair(d, K, "fp64", sample_tau=sample_tau, tau_fixed=2.0, max_kept=2)
        g.gibbs_sweep(3)
        s = g.get_state(0)
        o.begin_stage(1)
        blk = o.blocks[0]
        blk["X"], blk["W"] = s["X"], s["W"]
        want = o.sse(blk)
        got = g.stats()["train_sse"]
        assert got == pytest.approx(want, rel=1e-10)
        g.close()
