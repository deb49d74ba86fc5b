"""Per-column noise precisions on the GPU against the oracle (needs an MI355X).

The tau_d variant of Sec. 2.1: y_nd ~ N(x_n^T w_d, 1/tau_d) with one Gamma
tau_d per column of each block.  The library's row pass reads sqrt(tau_d) w_d
and sqrt(tau_d) r_nd (formed at the start of each sweep), its column pass and
closed-form column SSE use the column's own tau_d, and every tau_d is drawn from
its Gamma posterior after the column pass.  Checked step by step from loaded
states (the draws of the tau_d, then a row pass and a column pass under those
tau_d), as FP64 three-stage chains with identical noise, by the FP32 chain's
test RMSE, and as bit-identical batched and per-block runs.
"""
import numpy as np
import pytest

from gpu_helpers import TOL, load_state, pair, random_state, small_data

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel_rows(a, b):
    return (np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-3)).max()


@pytest.mark.parametrize("precision,K", [("fp64", 6), ("fp32", 10), ("fp32", 24), ("fp64", 33)])
def test_steps_under_column_precisions(precision, K):
    print("case", precision, K, flush=True)
    d = small_data(K, seed=30 + K)
    g, o = pair(d, K, precision, tau_per_column=True)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    st = random_state(np.random.default_rng(200 + K), blk["R"], blk["C"], K, scale=0.4)
    load_state(g, o, 0, st)
    blk["tau"] = np.full(blk["C"], o.a0 / o.b0)
    t = 3
    g.step(0, "tau", t)
    o.tau_draw(blk, t)
    tg = g.get_tau_cols(0)
    np.testing.assert_allclose(tg, blk["tau"], rtol=1e-10 if precision == "fp64" else 1e-5)
    assert tg.std() > 0.05 * tg.mean()                 # the columns' precisions differ
    blk["tau"] = tg.copy()                            # the same tau_d on both sides from here
    for which in ("rows", "cols"):
        g.step(0, which, t + 1)
        getattr(o, "update_" + which)(blk, t + 1)
        key = "X" if which == "rows" else "W"
        rel = _rel_rows(g.get_draw(0, 0 if which == "rows" else 1), blk[key])
        print(which, "max rel", rel, flush=True)
        assert rel <= TOL[precision] * 10
        # continue both sides from the library's stored state
        blk[key] = g.get_state(0)[key]
    g.close()


@pytest.mark.parametrize("IJ,order,K", [((2, 2), "random", 6), ((3, 2), "decreasing", 12)])
def test_fp64_pp_stages_track_oracle(IJ, order, K):
    d = small_data(K, seed=7, N=300, D=200, nnz=12000, empty_rows=0)
    I, J = IJ
    sweeps = 10
    g, o = pair(d, K, "fp64", I=I, J=J, order=order, burnin=2, thin=1, max_kept=sweeps, tau_per_column=True)
    for s in (1, 2, 3):
        g.pp_stage(s, sweeps)
        if o.stage_blocks(s):
            o.run_stage(s, sweeps)
            for blk in o.stage_blocks(s):
                # the draws follow chains that agree to FP64 rounding grown over the sweeps
                np.testing.assert_allclose(g.get_tau_cols(blk["b"]), blk["tau"], rtol=1e-6)
    pg = g.predict(d["test_row"], d["test_col"])
    for b in range(I * J):
        for side, key in ((0, "x"), (1, "w")):
            mg, Lg = g.get_mm(b, side)
            np.testing.assert_allclose(mg, o.mm[b][key + "_mu"], rtol=1e-6, atol=1e-7)
            np.testing.assert_allclose(Lg, o.mm[b][key + "_Lam"], rtol=1e-4, atol=1e-4)
    o.aggregate()
    po = o.predict(d["test_row"], d["test_col"])
    np.testing.assert_allclose(pg, po, rtol=1e-5, atol=1e-5)
    g.close()


def test_fp32_chain_rmse_matches_oracle():
    import synth
    K = 10
    d = synth.make("ratings", 3000, 1500, K, 300000, 0.8, 6)
    rg, ro = [], []
    for seed in (301, 302, 303):
        g, o = pair(d, K, "fp32", I=2, J=2, order="random", seed=seed, burnin=15, max_kept=25,
                    tau_per_column=True)
        for s in (1, 2, 3):
            g.pp_stage(s, 40)
            o.run_stage(s, 40)
        pg = g.predict(d["test_row"], d["test_col"])
        o.aggregate()
        po = o.predict(d["test_row"], d["test_col"])
        rg.append(np.sqrt(np.mean((pg - d["test_val"]) ** 2)))
        ro.append(np.sqrt(np.mean((po - d["test_val"]) ** 2)))
        g.close()
    print("tau_d rmse gpu", rg, "oracle", ro)
    assert abs(np.mean(rg) - np.mean(ro)) <= 0.005 * np.mean(ro)


def test_batched_equals_per_block():
    K = 24
    d = small_data(K, seed=12, N=500, D=260, nnz=16000)
    out = []
    for batched in (True, False):
        g, _ = pair(d, K, "fp32", I=2, J=2, order="random", seed=8, burnin=2, max_kept=6, batched=batched,
                    lane_nnz=16, tau_per_column=True)
        for s in (1, 2, 3):
            g.pp_stage(s, 8)
        out.append((g.predict(d["test_row"], d["test_col"]), g.get_tau_cols(3)))
        g.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
