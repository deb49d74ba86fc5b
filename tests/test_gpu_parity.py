"""GPU parity of the HIP path against the FP64 oracle (needs an MI355X).

Single conditional steps from an identical state with identical Philox noise
(rows, columns, Normal-Wishart draws, tau) in every precision and at ranks
served by both update kernels; then chains, PP stages, moment matching,
aggregation and prediction.
"""
import numpy as np
import pytest

from gpu_helpers import (TOL, cond_precision_trace, load_state, pair, random_state, rel_err_rows,
                         round_state, small_data)

pytestmark = pytest.mark.gpu

KS = [1, 3, 10, 16, 24, 32, 64]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("K", KS)
@pytest.mark.parametrize("which", ["rows", "cols"])
def test_single_step_update(precision, K, which):
    print("case", precision, K, which, flush=True)
    d = small_data(K, seed=K)
    g, o = pair(d, K, precision)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    st = random_state(np.random.default_rng(100 + K), blk["R"], blk["C"], K)
    load_state(g, o, 0, st)
    t = 5
    g.step(0, which, t)
    if which == "rows":
        o.update_rows(blk, t)
    else:
        o.update_cols(blk, t)
    key = "X" if which == "rows" else "W"
    draw = g.get_draw(0, 0 if which == "rows" else 1)     # FP64, or FP32 in FP32/BF16 modes
    state = g.get_state(0)[key]
    xo = blk[key]
    prior = blk["hx"][0] if which == "rows" else blk["hw"][0]
    tr = cond_precision_trace(blk, which, K, blk["tau"], prior)
    rel = rel_err_rows(draw, xo, tr, K)
    print("draw vs oracle: max rel", rel.max(), "p99.9", np.quantile(rel, 0.999), "median",
          np.median(rel))
    assert rel.max() <= TOL[precision]
    # the state holds the draw rounded to the state precision, bit for bit
    assert np.array_equal(state, round_state(draw, precision))
    s = g.stats()
    assert s["nonpd_rows"] == 0


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
@pytest.mark.parametrize("K", [32, 64])
def test_single_step_heavy_columns(precision, K):
    """Columns with several thousand entries: on the MFMA path they are split
    into segments whose partial Grams are summed before the factorisation."""
    print("case heavy", precision, K, flush=True)
    d = small_data(K, seed=40 + K, N=6000, D=40, nnz=90000, empty_rows=0)
    g, o = pair(d, K, precision)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    assert np.diff(blk["csc_ptr"]).max() > 2048              # split into segments
    st = random_state(np.random.default_rng(200 + K), blk["R"], blk["C"], K, scale=0.3)
    load_state(g, o, 0, st)
    g.step(0, "cols", 4)
    o.update_cols(blk, 4)
    draw = g.get_draw(0, 1)
    tr = cond_precision_trace(blk, "cols", K, blk["tau"], blk["hw"][0])
    rel = rel_err_rows(draw, blk["W"], tr, K)
    print("draw vs oracle: max rel", rel.max(), "median", np.median(rel))
    assert rel.max() <= TOL[precision]
    assert np.array_equal(g.get_state(0)["W"], round_state(draw, precision))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("lane_nnz", [1, 3, 8, 256])
def test_single_step_every_lane_group_size(precision, lane_nnz):
    """The register kernel gives an entity G = 1..256 lanes (G the power of two
    at or above degree / lane_nnz): with lane_nnz = 1 the entities of this data
    span every G, including groups of several wavefronts.  Rows, then columns,
    then the tau draw from the per-column residual SSE, against the oracle."""
    K = 10
    print("case lanes", precision, lane_nnz, flush=True)
    d = small_data(K, seed=70, N=2000, D=500, nnz=60000, empty_rows=3)
    g, o = pair(d, K, precision, lane_nnz=lane_nnz)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    assert np.diff(blk["csc_ptr"]).max() > 256                # groups of 256 lanes at lane_nnz 1
    st = random_state(np.random.default_rng(300 + lane_nnz), blk["R"], blk["C"], K)
    load_state(g, o, 0, st)
    for which, t in (("rows", 6), ("cols", 6)):
        g.step(0, which, t)
        if which == "rows":
            o.update_rows(blk, t)
        else:
            o.update_cols(blk, t)
        key = "X" if which == "rows" else "W"
        draw = g.get_draw(0, 0 if which == "rows" else 1)
        prior = blk["hx"][0] if which == "rows" else blk["hw"][0]
        tr = cond_precision_trace(blk, which, K, blk["tau"], prior)
        rel = rel_err_rows(draw, blk[key], tr, K)
        print(which, "max rel", rel.max(), flush=True)
        assert rel.max() <= TOL[precision]
        assert np.array_equal(g.get_state(0)[key], round_state(draw, precision))
        # the oracle continues from the library's state (identical values)
        blk[key] = g.get_state(0)[key]
    # tau from the per-column SSE kernel
    g.step(0, "tau", 7)
    o.tau_draw(blk, 7)
    assert g.get_state(0)["tau"] == pytest.approx(blk["tau"], rel=1e-9 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("lane_nnz", [1, 256])
def test_fp64_sweeps_every_lane_group_size(lane_nnz):
    """Whole FP64 sweeps, where the column pass also sums the residuals of each
    column for the tau draw (fused SSE), at every lane-group size."""
    K = 10
    print("case sweeps lanes", lane_nnz, flush=True)
    d = small_data(K, seed=71, N=2000, D=500, nnz=60000, empty_rows=3)
    g, o = pair(d, K, "fp64", lane_nnz=lane_nnz)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    st = random_state(np.random.default_rng(400 + lane_nnz), blk["R"], blk["C"], K, scale=0.3)
    load_state(g, o, 0, st)
    g.gibbs_sweep(3)
    o.sweep(3)
    s = g.get_state(0)
    np.testing.assert_allclose(s["X"], blk["X"], rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(s["W"], blk["W"], rtol=1e-8, atol=1e-9)
    assert s["tau"] == pytest.approx(blk["tau"], rel=1e-9)


@pytest.mark.parametrize("K", [2, 10, 33, 64])
@pytest.mark.parametrize("side", ["hyper_x", "hyper_w"])
def test_normal_wishart_draw(K, side):
    print("case", K, side, flush=True)
    d = small_data(K, seed=3)
    g, o = pair(d, K, "fp64")
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    st = random_state(np.random.default_rng(7), blk["R"], blk["C"], K)
    load_state(g, o, 0, st)
    g.step(0, side, 9)
    o.hyper_draw(blk, "x" if side == "hyper_x" else "w", 9)
    s = g.get_state(0)
    Lg, mg = s["hx"] if side == "hyper_x" else s["hw"]
    Lo, mo = blk["hx"] if side == "hyper_x" else blk["hw"]
    np.testing.assert_allclose(Lg, Lo, rtol=1e-9, atol=1e-9 * np.abs(Lo).max())
    np.testing.assert_allclose(mg, mo, rtol=1e-9, atol=1e-9 * np.abs(mo).max())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tau_draw(precision):
    K = 10
    d = small_data(K, seed=4)
    g, o = pair(d, K, precision)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    st = random_state(np.random.default_rng(8), blk["R"], blk["C"], K, scale=0.3)
    load_state(g, o, 0, st)
    g.step(0, "tau", 12)
    o.tau_draw(blk, 12)
    tg = g.get_state(0)["tau"]
    assert tg == pytest.approx(blk["tau"], rel=1e-12 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("K", [10, 32])
def test_fp32_fallback_path_redoes_rows_in_fp64(K):
    """pivot_theta close to 1 fails every FP32 pivot test: every row is redone by
    the FP64 pass, which then matches the oracle to FP32 input rounding (K = 32:
    light rows fail in the two-per-wavefront kernel, the others in the
    wavefront kernel)."""
    d = small_data(K, seed=5)
    g, o = pair(d, K, "fp32", pivot_theta=0.9999)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    st = random_state(np.random.default_rng(9), blk["R"], blk["C"], K)
    load_state(g, o, 0, st)
    g.step(0, "rows", 3)
    o.update_rows(blk, 3)
    assert g.stats()["fallback_rows"] == blk["R"]
    tr = cond_precision_trace(blk, "rows", K, blk["tau"], blk["hx"][0])
    rel = rel_err_rows(g.get_state(0)["X"], blk["X"], tr, K)
    assert rel.max() < 2e-6


@pytest.mark.parametrize("precision,K", [("fp32", 24), ("bf16", 32), ("bf16", 40), ("fp32", 64)])
def test_few_entry_entities_under_propagated_priors(precision, K):
    """Stage-3 single steps on a sparse 2 x 2 partition where a quarter of the
    rows and some columns have no entries in their block and most others one to
    eight: the former take the prior-factor kernel (x = mu + L^-T z, L the
    Cholesky factor of the moment-matched precision, factored once per stage),
    the latter the low-rank kernel (that factor updated by product-form
    rank-one modifications), the rest the factorising kernels; every draw
    against the oracle's from the same moment-matched priors and noise, and the
    column pass's residual SSE through the tau draw.  More kept samples than 2K
    keep the moment-matched precisions well conditioned."""
    print("case empty", precision, K, flush=True)
    d = small_data(K, seed=21 + K, N=400, D=240, nnz=1200, empty_rows=5, kind="uniform")
    S = 2 * K + 8
    g, o = pair(d, K, precision, I=2, J=2, order="random", max_kept=S)
    g.pp_stage(1, S)
    g.pp_stage(2, S)
    g.pp_stage(3, 0)                 # moment matching of stage 2 and the prior factors
    for b in range(4):
        if g.block_info(b)["stage"] < 3:
            mx, Lx = g.get_mm(b, 0)
            mw, Lw = g.get_mm(b, 1)
            o.mm[b] = dict(x_mu=mx, x_Lam=Lx, w_mu=mw, w_Lam=Lw, ridged=0)
    o.begin_stage(3)
    b = 3
    blk = o.blocks[b]
    assert g.block_info(b)["stage"] == 3
    st = random_state(np.random.default_rng(300 + K), blk["R"], blk["C"], K)
    for which, side, key, ptr in (("rows", 0, "X", "csr_ptr"), ("cols", 1, "W", "csc_ptr")):
        load_state(g, o, b, st)
        g.step(b, which, 4)
        if which == "rows":
            o.update_rows(blk, 4)
        else:
            o.update_cols(blk, 4)
        deg = np.diff(blk[ptr])
        empty = deg == 0
        few = (deg >= 1) & (deg <= 8)
        draw = g.get_draw(b, side)
        prior = blk["x_prior" if which == "rows" else "w_prior"][0]
        tr = cond_precision_trace(blk, which, K, blk["tau"], prior)
        rel = rel_err_rows(draw, blk[key], tr, K)
        print(which, "empty", int(empty.sum()), "1-8 entries", int(few.sum()), "of", empty.size,
              "max rel", rel.max(), "of the empty", rel[empty].max() if empty.any() else None,
              "of the 1-8", rel[few].max() if few.any() else None, flush=True)
        assert rel.max() <= TOL[precision]
        assert few.sum() >= (50 if which == "rows" else 20)
        assert np.array_equal(g.get_state(b)[key], round_state(draw, precision))
        assert empty.sum() >= (20 if which == "rows" else 5)
    # a whole sweep (its first, t = 0): the tau draw that closes it reads the
    # residual SSE the column pass left, per column, from the library's state
    load_state(g, o, b, st)
    g.gibbs_sweep(1)
    sg = g.get_state(b)
    blk["X"], blk["W"] = sg["X"].copy(), sg["W"].copy()
    o.tau_draw(blk, 0)
    print("tau", sg["tau"], "oracle", blk["tau"], flush=True)
    np.testing.assert_allclose(sg["tau"], blk["tau"], rtol=1e-4)
    assert g.stats()["nonpd_rows"] == 0


@pytest.mark.parametrize("precision,K", [("bf16", 32), ("fp32", 24), ("bf16", 48)])
def test_prior_factor_paths_same_in_every_launch_form(precision, K):
    """Stages 2 and 3 on a sparse 2 x 2 partition, where the prior-factor,
    low-rank, light and heavy kernels all take part: graph-replayed batched
    sweeps, eagerly launched batched sweeps and per-block launches (different
    item orders, so different pairings of entities in a wavefront) give the
    same states bit for bit."""
    print("case launch forms", precision, K, flush=True)
    d = small_data(K, seed=60 + K, N=500, D=260, nnz=3000, empty_rows=3)
    S = 2 * K + 4
    runs = []
    for batched, eager in ((True, False), (True, True), (False, False)):
        g, _ = pair(d, K, precision, I=2, J=2, order="random", batched=batched, max_kept=S)
        if eager:
            g.enable_timing(True)
        out = []
        for s, nsw in ((1, S), (2, S), (3, 4)):
            g.pp_stage(s, nsw)
            for b in range(4):
                if g.block_info(b)["stage"] == s:
                    st = g.get_state(b)
                    out += [st["X"], st["W"], st["tau"]]
        runs.append(out)
        assert g.stats()["nonpd_rows"] == 0
        g.close()
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_batched_equals_per_block_and_is_deterministic(precision):
    K = 10
    d = small_data(K, seed=6)
    runs = []
    for batched in (True, False, True):
        g, _ = pair(d, K, precision, I=2, J=2, order="random", batched=batched, max_kept=2,
                    lane_nnz=16)
        g.pp_stage(1, 3)
        runs.append([g.get_state(0)[k] for k in ("X", "W", "tau")])
        g.close()
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    for a, b in zip(runs[0], runs[2]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_graph_replays_match_eager_sweeps(precision):
    """Sweeps replayed from the captured graph, with eager copies and
    synchronisations between replays, equal eagerly launched sweeps bit for bit,
    replay after replay."""
    K = 10
    d = small_data(K, seed=8)
    g, _ = pair(d, K, precision, I=2, J=2, order="random", lane_nnz=16, max_kept=6, burnin=2)
    e, _ = pair(d, K, precision, I=2, J=2, order="random", lane_nnz=16, max_kept=6, burnin=2)
    e.enable_timing(True)                    # per-launch events: eager sweeps
    g.gibbs_sweep(0)
    e.gibbs_sweep(0)
    for rep in range(5):
        g.gibbs_sweep(1)
        e.gibbs_sweep(1)
        for b in (0,):
            sg, se = g.get_state(b), e.get_state(b)
            for key in ("X", "W", "tau"):
                assert np.array_equal(sg[key], se[key]), (rep, key)
            assert np.array_equal(sg["hx"][0], se["hx"][0])
    g.pp_stage(2, 3)
    e.pp_stage(2, 3)
    for b in range(4):
        if g.block_info(b)["stage"] == 2:
            sg, se = g.get_state(b), e.get_state(b)
            assert np.array_equal(sg["X"], se["X"]) and np.array_equal(sg["W"], se["W"])
    for b in (1, 2):
        np.testing.assert_array_equal(g.get_mm(0, 0)[0], e.get_mm(0, 0)[0])


def test_fp64_chain_tracks_oracle_1x1():
    """Whole FP64 sweeps (rows, cols, NW draws, tau, sample store) with identical
    noise stay on the oracle's trajectory; moment matching and predictions agree."""
    import synth
    d = synth.config(1, seed=1)
    K = 10
    g, o = pair(d, K, "fp64", burnin=5, thin=1, max_kept=10)
    g.gibbs_sweep(15)
    o.begin_stage(1)
    o.sweep(15)
    sg = g.get_state(0)
    blk = o.blocks[0]
    np.testing.assert_allclose(sg["X"], blk["X"], rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(sg["W"], blk["W"], rtol=1e-7, atol=1e-8)
    assert sg["tau"] == pytest.approx(blk["tau"], rel=1e-8)
    o.finalize_stage()
    mg, Lg = g.get_mm(0, 0)
    np.testing.assert_allclose(mg, o.mm[0]["x_mu"], rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(Lg, o.mm[0]["x_Lam"], rtol=1e-5, atol=1e-6)
    pg = g.predict(d["test_row"], d["test_col"])
    o.aggregate()
    po = o.predict(d["test_row"], d["test_col"])
    np.testing.assert_allclose(pg, po, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("IJ,order,K,sweeps", [((2, 2), "random", 6, 8), ((3, 2), "decreasing", 6, 8),
                                               ((2, 1), "given", 6, 8), ((2, 3), "random", 5, 8),
                                               ((2, 2), "random", 17, 40)])
def test_fp64_pp_stages_track_oracle(IJ, order, K, sweeps):
    """PP stages 1-3 with propagated per-row priors, moment matching, Algorithm 2
    aggregation (with its eigenvalue corrections) and prediction, FP64,
    identical noise.  K = 17 keeps more samples than 2K, so that moment matching
    is not ridged and its precisions are well conditioned."""
    d = small_data(K, seed=7, N=300, D=200, nnz=12000, empty_rows=0)
    I, J = IJ
    g, o = pair(d, K, "fp64", I=I, J=J, order=order, burnin=2, thin=1, max_kept=sweeps)
    for s in (1, 2, 3):
        g.pp_stage(s, sweeps)
        if o.stage_blocks(s):
            o.run_stage(s, sweeps)
    for b in range(I * J):
        for side, key in ((0, "x"), (1, "w")):
            mg, Lg = g.get_mm(b, side)
            np.testing.assert_allclose(mg, o.mm[b][key + "_mu"], rtol=1e-6, atol=1e-7)
            np.testing.assert_allclose(Lg, o.mm[b][key + "_Lam"], rtol=1e-4, atol=1e-4)
    pg = g.predict(d["test_row"], d["test_col"])
    o.aggregate()
    po = o.predict(d["test_row"], d["test_col"])
    print("aggregation corrections: gpu", g.stats()["agg_corrections"], "oracle", o.corrections)
    assert g.stats()["agg_corrections"] == o.corrections
    np.testing.assert_allclose(pg, po, rtol=1e-5, atol=1e-5)
    mx = g.get_aggregate(0)
    for r in range(0, d["N"], 7):
        i, n = o.plan.row_block[r], o.plan.row_local[r]
        np.testing.assert_allclose(mx[r], o.mu_x[i][n], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("precision,K", [("fp32", 10), ("bf16", 10), ("bf16", 32), ("fp32", 32)])
def test_chain_rmse_matches_oracle(precision, K):
    """Test RMSE after burn-in within 0.5 % of the oracle's (mean of 3 seeds) on
    a ratings-shaped workload where independent chains agree to ~0.1 %."""
    import synth
    d = synth.make("ratings", 3000, 1500, K, 300000, 0.8, 5)
    rg, ro = [], []
    for seed in (101, 102, 103):
        g, o = pair(d, K, precision, seed=seed, burnin=20, max_kept=40)
        g.gibbs_sweep(60)
        pg = g.predict(d["test_row"], d["test_col"])
        o.run_stage(1, 60)
        o.aggregate()
        po = o.predict(d["test_row"], d["test_col"])
        rg.append(np.sqrt(np.mean((pg - d["test_val"]) ** 2)))
        ro.append(np.sqrt(np.mean((po - d["test_val"]) ** 2)))
        g.close()
    print("rmse gpu", rg, "oracle", ro)
    assert abs(np.mean(rg) - np.mean(ro)) <= 0.005 * np.mean(ro)


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_pp_chain_rmse_matches_oracle(precision):
    """Posterior propagation on a 2 x 2 partition (stages 1-3 under propagated
    priors, moment matching, Algorithm 2 aggregation, prediction): test RMSE
    within 0.5 % of the oracle's PP chains (mean of 3 seeds)."""
    import synth
    K = 10
    d = synth.make("ratings", 3000, 1500, K, 300000, 0.8, 6)
    rg, ro = [], []
    for seed in (201, 202, 203):
        g, o = pair(d, K, precision, I=2, J=2, order="random", seed=seed, burnin=15, max_kept=25)
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
    print("pp rmse gpu", rg, "oracle", ro)
    assert abs(np.mean(rg) - np.mean(ro)) <= 0.005 * np.mean(ro)
