"""The error of every result of the FP32 and BF16 arms against FP64 arithmetic
(needs an MI355X).

Each result is compared where the arm and an FP64 computation see the same
inputs, so that the difference is the arm's own rounding and never the
divergence of two Markov chains:

* x_n, w_d: one conditional draw of every row and every column (Sec. 2.1)
  from the same state and the same noise as the oracle, in stage 1 (the
  Normal-Wishart prior) and in stage 3 (moment-matched per-row priors, Sec. 3.2,
  including the entities without entries and with one to eight entries that
  use the stored prior factor); the draw before rounding, with rel_n of the
  parity tests, and the stored state as its exact rounding;
* Lambda_X, mu_X, Lambda_W, mu_W and tau: one draw of each from the arm's
  stored state and the same noise (FP64 on both sides);
* mu_hat, Lambda_hat: moment matching (Sec. 4.1) of the arm's own kept
  samples against the mean and inverse 1/(S - 1) covariance in numpy FP64;
* mu*: Algorithm 2 (Sec. 4.2) of the arm's moment-matched rows against the
  oracle's aggregation of the same rows, with equal correction counts;
* y_hat and the test RMSE: prediction from those aggregated means.

Every quantity prints one "error-statement" line with the measured maximum;
the asserted bounds are the ones the documentation states for the arms.  The
chain-level statement (the arms' test RMSE against the FP64 oracle's over
whole chains) is the subject of the chain tests.
"""
import numpy as np
import pytest

from gpu_helpers import cond_precision_trace, load_state, pair, random_state, rel_err_rows, round_state, small_data

pytestmark = pytest.mark.gpu

K = 32
BOUND = dict(draw=1e-4, hyper=1e-8, tau=1e-6, mm=1e-8, agg=1e-8, pred=1e-6)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(precision, what, value, bound):
    print("error-statement %s %-12s max %.3e (bound %.0e)" % (precision, what, value, bound), flush=True)
    assert value <= bound, (what, value, bound)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _draws(g, o, b, precision, t, st):
    """One row pass and one column pass of block b from state st on both sides."""
    blk = o.blocks[b]
    out = {}
    for which, side, key in (("rows", 0, "X"), ("cols", 1, "W")):
        load_state(g, o, b, st)
        g.step(b, which, t)
        getattr(o, "update_" + which)(blk, t)
        draw = g.get_draw(b, side)
        prop = blk.get("x_prior" if which == "rows" else "w_prior")
        prior = prop[0] if prop is not None else blk["hx" if which == "rows" else "hw"][0]
        tr = cond_precision_trace(blk, which, K, blk["tau"], prior)
        out[which] = rel_err_rows(draw, blk[key], tr, K).max()
        assert np.array_equal(g.get_state(b)[key], round_state(draw, precision))
    return out


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_error_of_every_result(precision):
    print("case", precision, flush=True)
    d = small_data(K, seed=77, N=400, D=240, nnz=1200, empty_rows=5, kind="uniform")
    S = 2 * K + 8                            # kept samples per stage (moment matching well conditioned)

    # stage 1: draws, Normal-Wishart and tau from an identical state
    g1, o1 = pair(d, K, precision)
    g1.pp_stage(1, 0)
    o1.begin_stage(1)
    blk = o1.blocks[0]
    st = random_state(np.random.default_rng(501), blk["R"], blk["C"], K)
    e = _draws(g1, o1, 0, precision, 3, st)
    _say(precision, "x_n stage1", e["rows"], BOUND["draw"])
    _say(precision, "w_d stage1", e["cols"], BOUND["draw"])
    for side, name in (("hyper_x", "x"), ("hyper_w", "w")):
        load_state(g1, o1, 0, st)
        g1.step(0, side, 9)
        o1.hyper_draw(blk, name, 9)
        Lg, mg = g1.get_state(0)["h" + name]
        Lo, mo = blk["h" + name]
        _say(precision, "Lambda_" + name.upper(), _rel(Lg, Lo), BOUND["hyper"])
        _say(precision, "mu_" + name.upper(), _rel(mg, mo), BOUND["hyper"])
    load_state(g1, o1, 0, st)
    g1.step(0, "tau", 12)
    o1.tau_draw(blk, 12)
    _say(precision, "tau", abs(g1.get_state(0)["tau"] - blk["tau"]) / blk["tau"], BOUND["tau"])
    g1.close()

    # the arm's own PP chain on a 2 x 2 partition: every block's kept samples,
    # read while its stage is active, give the FP64 reference moments
    g, o = pair(d, K, precision, I=2, J=2, order="random", max_kept=S, burnin=0)
    ref = {}
    for s in (1, 2, 3):
        g.pp_stage(s, S)
        for b in range(4):
            if g.block_info(b)["stage"] != s:
                continue
            for side in (0, 1):
                X = np.stack([g.get_sample(b, side, k) for k in range(S)], axis=1)   # n x S x K
                mu = X.mean(axis=1)
                Xc = X - mu[:, None, :]
                ref[b, side] = (mu, np.linalg.inv(np.einsum("nsk,nsl->nkl", Xc, Xc) / (S - 1)))

    # stage 3 draws under the library's own moment-matched priors
    for b in range(4):
        if g.block_info(b)["stage"] < 3:
            mx, Lx = g.get_mm(b, 0)
            mw, Lw = g.get_mm(b, 1)
            o.mm[b] = dict(x_mu=mx, x_Lam=Lx, w_mu=mw, w_Lam=Lw, ridged=0)
    o.begin_stage(3)
    blk3 = o.blocks[3]
    st3 = random_state(np.random.default_rng(502), blk3["R"], blk3["C"], K)
    e3 = _draws(g, o, 3, precision, 4, st3)
    _say(precision, "x_n stage3", e3["rows"], BOUND["draw"])
    _say(precision, "w_d stage3", e3["cols"], BOUND["draw"])

    # moment matching (stage 3's at aggregation) against the reference moments
    g.aggregate()
    worst_mu = worst_lam = 0.0
    for b in range(4):
        got = {}
        for side, key in ((0, "x"), (1, "w")):
            mg, Lg = g.get_mm(b, side)
            mu, lam = ref[b, side]
            worst_mu = max(worst_mu, (np.linalg.norm(mg - mu, axis=1) /
                                      np.maximum(np.linalg.norm(mu, axis=1), 1e-12)).max())
            worst_lam = max(worst_lam, (np.linalg.norm(Lg - lam, axis=(1, 2)) /
                                        np.linalg.norm(lam, axis=(1, 2))).max())
            got[key + "_mu"], got[key + "_Lam"] = mg, Lg
        o.mm[b] = dict(got, ridged=0)
    assert g.stats()["mm_ridged"] == 0
    _say(precision, "mu_hat", worst_mu, BOUND["mm"])
    _say(precision, "Lambda_hat", worst_lam, BOUND["mm"])

    # Algorithm 2 and prediction from the arm's moment-matched rows
    o.aggregate()
    p = o.plan
    mx = np.empty((o.N, K))
    mw = np.empty((o.D, K))
    for i in range(2):
        mx[p.row_ids[i]] = o.mu_x[i]
    for j in range(2):
        mw[p.col_ids[j]] = o.mu_w[j]
    _say(precision, "mu*_X", _rel(g.get_aggregate(0), mx), BOUND["agg"])
    _say(precision, "mu*_W", _rel(g.get_aggregate(1), mw), BOUND["agg"])
    print("aggregation corrections", g.stats()["agg_corrections"], "oracle", o.corrections, flush=True)
    assert g.stats()["agg_corrections"] == o.corrections
    # predictions are returned in FP32
    pg = g.predict(d["test_row"], d["test_col"]).astype(np.float64)
    po = o.predict(d["test_row"], d["test_col"])
    _say(precision, "y_hat", _rel(pg, po), BOUND["pred"])
    rg = np.sqrt(np.mean((pg - d["test_val"]) ** 2))
    ro = np.sqrt(np.mean((po - d["test_val"]) ** 2))
    _say(precision, "rmse", abs(rg - ro) / ro, BOUND["pred"])
    g.close()
