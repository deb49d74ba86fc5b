"""GPU parity at the benchmark workloads' full sizes (needs an MI355X).

Sweeps run exactly as bench.py times them (batched, replayed from the captured
graph, with the schedule the autotuner picks at stage begin; or, for the plain
FP32 arm, one launch sequence per block), from states loaded identically into
the library and the oracle.  Every row and column a sweep draws is compared
with the oracle's FP64 conditional draw with the same Philox noise:

* the FP32 draw the library keeps as the sweep's sample (before any BF16
  rounding) within 1e-4, relative to max(||x_n||, sqrt(tr(A_n^-1) / K)), with
  A_n the entity's conditional precision, and
* the state it stores: bit for bit the round-to-nearest-even of that draw to
  the state precision, hence (BF16 unit roundoff 2^-8 per entry) within
  2^-8 + 1e-4 of the oracle's draw in the same measure.

The oracle's draw is never rounded.  Then the
Normal-Wishart and tau draws that close the sweep, and, for the 8 x 8 PP
workload, the moment-matched priors of the stage-2 source blocks computed
from the library's own kept samples.
"""
import numpy as np
import pytest

from gpu_helpers import load_state, pair, random_state, round_state
from oracle import native
from oracle.native import ptr

pytestmark = pytest.mark.gpu

TOL_DRAW = 1e-4                  # FP32 arithmetic from identical inputs
TOL_STATE = 2.0 ** -8 + TOL_DRAW   # BF16 state: the draw's rounding on top


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _scale(blk, which, K, prior, chunk=20000):
    """sqrt(tr(A_n^-1) / K) of every entity of one side of a block, with A_n the
    oracle's conditional precision at the block's current state."""
    if which == "rows":
        p_, idx, val, other, n = blk["csr_ptr"], blk["csr_idx"], blk["csr_val"], blk["W"], blk["R"]
    else:
        p_, idx, val, other, n = blk["csc_ptr"], blk["csc_idx"], blk["csc_val"], blk["X"], blk["C"]
    P, m = prior
    per_row = 1 if P.ndim == 3 else 0
    other = np.ascontiguousarray(other)
    out = np.empty(n)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        A = np.zeros((b - a, K, K))
        Pc = np.ascontiguousarray(P[a:b]) if per_row else np.ascontiguousarray(P)
        mc = np.ascontiguousarray(m[a:b]) if per_row else np.ascontiguousarray(m)
        native.lib().orc_cond_precision(b - a, K, ptr(np.ascontiguousarray(p_[a:b + 1])), ptr(idx), ptr(val),
                                        ptr(other), per_row, ptr(Pc), ptr(mc), float(blk["tau"]), ptr(A))
        out[a:b] = np.sqrt(np.trace(np.linalg.inv(A), axis1=1, axis2=2) / K)
    return out


def _rel(x, xo, scale):
    return np.linalg.norm(x - xo, axis=1) / np.maximum(np.linalg.norm(xo, axis=1), scale)


def _check_side(name, o, blk, which, K, prior, draw, state, tol_state, precision):
    """Run the oracle's pass from the block's current state and compare."""
    scale = _scale(blk, which, K, prior)
    if which == "rows":
        o.update_rows(blk, blk["t"])
        xo = blk["X"]
    else:
        o.update_cols(blk, blk["t"])
        xo = blk["W"]
    assert np.array_equal(state, round_state(draw, precision)), (name, which)
    r = _rel(draw, xo, scale)
    q = _rel(state, xo, scale)
    print("%s %s: draw max %.3g p99.9 %.3g median %.3g | state max %.3g (%d entities)"
          % (name, which, r.max(), np.quantile(r, 0.999), np.median(r), q.max(), r.size), flush=True)
    assert r.max() <= TOL_DRAW, (name, which, r.max())
    assert q.max() <= tol_state, (name, which, q.max())


def _prior(blk, which):
    if which == "rows":
        return blk["x_prior"] if blk["x_prior"] is not None else blk["hx"]
    return blk["w_prior"] if blk["w_prior"] is not None else blk["hw"]


def _sweep_and_check(name, g, o, bs, K, precision, slot):
    """One sweep of the library's active stage (already loaded), then, for every
    block in bs, the oracle's rows from the loaded state, its columns from the
    library's new rows, and its NW and tau draws from the library's new state."""
    tol_state = TOL_STATE if precision == "bf16" else TOL_DRAW
    g.gibbs_sweep(1)
    for b in bs:
        blk = o.blocks[b]
        s = g.get_state(b)
        _check_side("%s block %d" % (name, b), o, blk, "rows", K, _prior(blk, "rows"),
                    g.get_sample(b, 0, slot), s["X"], tol_state, precision)
        blk["X"] = s["X"].copy()
        _check_side("%s block %d" % (name, b), o, blk, "cols", K, _prior(blk, "cols"),
                    g.get_sample(b, 1, slot), s["W"], tol_state, precision)
        blk["W"] = s["W"].copy()
        for side, key in (("x", "hx"), ("w", "hw")):
            if blk[side + "_prop"]:
                continue
            o.hyper_draw(blk, side, blk["t"])
            np.testing.assert_allclose(s[key][0], blk[key][0], rtol=1e-6, atol=1e-9 * np.abs(blk[key][0]).max())
            np.testing.assert_allclose(s[key][1], blk[key][1], rtol=1e-6, atol=1e-9)
        o.tau_draw(blk, blk["t"])
        np.testing.assert_allclose(s["tau"], blk["tau"], rtol=1e-4)
    assert g.stats()["nonpd_rows"] == 0


@pytest.mark.parametrize("cid,precision,batched", [(2, "bf16", True), (3, "bf16", True), (4, "bf16", True),
                                                   (2, "fp32", False)])
def test_full_size_sweep_matches_oracle(cid, precision, batched):
    import synth
    cfg = synth.CONFIGS[cid]
    print("case: full-size workload", cid, precision, "batched" if batched else "per block", flush=True)
    d = synth.config(cid, seed=1)
    K = d["K"]
    g, o = pair(d, K, precision, I=cfg["I"], J=cfg["J"], order=cfg["order"], seed=101, max_kept=1,
                batched=batched)
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    assert g.block_info(0)["stage"] == 1
    st = random_state(np.random.default_rng(70 + cid), blk["R"], blk["C"], K)
    load_state(g, o, 0, st)
    print("schedule", g.schedule(), "rows", blk["R"], "cols", blk["C"], flush=True)
    _sweep_and_check("workload %d" % cid, g, o, [0], K, precision, 0)
    g.close()


def _check_mm(g, b, side, K, S):
    """Moment matching of the library (Sec. 4.1) against the oracle's, both from
    the S kept samples of block b the library holds (FP32 draws)."""
    info = g.block_info(b)
    n = info["R"] if side == 0 else info["C"]
    smp = np.stack([g.get_sample(b, side, q) for q in range(S)])
    mu = np.zeros((n, K))
    Lam = np.zeros((n, K, K))
    ridged = native.lib().orc_mm(n, K, S, ptr(np.ascontiguousarray(smp)), ptr(mu), ptr(Lam))
    gm, gL = g.get_mm(b, side)
    scale_mu = np.sqrt(np.var(smp, axis=0).sum(1) / K) + 1e-30
    emu = (np.abs(gm - mu).max(1) / scale_mu).max()
    eL = (np.abs(gL - Lam).max((1, 2)) / np.abs(Lam).max((1, 2))).max()
    print("MM block %d side %d: %d rows, mean rel %.3g, precision rel %.3g, ridged %d"
          % (b, side, n, emu, eL, ridged), flush=True)
    assert emu <= 1e-9 and eL <= 1e-7
    return ridged


def test_full_size_pp_stages_match_oracle():
    """The 480k x 17.8k, K = 32 workload on its 8 x 8 partition (decreasing
    order), BF16 state, batched and graph-replayed: one sweep of the stage-1
    block, of the two densest stage-2 blocks and of all 49 stage-3 blocks
    from loaded states, each against the oracle under the same priors (stage 3:
    the library's own moment-matched priors, themselves checked against the
    oracle's moment matching of the library's kept samples).  Stage 3 takes
    every update kernel: the prior-factor path (rows without entries), the
    low-rank path (one to eight entries), the two-per-wavefront kernel, the
    MFMA wavefront kernel and the segment Grams of heavy columns."""
    import synth
    cfg = synth.CONFIGS[5]
    print("case: full-size workload 5, stages 1-3", flush=True)
    d = synth.config(5, seed=1, progress=lambda m: print("data:", m, flush=True))
    K = d["K"]
    S = 2 * K + 2
    I, J = cfg["I"], cfg["J"]
    g, o = pair(d, K, "bf16", I=I, J=J, order=cfg["order"], seed=101, max_kept=S)
    print("library and oracle built", flush=True)
    rng = np.random.default_rng(75)
    # stage 1
    g.pp_stage(1, 0)
    o.begin_stage(1)
    blk = o.blocks[0]
    load_state(g, o, 0, random_state(rng, blk["R"], blk["C"], K))
    _sweep_and_check("stage 1", g, o, [0], K, "bf16", 0)
    g.gibbs_sweep(S - 1)
    # stage 2: the propagated W of (1, 0) and the propagated X of (0, 1) come
    # from block (0, 0)'s moment matching
    g.pp_stage(2, 0)
    mx0, Lx0 = g.get_mm(0, 0)
    mw0, Lw0 = g.get_mm(0, 1)
    o.mm[0] = dict(x_mu=mx0, x_Lam=Lx0, w_mu=mw0, w_Lam=Lw0, ridged=0)
    o.begin_stage(2)                       # binds block (0, 0)'s moments
    two = [1, J]
    for b in two:
        blk = o.blocks[b]
        load_state(g, o, b, random_state(rng, blk["R"], blk["C"], K))
    _sweep_and_check("stage 2", g, o, two, K, "bf16", 0)
    o.mm.clear()
    del mx0, Lx0, mw0, Lw0
    g.gibbs_sweep(S - 1)
    # moment matching of stage-2 source blocks: rows of (1, 0) and (7, 0), columns
    # of (0, 1) and (0, 7)
    ridged = 0
    for b, side in ((J, 0), ((I - 1) * J, 0), (1, 1), (J - 1, 1)):
        ridged += _check_mm(g, b, side, K, S)
    assert ridged == 0
    # stage 3: every block
    g.pp_stage(3, 0)
    # the library's moments of the source blocks: rows of (i, 0), columns of (0, j)
    for i in range(1, I):
        mx, Lx = g.get_mm(i * J, 0)
        o.mm[i * J] = dict(x_mu=mx, x_Lam=Lx, ridged=0)
    for j in range(1, J):
        mw, Lw = g.get_mm(j, 1)
        o.mm[j] = dict(w_mu=mw, w_Lam=Lw, ridged=0)
    o.begin_stage(3)
    blocks3 = [b for b in range(I * J) if g.block_info(b)["stage"] == 3]
    assert len(blocks3) == (I - 1) * (J - 1)
    empty = few = 0
    for b in blocks3:
        blk = o.blocks[b]
        deg = np.diff(blk["csr_ptr"])
        empty += int((deg == 0).sum())
        few += int(((deg >= 1) & (deg <= 8)).sum())
        load_state(g, o, b, random_state(rng, blk["R"], blk["C"], K))
    print("stage 3: rows without entries", empty, "rows with 1-8 entries", few, flush=True)
    assert empty > 100000 and few > 100000
    _sweep_and_check("stage 3", g, o, blocks3, K, "bf16", 0)
    g.close()
