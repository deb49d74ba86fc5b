"""The oracle's BPMF chain, posterior-propagation stages, aggregation, prediction.

TEST INFRASTRUCTURE ONLY (FP64).  Sweep order and readings:

* r_nd = y_nd - y_bar with y_bar the sequential FP64 mean of the training
  values; predictions add y_bar back (centering is a reading: the paper does
  not state it).
* Stages (Sec. 3.2, eq. stage1, stage2a, stage2b, stage3; Algorithm 1), 0-based
  block (i, j): stage 1 is (0, 0); stage 2 the blocks with exactly one zero
  index; stage 3 the rest.  The X side of (i, j) is propagated iff j > 0, from
  the moment-matched X of block (i, 0); the W side iff i > 0, from the W of
  block (0, j).  A propagated side takes no Normal-Wishart draw (Sec. 5.1).
* Initialisation (reading): a propagated side starts at the propagated means;
  other factors at K^(-1/4) z; hyperparameters (mu, Lambda) = (0, I);
  tau = tau_fixed, or a0 / b0 when tau is sampled.
* Sweep t of a block: (a) every row given W, (b) every column given the new X,
  (c) NW draw for X if not propagated, (d) NW draw for W if not propagated,
  (e) tau ~ Gamma if sampled, (f) keep the sample if t >= burnin and
  (t - burnin) % thin == 0.
* Moment matching at the end of a stage (Sec. 4.1): per-row mean and inverse
  sample covariance (1/(S-1) normaliser, ridge when S <= K or not SPD).
* Dominant mode and mixture approximations (Sec. 4.1; Sec. 5.1): each row's
  kept samples are clustered by lambda-means (orc_lmeans, with its readings);
  the dominant-mode fit is the moment matching of the largest cluster (lowest
  index on ties; all samples when it has fewer than two); the mixture keeps the
  `ncomp` largest clusters with at least two members (all samples as one
  component when none has), weights proportional to their sizes, each
  component moment-matched.  A mixture prior (Sec. 5.1, GMM prior Gibbs) is
  applied per row and sweep as the component of largest pi_c N(x_n | mu_c,
  Lambda_c^-1) at the row's current value (lowest index on ties); a side
  propagated by a mixture starts at the mean of its largest component.  For
  aggregation a mixture is pooled (Sec. 4.2, eq. marginal_mixture): mean
  sum_c pi_c mu_c, covariance sum_c pi_c (Lambda_c^-1 + (mu_c - mu)(mu_c - mu)^T).
* Aggregation (Sec. 4.2, eq. post_marg_aggregation and Algorithm 2): for the
  rows of row block i the base is block (i, 0) and the siblings are (i, j),
  j >= 1; for a column block j the base is (0, j) and the siblings (i, j),
  i >= 1.  A sibling whose difference to the base is not SPD is corrected by
  (|lambda_min| + eps) I with eps = 1e-6 tr(Lambda_base) / K (the "small
  constant" is a reading).  With no siblings, mu* is the base mean itself.
* Prediction (Sec. 5.2): y_hat = y_bar + mu*_x^T mu*_w with posterior means.
* Per-column noise precisions (the tau_d variant of Sec. 2.1, tau_per_column):
  y_nd ~ N(x_n^T w_d, 1/tau_d) with tau_d ~ Gamma(a0, b0) per column of each
  block; the row update weights each entry by its column's tau_d, the column
  update uses its own tau_d, and the draw is tau_d ~ Gamma(a0 + M_d/2,
  b0 + SSE_d/2) over the column's M_d entries, on counter (d, t, TAU, k).
"""
import numpy as np

from . import native
from .native import ptr
from .plan import Plan, counter_c2, stage_of


def nw_scale_inverse(W0):
    L = native.cholesky(W0)
    if L is None:
        raise ValueError("W0 must be SPD")
    Li = np.linalg.solve(L, np.eye(W0.shape[0]))
    return np.ascontiguousarray(Li.T @ Li)


class Oracle:
    def __init__(self, N, D, K, row, col, val, I=1, J=1, order="given", mu0=None, beta0=2.0,
                 nu0=None, W0=None, sample_tau=True, tau_a0=1.0, tau_b0=1.0, tau_fixed=1.0,
                 seed=0, burnin=0, thin=1, nthreads=0, approx="mm", lambda_scale=2.0, ncomp=3,
                 tau_per_column=False):
        self.tau_per_column = bool(tau_per_column)
        if approx not in ("mm", "dm", "gmm"):
            raise ValueError("approx must be mm, dm or gmm")
        self.approx, self.lambda_scale, self.ncomp = approx, float(lambda_scale), int(ncomp)
        self.N, self.D, self.K = int(N), int(D), int(K)
        self.I, self.J = int(I), int(J)
        self.seed = int(seed)
        self.mu0 = np.zeros(K) if mu0 is None else np.asarray(mu0, dtype=np.float64).copy()
        self.beta0 = float(beta0)
        self.nu0 = float(K if nu0 is None else nu0)
        W0 = np.eye(K) if W0 is None else np.asarray(W0, dtype=np.float64)
        self.W0inv = nw_scale_inverse(W0)
        self.sample_tau = bool(sample_tau)
        self.a0, self.b0, self.tau_fixed = float(tau_a0), float(tau_b0), float(tau_fixed)
        self.burnin, self.thin = int(burnin), int(thin)
        self.nthreads = int(nthreads)
        val = np.asarray(val, dtype=np.float32)
        self.ybar = native.seq_mean(val)
        self.plan = Plan(N, D, row, col, I, J, order, seed)
        r = val.astype(np.float64) - self.ybar
        self.blocks = []
        for b, pb in enumerate(self.plan.blocks):
            blk = dict(pb)
            blk["b"] = b
            blk["stage"] = stage_of(pb["i"], pb["j"])
            blk["csr_val"] = np.ascontiguousarray(r[pb["csr_entry"]])
            blk["csc_val"] = np.ascontiguousarray(r[pb["csc_entry"]])
            blk["x_prop"] = pb["j"] > 0
            blk["w_prop"] = pb["i"] > 0
            self.blocks.append(blk)
        self.stage = 0
        self.mm = {}          # block -> dict(x_mu, x_Lam, w_mu, w_Lam, ridged)

    # ------------------------------------------------------------------ stages
    def stage_blocks(self, s):
        return [blk for blk in self.blocks if blk["stage"] == s]

    def begin_stage(self, s):
        K = self.K
        for blk in self.stage_blocks(s):
            b, i, j = blk["b"], blk["i"], blk["j"]
            if blk["x_prop"]:
                src = self.mm[i * self.J + 0]
                if self.approx == "gmm":
                    blk["x_prior"] = ("gmm", src["x_gmm"])
                    blk["X"] = src["x_gmm"]["mu"][:, 0].copy()
                else:
                    blk["x_prior"] = (src["x_Lam"], src["x_mu"])
                    blk["X"] = src["x_mu"].copy()
            else:
                blk["x_prior"] = None
                X = np.zeros((blk["R"], K))
                native.lib().orc_init_side(blk["R"], K, self.seed, counter_c2(b, "INIT_X"), ptr(X))
                blk["X"] = X
            if blk["w_prop"]:
                src = self.mm[0 * self.J + j]
                if self.approx == "gmm":
                    blk["w_prior"] = ("gmm", src["w_gmm"])
                    blk["W"] = src["w_gmm"]["mu"][:, 0].copy()
                else:
                    blk["w_prior"] = (src["w_Lam"], src["w_mu"])
                    blk["W"] = src["w_mu"].copy()
            else:
                blk["w_prior"] = None
                W = np.zeros((blk["C"], K))
                native.lib().orc_init_side(blk["C"], K, self.seed, counter_c2(b, "INIT_W"), ptr(W))
                blk["W"] = W
            blk["hx"] = (np.eye(K), np.zeros(K))      # (Lambda_X, mu_X)
            blk["hw"] = (np.eye(K), np.zeros(K))
            blk["tau"] = self.a0 / self.b0 if self.sample_tau else self.tau_fixed
            if self.tau_per_column:
                blk["tau"] = np.full(blk["C"], blk["tau"])
            blk["t"] = 0
            blk["samples_x"] = []
            blk["samples_w"] = []
        self.stage = s

    # -------------------------------------------------------------- sub-steps
    def update_rows(self, blk, t=None):
        t = blk["t"] if t is None else t
        self._update(blk, "rows", t)

    def update_cols(self, blk, t=None):
        t = blk["t"] if t is None else t
        self._update(blk, "cols", t)

    def _update(self, blk, which, t):
        K = self.K
        if which == "rows":
            n, ptr_, idx, val = blk["R"], blk["csr_ptr"], blk["csr_idx"], blk["csr_val"]
            other, prop, hyp, purpose, key = blk["W"], blk["x_prior"], blk["hx"], "ROW", "X"
        else:
            n, ptr_, idx, val = blk["C"], blk["csc_ptr"], blk["csc_idx"], blk["csc_val"]
            other, prop, hyp, purpose, key = blk["X"], blk["w_prior"], blk["hw"], "COL", "W"
        if prop is not None and isinstance(prop[0], str):
            choice = gmm_choice(prop[1], blk[key])
            blk[key + "_choice"] = choice
            rows = np.arange(n)
            P = np.ascontiguousarray(prop[1]["Lam"][rows, choice])
            m = np.ascontiguousarray(prop[1]["mu"][rows, choice])
            per_row = 1
        elif prop is not None:
            P = np.ascontiguousarray(prop[0])
            m = np.ascontiguousarray(prop[1])
            per_row = 1
        else:
            P = np.ascontiguousarray(hyp[0])
            m = np.ascontiguousarray(hyp[1])
            per_row = 0
        out = blk[key].copy()
        other = np.ascontiguousarray(other)
        if self.tau_per_column:
            # rows: entry weights tau_d of the gathered columns; columns: their own tau_d
            tcol = np.ascontiguousarray(blk["tau"], dtype=np.float64)
            wt, taus = (tcol, None) if which == "rows" else (None, tcol)
            fails = native.lib().orc_update_side_w(
                n, K, ptr(ptr_), ptr(idx), ptr(val), ptr(other), ptr(wt), ptr(taus), per_row, ptr(P),
                ptr(m), 1.0, self.seed, t & 0xFFFFFFFF, counter_c2(blk["b"], purpose), ptr(out), self.nthreads)
        else:
            fails = native.lib().orc_update_side(
                n, K, ptr(ptr_), ptr(idx), ptr(val), ptr(other), per_row, ptr(P), ptr(m),
                float(blk["tau"]), self.seed, t & 0xFFFFFFFF, counter_c2(blk["b"], purpose),
                ptr(out), self.nthreads)
        if fails:
            raise FloatingPointError("oracle: %d non-SPD conditional precisions" % fails)
        blk[key] = out

    def hyper_draw(self, blk, side, t=None):
        t = blk["t"] if t is None else t
        K = self.K
        X = np.ascontiguousarray(blk["X"] if side == "x" else blk["W"])
        Lam = np.zeros((K, K))
        mu = np.zeros(K)
        purpose = "HYPER_X" if side == "x" else "HYPER_W"
        rc = native.lib().orc_nw_draw(X.shape[0], K, ptr(X), ptr(self.mu0), self.beta0, self.nu0,
                                      ptr(self.W0inv), self.seed, t & 0xFFFFFFFF,
                                      counter_c2(blk["b"], purpose), ptr(Lam), ptr(mu))
        if rc != 0:
            raise FloatingPointError("oracle: NW draw failed")
        blk["hx" if side == "x" else "hw"] = (Lam, mu)

    def sse(self, blk):
        return native.lib().orc_sse(blk["R"], self.K, ptr(blk["csr_ptr"]), ptr(blk["csr_idx"]),
                                    ptr(blk["csr_val"]), ptr(np.ascontiguousarray(blk["X"])),
                                    ptr(np.ascontiguousarray(blk["W"])))

    def col_sse(self, blk):
        """Residual SSE of every column of a block (entries in CSC order)."""
        X, W = blk["X"], blk["W"]
        cols = np.repeat(np.arange(blk["C"]), np.diff(blk["csc_ptr"]))
        res = blk["csc_val"] - np.einsum("ek,ek->e", X[blk["csc_idx"]], W[cols])
        return np.bincount(cols, weights=res * res, minlength=blk["C"])

    def tau_draw(self, blk, t=None):
        t = blk["t"] if t is None else t
        if self.tau_per_column:
            sse = np.ascontiguousarray(self.col_sse(blk))
            cnt = np.ascontiguousarray(np.diff(blk["csc_ptr"]).astype(np.int64))
            tau = np.zeros(blk["C"])
            native.lib().orc_tau_cols(blk["C"], ptr(sse), ptr(cnt), self.a0, self.b0, self.seed, t & 0xFFFFFFFF,
                                      counter_c2(blk["b"], "TAU"), ptr(tau))
            blk["tau"] = tau
            return
        s = self.sse(blk)
        blk["tau"] = native.lib().orc_tau_draw(s, blk["M"], self.a0, self.b0, self.seed,
                                               t & 0xFFFFFFFF, counter_c2(blk["b"], "TAU"))

    def sweep_block(self, blk):
        t = blk["t"]
        self.update_rows(blk, t)
        self.update_cols(blk, t)
        if not blk["x_prop"]:
            self.hyper_draw(blk, "x", t)
        if not blk["w_prop"]:
            self.hyper_draw(blk, "w", t)
        if self.sample_tau:
            self.tau_draw(blk, t)
        if t >= self.burnin and (t - self.burnin) % self.thin == 0:
            blk["samples_x"].append(blk["X"].copy())
            blk["samples_w"].append(blk["W"].copy())
        blk["t"] = t + 1

    def sweep(self, n=1):
        for _ in range(n):
            for blk in self.stage_blocks(self.stage):
                self.sweep_block(blk)

    # ------------------------------------------------------------ moment match
    def finalize_stage(self):
        for blk in self.stage_blocks(self.stage):
            self.mm[blk["b"]] = self.moment_match(blk)

    def moment_match(self, blk):
        out = {}
        ridged = 0
        for side in ("x", "w"):
            S = len(blk["samples_" + side])
            if S < 1:
                raise RuntimeError("no kept samples in block %d" % blk["b"])
            smp = np.ascontiguousarray(np.stack(blk["samples_" + side]))
            R = smp.shape[1]
            mu = np.zeros((R, self.K))
            Lam = np.zeros((R, self.K, self.K))
            if S >= 2 and self.approx != "mm":
                fit = self.cluster_fit(smp)
                ridged += fit.pop("ridged")
                mu, Lam = fit.pop("mu"), fit.pop("Lam")
                out[side + "_labels"] = fit.pop("labels")
                if self.approx == "gmm":
                    out[side + "_gmm"] = dict(pi=fit["pi"], mu=fit["cmu"], Lam=fit["cLam"], logdet=fit["logdet"])
            elif S >= 2:
                ridged += native.lib().orc_mm(R, self.K, S, ptr(smp), ptr(mu), ptr(Lam))
            else:
                mu[:] = smp[0]
                Lam[:] = np.nan
            out[side + "_mu"] = mu
            out[side + "_Lam"] = Lam
        out["ridged"] = ridged
        return out

    def cluster_fit(self, smp):
        """Dominant-mode or mixture fit of one side from its samples (S, R, K)."""
        S, R, K = smp.shape
        lab = np.zeros((R, S), dtype=np.int32)
        ncl = np.zeros(R, dtype=np.int32)
        native.lib().orc_lmeans(R, K, S, ptr(smp), self.lambda_scale, LMEANS_CMAX, LMEANS_MAXIT,
                                ptr(lab), ptr(ncl))
        sizes = np.zeros((R, LMEANS_CMAX), dtype=np.int64)
        for q in range(S):
            sizes[np.arange(R), lab[:, q]] += 1
        # clusters by decreasing size, lower index first on ties
        order = np.argsort(-sizes, axis=1, kind="stable")
        C = 1 if self.approx == "dm" else self.ncomp
        which = np.full((R, C), -2, dtype=np.int32)          # -2: no component
        for c in range(C):
            cid = order[:, c]
            ok = sizes[np.arange(R), cid] >= 2
            which[ok, c] = cid[ok]
        none = which[:, 0] == -2
        which[none, 0] = -1                                  # every sample
        cnt_sel = np.zeros((R, C), dtype=np.int32)
        mu = np.zeros((R, C, K))
        Lam = np.zeros((R, C, K, K))
        logdet = np.zeros((R, C))
        ridged = 0
        for c in range(C):
            has = which[:, c] != -2
            w = np.where(has, which[:, c], -1).astype(np.int32)
            m = np.zeros((R, K))
            L = np.zeros((R, K, K))
            ld = np.zeros(R)
            cn = np.zeros(R, dtype=np.int32)
            rid = native.lib().orc_mm_sel(R, K, S, ptr(smp), ptr(lab), ptr(w), ptr(m), ptr(L), ptr(ld), ptr(cn))
            if c == 0:
                ridged += rid
            mu[:, c], Lam[:, c], logdet[:, c], cnt_sel[:, c] = m, L, ld, np.where(has, cn, 0)
        if self.approx == "dm":
            return dict(mu=mu[:, 0], Lam=Lam[:, 0], labels=lab, ridged=ridged)
        pi = cnt_sel / cnt_sel.sum(1, keepdims=True)
        # pooled moments for aggregation (eq. marginal_mixture)
        mp = np.einsum("nc,nck->nk", pi, mu)
        Sig = np.zeros((R, K, K))
        for c in range(C):
            dm = mu[:, c] - mp
            Sc = np.linalg.inv(Lam[:, c])
            Sig += pi[:, c, None, None] * (Sc + dm[:, :, None] * dm[:, None, :])
        return dict(mu=mp, Lam=np.linalg.inv(Sig), labels=lab, ridged=ridged,
                    pi=pi, cmu=mu, cLam=Lam, logdet=logdet)

    def run_stage(self, s, nsweeps):
        self.begin_stage(s)
        self.sweep(nsweeps)
        self.finalize_stage()

    def run_pp(self, nsweeps):
        for s in (1, 2, 3):
            if self.stage_blocks(s):
                self.run_stage(s, nsweeps)

    # -------------------------------------------------------------- aggregate
    def aggregate(self):
        """Per-row aggregated means (Algorithm 2) for every row and column block."""
        I, J, K = self.I, self.J, self.K
        self.mu_x, self.lam_x = [], []
        self.mu_w, self.lam_w = [], []
        self.corrections = 0
        for i in range(I):
            base = self.mm[i * J + 0]
            sib = [self.mm[i * J + j] for j in range(1, J)]
            lam = []
            mu, ncor = aggregate_side(base["x_mu"], base["x_Lam"],
                                      [s["x_mu"] for s in sib], [s["x_Lam"] for s in sib], K, lam)
            self.corrections += ncor
            self.mu_x.append(mu)
            self.lam_x.append(np.array(lam))
        for j in range(J):
            base = self.mm[0 * J + j]
            sib = [self.mm[i * J + j] for i in range(1, I)]
            lam = []
            mu, ncor = aggregate_side(base["w_mu"], base["w_Lam"],
                                      [s["w_mu"] for s in sib], [s["w_Lam"] for s in sib], K, lam)
            self.corrections += ncor
            self.mu_w.append(mu)
            self.lam_w.append(np.array(lam))

    def predict(self, row, col):
        """y_hat = y_bar + mu*_x^T mu*_w for every pair (original ids)."""
        p = self.plan
        row = np.asarray(row, dtype=np.int64)
        col = np.asarray(col, dtype=np.int64)
        # aggregated means of every row and column, indexed by original id
        mx = np.empty((self.N, self.K))
        mw = np.empty((self.D, self.K))
        for i in range(self.I):
            mx[p.row_ids[i]] = self.mu_x[i]
        for j in range(self.J):
            mw[p.col_ids[j]] = self.mu_w[j]
        out = np.empty(row.size, dtype=np.float64)
        step = 1 << 20
        for a in range(0, row.size, step):
            b = min(row.size, a + step)
            out[a:b] = self.ybar + np.einsum("qk,qk->q", mx[row[a:b]], mw[col[a:b]])
        return out


LMEANS_CMAX = 16      # clusters per row at most (lambda-means reading)
LMEANS_MAXIT = 32     # lambda-means rounds at most


def gmm_choice(g, X):
    """Per row, the component c of largest log pi_c + log det(Lambda_c) / 2
    - (x - mu_c)^T Lambda_c (x - mu_c) / 2 at the current value x (the common
    constant of the Gaussian densities cancels); components with pi_c = 0 are
    absent; the lowest index wins a tie."""
    R, C, K = g["mu"].shape
    best = np.zeros(R, dtype=np.int64)
    bval = np.full(R, -np.inf)
    for c in range(C):
        d = X - g["mu"][:, c]
        q = np.einsum("nk,nkl,nl->n", d, g["Lam"][:, c], d)
        v = np.where(g["pi"][:, c] > 0, np.log(np.maximum(g["pi"][:, c], 1e-300)) + 0.5 * g["logdet"][:, c] - 0.5 * q,
                     -np.inf)
        take = v > bval
        best[take] = c
        bval[take] = v[take]
    return best


def aggregate_side(mu_b, Lam_b, mus, Lams, K, lam_out=None):
    """Algorithm 2 for every row of one side: returns (mu*, #corrections); the
    aggregated precisions Lambda* are appended to lam_out when it is a list."""
    if not mus:
        if lam_out is not None:
            lam_out.extend(np.array(Lam_b))
        return mu_b.copy(), 0
    R = mu_b.shape[0]
    Jn = len(mus) + 1
    out = np.zeros_like(mu_b)
    ncor = 0
    for n in range(R):
        Lb = Lam_b[n]
        eps = 1e-6 * np.trace(Lb) / K
        Lstar = (2 - Jn) * Lb
        rhs = (2 - Jn) * (Lb @ mu_b[n])
        for mj, Lj in zip(mus, Lams):
            Dj = Lj[n] - Lb
            if native.cholesky(Dj) is not None:
                Lsj = Lj[n]
            else:
                lam_min = np.linalg.eigvalsh(Dj)[0]
                Lsj = Dj + (abs(lam_min) + eps) * np.eye(K) + Lb
                ncor += 1
            Lstar = Lstar + Lsj
            rhs = rhs + Lsj @ mj[n]
        out[n] = np.linalg.solve(Lstar, rhs)
        if lam_out is not None:
            lam_out.append(Lstar)
    return out, ncor
