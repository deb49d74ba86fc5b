"""Write sim30_oracle_rmse.txt: the oracle's test RMSE on the paper's simulated
workload (Sec. 5.3: 6040 x 3706, K = 5, tau = 1 fixed, 80 % of the cells missing
at random, data seed 1) at the 30 x 30 partition in random order, with the
paper's schedule (1200 sweeps, 800 burn-in, every second sample kept; Sec. 5.2),
moment-matched propagation and Algorithm 2, for two chain seeds.

Run from the repository root:  python tests/golden/make_sim30_oracle.py
(about 4 minutes per chain on 8 host cores)."""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle.bpmf import Oracle  # noqa: E402

SEEDS = (101, 104)


def main():
    d = synth.simulated(1, "mar")
    lines = ["# Oracle test RMSE, simulated workload (data seed 1, missing at random), 30 x 30",
             "# partition, random order, 1200 sweeps / 800 burn-in / thin 2, moment matching.",
             "# Written by tests/golden/make_sim30_oracle.py.",
             "# chain_seed  rmse  agg_corrections"]
    for seed in SEEDS:
        t0 = time.time()
        o = Oracle(d["N"], d["D"], 5, d["row"], d["col"], d["val"], I=30, J=30, order="random",
                   sample_tau=False, tau_fixed=1.0, seed=seed, burnin=800, thin=2)
        o.run_pp(1200)
        o.aggregate()
        p = o.predict(d["test_row"], d["test_col"])
        rmse = float(np.sqrt(np.mean((p - d["test_val"]) ** 2)))
        print("seed %d: rmse %.6f, corrections %d, %.0f s" % (seed, rmse, o.corrections, time.time() - t0),
              flush=True)
        lines.append("%d %.6f %d" % (seed, rmse, o.corrections))
    with open(os.path.join(HERE, "sim30_oracle_rmse.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
