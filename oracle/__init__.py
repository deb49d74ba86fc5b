"""FP64 CPU oracle for the BPMF Gibbs sweep under posterior propagation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1703_00734_amd``) and never imports it.

Layout:
  bmf_oracle.c  -- Philox4x32-10, Box-Muller, Marsaglia-Tsang, Cholesky, the
                   row/column conditional update, NW and tau draws, SSE, MM.
  native.py     -- builds and loads bmf_oracle.c through ctypes.
  plan.py       -- ordering, r x c partition and per-block CSR/CSC (numpy).
  bpmf.py       -- the sweep order, PP stages, aggregation and prediction.
"""
from .native import build, lib  # noqa: F401
