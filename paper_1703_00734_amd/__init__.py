"""MI355X (gfx950) library for the BPMF Gibbs sweep of posterior-propagation
Bayesian matrix factorization (Qin et al., arXiv:1703.00734).

The compute path is libbmf.so (hand-written HIP, C ABI in include/bmf.h);
``binding`` marshals arguments to it.  Build with ``build.build()``.
"""
from .binding import BMF, BMFError, LIB_PATH, load, exported_symbols  # noqa: F401
