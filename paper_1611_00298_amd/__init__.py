"""MI355X (gfx950) EOFA hot path: Moebius domain-wall operator, Cayley-form
even-odd CG solves for the exact one-flavour algorithm, the EOFA action, its
pseudofermion force and its rational heatbath, and the Iwasaki gauge
action with its force (arXiv:1611.00298).

All arithmetic runs in libeofa.so (HIP kernels behind the C ABI in
include/eofa.h); this package only marshals torch tensors to it.
"""
from ._lib import EOFAError, PREC, load  # noqa: F401
from .api import (IWASAKI_C1, Context, dwf_apply, eofa_ctx_create, eofa_ctx_destroy,  # noqa: F401
                  eofa_ctx_update_gauge, eofa_force, eofa_gauge_action, eofa_gauge_force,
                  eofa_heatbath, eofa_md_update, eofa_solve, eofa_solve_dense, make_solver,
                  rational_inv_sqrt)
from .autograd import EOFAAction, eofa_action  # noqa: F401
