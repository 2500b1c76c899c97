"""Plain FP64 CPU oracle for the over-parameterised SOS objective.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library or its Python binding and never uses the closed-form ranking that the
GPU path uses; index maps here come from brute-force enumeration, sorting and
binary search.

Every function cites the passage of the paper it follows.  Pins (what each
function is checked against, other than itself) live in ``tests/test_oracle_*``.
"""
from .sos import (  # noqa: F401
    monomials,
    monomials_bruteforce,
    MonomialIndex,
    monomials_sparse,
    SparseIndex,
    merge_lists,
    pair_ranks,
    pair_ranks_sparse,
    coefficients,
    coefficients_abs,
    residual,
    loss_grad,
    poly_vector,
    evaluate_poly,
    evaluate_sos,
    adam_step,
    AdamState,
    solve,
    sample_coefficients,
    sample_gradient_rows,
)
from .convex import psd_distance  # noqa: F401
from .network import (  # noqa: F401
    network_chain,
    network_factor,
    network_loss_grad,
    network_quartic_coefficients,
)
