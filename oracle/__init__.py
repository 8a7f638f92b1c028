"""FP64 CPU oracle for dense CP-ALS with dimension trees, multi-sweep dimension
trees (MSDT) and pairwise perturbation (PP).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
statement of what the GPU path computes.  Only the test suite, the smoke check
of the entry module and the CPU-baseline leg of the benchmark may import it.
The product path (the HIP library and its Python binding) never imports, links
or calls anything here, and this package imports nothing from the product.

Conventions (the paper's notation, Sec. II-A, with C-order storage):
  * modes are 0-based in code (the paper counts from 1);
  * a tensor of shape (s_0, ..., s_{N-1}) is stored row-major (last index
    fastest); factor A[n] has shape (s_n, R);
  * the Khatri-Rao product of a list of factors puts the LEFT factor's index
    slowest, which matches the C-order flattening of the remaining modes.  The
    paper unfolds first-index-fastest and therefore writes the product in the
    reverse order; both give the same MTTKRP (Sec. II-B).

Parity pins: every function here is checked by tests marked "not gpu"
against brute force, closed forms, invariants or library routines; see the
module docstrings for which pin covers which function.  Functions without such
a pin say "parity unpinned" in their docstring.
"""

from .core import (  # noqa: F401
    krp,
    mttkrp_naive,
    mttkrp_bruteforce,
    partial_mttkrp,
    reconstruct,
    gram,
    gamma,
    spd_solve,
    residual_fast,
    residual_explicit,
)
from .als import als_sweep, als_run, AlsState  # noqa: F401
from .trees import DTCache, als_sweep_tree, dt_path, msdt_path, pp_tree_levels, dt_flops_closed, msdt_flops_closed  # noqa: F401
from .pp import (  # noqa: F401
    pp_operators,
    pp_mode_mttkrp,
    pp_v_literal,
    pp_v_recurrence,
    pp_approx_mttkrp,
    PPState,
    pp_als_step,
)
from .quant import e4m3_values, e4m3_round, quantize_columns  # noqa: F401
