"""MI355X (gfx950) implementation of robust blockwise random pivoting (RBRP)
for the interpolative decomposition (Dong, Chen, Martinsson, Pearce,
arXiv:2309.16002).

The computation runs in the HIP library ``lib/librbrp.so`` (C ABI in
``include/rbrp.h``); this package is its thin Python binding.
"""

from ._binding import (  # noqa: F401
    LIB_PATH, BatchPlan, IDResult, RBRPError, batch_autotune, block_cpqr, err_bound_increment,
    lib, rbrp_id, rbrp_id_batched, rbrp_id_batched_noalloc, row_norms, sample_block,
    sketchy_id, status_string, workspace_size,
)
