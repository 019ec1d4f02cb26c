"""CPU oracle for butterfly-format ALS completion (test infrastructure only).

This package is a plain, slow FP64/complex128 NumPy statement of what the GPU
library computes.  It exists to check the GPU path; it is not part of the
product.  Only the tests, the smoke check and the bench's CPU-baseline leg may
import it.  It shares no code with the HIP library or its Python binding.
"""
from .butterfly_als import (  # noqa: F401
    OracleNotSPD,
    block_keys,
    core_shapes,
    digits,
    dense_tensor_network,
    design_matrix_bruteforce,
    design_rows,
    left_env,
    right_env,
    num_blocks,
    objective,
    predict,
    psi_inv,
    relative_error,
    residual_sq,
    run_als,
    sweep,
    update_core,
)
from .lowrank_to_butterfly import (  # noqa: F401
    householder_qrcp,
    lowrank_to_butterfly,
    side_levels,
    sketch_shapes,
)
from .adam import adam_state, adam_sweep, adam_update, gradient  # noqa: F401
from .adf import (  # noqa: F401
    adf_core_step,
    adf_sweep,
    orthogonalize_left,
    orthogonalize_right,
    right_to_left_sweep,
)
from . import mlp  # noqa: F401
