"""qdpath: Newton corrector and path tracker for polynomial homotopies in
double-double / quad-double complex arithmetic, as HIP kernels for MI355X
(gfx950) behind the C-ABI in ``include/qdpath.h``.

The Python layer only marshals arguments (``binding``); the compute path is
``libqdpath.so``.
"""

from .binding import (  # noqa: F401
    ELIM_AUTO,
    ELIM_BLOCKS,
    ELIM_COLUMNS,
    ELIM_POINT,
    PRED_LEARNED,
    PRED_QUADRATIC,
    PRED_SECANT,
    QDP_DD,
    QDP_F64,
    QDP_QD,
    SOLVE_FULL,
    SOLVE_MIXED_IR,
    Homotopy,
    Policy,
    QdpError,
    System,
    arith_batch,
    default_track_params,
    eval_homotopy,
    eval_homotopy_dev,
    eval_jacobian,
    eval_jacobian_dev,
    eval_homotopy_batch_dev,
    last_info,
    last_info_batch,
    newton_batch_dev,
    lib,
    newton_step,
    newton_step_dev,
    newton_step_noalloc_dev,
    info_from_bytes,
    set_elimination,
    track_path,
    track_paths,
    version,
)
