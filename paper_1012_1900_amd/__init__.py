"""gammax: gamma-index dose comparison on AMD Instinct MI355X (gfx950).

The method of Gu, Jia & Jiang, "GPU-based fast gamma index calculation" (Sec. 2,
Algorithms A1/A2), computed by the hand-written HIP kernels of ``libgammax.so``.
This package is the thin Python binding of its C ABI (``include/gammax.h``).
"""
from ._abi import (  # noqa: F401
    Context,
    GammaResult,
    Model,
    MODEL_NPARAM,
    model_features,
    predict_nodes,
    GammaxError,
    build_table,
    context,
    gamma_map,
    gammax_batch,
    gammax_map,
    gammax_map_async,
    gammax_map_many,
    gammax_map_noalloc,
    NOALLOC_MAX_NODES,
    NOALLOC_MAX_TABLE,
    gammax_map_grids,
    MapTicket,
    ASYNC_SLOTS,
    pass_count,
    sort_pairs,
    status_string,
    tune_load,
    tune_save,
    LIB_PATH,
)
