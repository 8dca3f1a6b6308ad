"""MI355X (gfx950) fast multipole method: the per-rank hot path of
AbdulJabbar, Yokota & Keyes, "Asynchronous Execution of the Fast Multipole
Method Using Charm++" (arXiv 1405.7487).

Tree build, dual tree traversal, P2M/M2M, M2L, L2L/L2P, P2P and the adjoint
all run as HIP kernels in ``libfmm_hip.so`` behind the C ABI of
``include/fmm.h``; this package only marshals arguments.
"""
from ._binding import (  # noqa: F401
    CallbackAllocator,
    EXPORTS,
    FMMError,
    FMMFunction,
    LIB_PATH,
    Params,
    Plan,
    build,
    evaluate,
    evaluate_noalloc,
    let_evaluate,
    load,
    mfma_layout,
)
