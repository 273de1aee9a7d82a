"""MI355X (gfx950) library for the 2-D five-point Jacobi (Laplace) sweep.

The computation is the hot path of the stencil abstraction in "An Adaptive
Distributed Stencil Abstraction for GPUs" (listing of the 2-D Laplace solver,
Section III-A; benchmarks of Section V). All arithmetic runs in the HIP
kernels of ``libsten.so`` (C ABI in ``include/sten.h``); this package only
marshals arguments. There is no CPU fallback: loading fails loudly when the
library is missing.
"""

from ._lib import StenError, load  # noqa: F401
from .ops import (  # noqa: F401
    BatchPlan,
    TiledGrid,
    HiLoGrid,
    hilo_decode,
    hilo_encode,
    jacobi5,
    jacobi5_tb,
    jacobi5_hilo,
    jacobi5_hilo_encoded,
    set_hilo_variant,
    set_sweep_rows,
    star,
    star_iterate,
    sweep,
)

__all__ = ["StenError", "load", "BatchPlan", "TiledGrid", "jacobi5", "jacobi5_tb", "jacobi5_hilo", "jacobi5_hilo_encoded", "hilo_encode",
           "hilo_decode", "HiLoGrid", "set_sweep_rows", "set_hilo_variant", "sweep", "star", "star_iterate"]
