"""Dense orbital minimization method (OMM) on AMD Instinct MI355X.

The minimization runs in the HIP kernels of ``libomm.so`` (built in-tree by
``python -m paper_1312_1549_amd.build``); this package only marshals arguments to its C-ABI.
"""

from .omm import (  # noqa: F401
    OMM,
    OMMBatch,
    OMMBatchComplex,
    OMMComplex,
    OMMError,
    PRECISIONS,
    flops_per_iteration,
    omm_energy,
)
