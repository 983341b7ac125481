"""MI355X (gfx950) ST-HOSVD: sequentially truncated HOSVD of dense N-way
tensors on one GPU, with hand-written HIP kernels behind the C-ABI declared
in ``include/tucker.h``.

The public functions live in :mod:`paper_1510_06689_amd.tucker`; importing
the package does not load the GPU library.
"""
from .tucker import (Compressor, TuckerError, TuckerTensor, error_metrics, gram,  # noqa: F401
                     library, reconstruct, sthosvd, ttm)

__all__ = ["Compressor", "TuckerError", "TuckerTensor", "error_metrics", "gram", "library",
           "reconstruct", "sthosvd", "ttm"]
