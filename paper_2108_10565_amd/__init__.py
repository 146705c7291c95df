"""MI355X-native element-local space-time predictor of ADER-DG for Biot
poroelasticity (Wolf et al., arXiv 2108.10565): block-wise back-substitution
(Algorithm 3) in hand-written HIP kernels for gfx950 behind a C ABI.

    from paper_2108_10565_amd import predict
    Q, Qint = predict(Q0, star, E, dt, degree)        # torch tensors on cuda

The Python layer only marshals arguments; see ``include/stp.h``.
"""
from .api import (flops, predict, reference_matrices, validate, workspace_size)  # noqa: F401
from ._lib import StpError  # noqa: F401
