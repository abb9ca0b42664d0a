"""MI355X-native randomized SVD (Halko-Martinsson-Tropp range finder over
block-cyclic tiles with power iteration), behind the C ABI of librsvd.so.

    from paper_1907_06470_amd import factor, Plan
    U, S, V, info = factor(A_cuda_fp32, k=100, p=20, q=2)
"""

from .api import Checkpoint, Plan, RSVD, factor, omega, philox_raw, col_major  # noqa: F401

__all__ = ["Checkpoint", "Plan", "RSVD", "factor", "omega", "philox_raw", "col_major"]
