"""N-BVH neural ray queries and training on MI355X (gfx950).

The compute lives in libnbvh.so (hand-written HIP kernels behind the C ABI of
include/nbvh.h); this package only marshals torch tensors into those calls.
"""
from ._abi import NbvhError, load  # noqa: F401
from .nbvh import NBVH, NBVHBatch, hits_leaf, make_config  # noqa: F401
from .autograd import NBVHFunction, nbvh_forward  # noqa: F401

__all__ = ["NBVH", "NBVHBatch", "NBVHFunction", "NbvhError", "hits_leaf", "load", "make_config", "nbvh_forward"]
