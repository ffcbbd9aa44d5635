"""Seeded synthetic inputs for the N-BVH neural ray query and training step.

Input preparation only: meshes, neural-leaf boxes, rays, probe segments and
their classical (Moller-Trumbore) ground truth. Shared by the GPU library's
tests/benchmark and by the FP64 oracle; it contains none of the neural query's
own arithmetic (traversal of the neural BVH, hash encoding, MLP, losses).
"""
from . import scene, configs  # noqa: F401
from .configs import NetConfig, init_params, make_scene  # noqa: F401
