"""MI355X-native Vecchia hot path (GraphGP): host graph build in C++, factor /
forward / inverse / logdet / adjoint in hand-written HIP for gfx950, behind
the C ABI of include/vecchia.h.  PyTorch provides device memory and streams.
"""
from ._lib import VecchiaError, load as load_library
from .vecchia import (EXP, M32, SE, M52, MATERN, FP64, FP32, KernelParams, Graph, DeviceGraph, Factor, FusedForward,
                      workspace_bytes)

__all__ = ["VecchiaError", "load_library", "EXP", "M32", "SE", "M52", "MATERN", "FP64", "FP32", "KernelParams", "Graph",
           "DeviceGraph", "Factor", "FusedForward", "workspace_bytes"]
