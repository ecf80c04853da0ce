"""Gaussian beam summation on AMD Instinct MI355X (gfx950).

The compute path is the HIP library libgbs.so (C ABI in include/gbs.h);
this package is its Python binding.  Importing it does not load the
library; the first call does, and fails loudly if it is not built.
"""
from .gbs import (Context, GBSFunction, Graph, Table, air_absorption, autotune, backward, context, forward,
                  forward_noalloc, impulse_response, stats, trace)

__all__ = ["Context", "GBSFunction", "Graph", "Table", "air_absorption", "autotune", "backward", "context",
           "forward", "forward_noalloc", "impulse_response", "stats", "trace"]


def build(verbose: bool = False) -> str:
    from .build import build as _build
    return _build(verbose=verbose)
