"""Krylov-space equilibrium / nonequilibrium Green's functions on MI355X.

Thin Python binding of libkgf.so (HIP, gfx950).  Every numerical step runs
in the library's kernels; this module only marshals arguments (torch
tensors are passed as device pointers on the current stream).  There is no
CPU fallback: importing the binding without the built library raises.

Method: Balzer, Gdaniec & Potthoff, "Krylov-space approach to the
equilibrium and the nonequilibrium single-particle Green's function".
"""
from ._lib import (KgfError, Context, Model, Sector, lib_path, load_library,  # noqa: F401
                   DIRECTION_FORWARD, DIRECTION_BACKWARD, DIRECTION_IMAGINARY)

__all__ = ["KgfError", "Context", "Model", "Sector", "lib_path", "load_library",
           "DIRECTION_FORWARD", "DIRECTION_BACKWARD", "DIRECTION_IMAGINARY"]
