"""pkm: preconditioned CG on kernel matrices for AMD MI355X (gfx950).

The compute path is the HIP library libpkm.so (C ABI in include/pkm.h);
``binding`` marshals arguments to it.  Importing the package does not load
the library; the first binding call does, and fails loudly if it is missing.
"""
from . import binding  # noqa: F401

__all__ = ["binding"]
