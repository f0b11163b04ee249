"""MI355X (gfx950) kernel-polynomial-method library for the renormalized
mean-field t-t'-J model with vortices (arXiv:2212.05685, App. B).

The compute path is the HIP library libkpm.so (C ABI in include/kpm.h);
``kpm`` is its ctypes binding, ``solver`` a convenience layer that allocates
torch device buffers, and ``autograd.GrandPotential`` exposes the grand
potential as a differentiable torch function whose backward pass is the
adjoint Chebyshev kernel.
"""
from . import kpm  # noqa: F401  (raises ImportError if libkpm.so is missing)

__all__ = ["kpm"]
