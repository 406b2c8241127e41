"""MI355X (gfx950) implementation of the overlapping Rao-Blackwellized Monte
Carlo estimator of diag(Q^-1) and tr(Q^-1 dQ/dtheta) for space-time GMRFs
(arXiv 2309.05435).

The compute path is librbmc.so (HIP kernels behind the C ABI in
include/rbmc.h); ``binding`` is its ctypes binding and ``inputs`` the seeded
synthetic workload generator.  Importing the package loads nothing.
"""
__all__ = ["binding", "inputs", "build"]
