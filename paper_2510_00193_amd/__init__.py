"""MI355X (gfx950) Moment Tensor Potential library: Python side of libmtp.so.

The hot path (neighbour list, radial basis, moments, contractions, energy,
adjoint to forces and virial, extrapolation grade, parameter gradients) runs
in hand-written HIP kernels behind the C ABI declared in include/mtp.h.
This package only builds the library and marshals arguments to it.
"""
from .api import Batch, NeighborList, Potential, compiled_levels, level_info  # noqa: F401
from .autograd import MTPBatchFunction, MTPFunction, batch_energy_forces, energy_forces  # noqa: F401
