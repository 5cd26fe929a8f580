"""MI355X-native encrypted linear-layer product of Pencil (NDSS 2024).

The model owner's homomorphic product of a linear layer (Alg. 1 forward, the
input gradient by the same pattern, Alg. 2's weight-gradient cross terms) on
coefficient-encoded RNS-BFV ciphertexts, as HIP kernels for gfx950 behind the
C ABI of include/pencil.h.  This package is the binding: argument marshalling
over ctypes, PyTorch for device memory and streams.
"""
from ._abi import PencilError, load  # noqa: F401
from .api import Context, Step, layer_struct, plan_struct, plan_dict  # noqa: F401
