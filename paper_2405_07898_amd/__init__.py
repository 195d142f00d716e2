"""MI355X-native EAM molecular-dynamics timestep loop (HIP kernels behind a C ABI).

The compute path is libmdeam.so (hand-written HIP for gfx950); this package is
its ctypes binding plus a torch autograd wrapper for force matching.
"""
from . import md  # noqa: F401
