"""MI355X-native encrypted LIF inference: TFHE programmable bootstrapping on
gfx950 behind the C ABI of include/fhesnn.h.

The compute lives in libfhesnn.so (HIP kernels + host C++); ``fhesnn`` is
its ctypes binding and ``network`` drives LIF layers and whole networks
through it.
"""
from . import fhesnn  # noqa: F401
