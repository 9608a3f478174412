"""MI355X-native explicit step of the Optimal Transportation Meshfree method.

The compute path is libotm.so (hand-written HIP for gfx950) behind the C ABI
in include/otm.h.  ``_lib`` is the ctypes view of that ABI and ``sim`` keeps
the device state in torch tensors.
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = []
