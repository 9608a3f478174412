"""MI355X-native explicit step of the Optimal Transportation Meshfree method.

The compute path is libotm.so (hand-written HIP for gfx950) behind the C ABI
in include/otm.h.  ``_lib`` is the ctypes view of that ABI, ``sim`` keeps
the device state in torch tensors (``Sim``) and ``adjoint`` holds the
checkpointed reverse-mode rollout (``OTMRollout``, ``OTMRolloutField``).
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["Sim", "OTMRollout", "OTMRolloutField"]


def __getattr__(name):
    if name == "Sim":
        from .sim import Sim
        return Sim
    if name in ("OTMRollout", "OTMRolloutField"):
        from . import adjoint
        return getattr(adjoint, name)
    raise AttributeError(name)
