"""MI355X-native hot path of a 1D3V electrostatic PIC-MCC time step.

libpic.so (HIP, gfx950) holds every step of the method; ``pic`` is its
ctypes binding.  See include/pic.h for the C ABI.
"""
from . import pic  # noqa: F401
from .pic import PicSim, PicError  # noqa: F401

__all__ = ["pic", "PicSim", "PicError"]
