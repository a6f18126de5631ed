"""MI355X-native binary Shan-Chen capillary-filling library (HIP for gfx950).

``inputs``  seeded synthetic fields and parameter sets (no model arithmetic)
``_lib``    ctypes binding of libscf.so, one function per C ABI entry point (include/scf.h)
``scf``     Channel and Batch: PyTorch device workspace and stream, calls through the C ABI
``build``   in-tree hipcc build of libscf.so
"""
__all__ = ["inputs"]
