"""MI355X-native encoded-shot FWI gradient (forward solve, adjoint-state gradient over
+-1-encoded supergathers batched over posterior samples, Langevin update).

The numerical work runs in the gfx950 HIP library ``libfwi_mi355.so`` (C ABI in
include/fwi.h); ``fwi`` is its thin Python binding.
"""
__all__ = ["fwi", "problems"]
