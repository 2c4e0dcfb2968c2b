"""MI355X-native masked-input FSS evaluation (OblivGM's server hot path).

The product is the HIP library ``liboblivgm_fss.so`` (sources in ``csrc/``,
C ABI in ``include/oblivgm_fss.h``); ``fss`` is its ctypes binding.
"""
__all__ = ["fss", "build"]
