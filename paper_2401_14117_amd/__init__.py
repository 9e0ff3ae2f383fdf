"""MI355X-native Posit(32,2) dense linear algebra.

The compute path is the HIP library ``libposit32.so`` (sources under
``csrc/``, C ABI in ``include/posit32.h``); :mod:`paper_2401_14117_amd.posit32`
is a thin ctypes binding over it that takes torch device tensors.
"""
__version__ = "0.1.0"
