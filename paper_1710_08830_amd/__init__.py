"""MI355X-native truncated-unity fRG flow right-hand side (arXiv:1710.08830).

The compute path is the HIP library ``libtufrg.so`` (C ABI in include/tufrg.h);
``paper_1710_08830_amd.tufrg`` is its ctypes binding.  Importing the binding
raises if the library has not been built.
"""

LIB_NAME = "libtufrg.so"
