"""MI355X-native dynamic cutoff method (DCM) hot path.

The HIP kernels live in ``csrc/`` and are built into ``libdcm.so``; ``dcm`` is the thin
ctypes binding over its C-ABI (``include/dcm.h``). Importing this package loads nothing:
``paper_1502_03234_amd.dcm`` loads the library and raises if it is missing.
"""
