"""MI355X-native ConnectIt: static and batch-incremental graph connectivity.

The device path is the HIP library ``libconnectit_hip.so`` behind the C ABI
in ``include/connectit_hip.h``; ``paper_2008_03909_amd.binding`` is its thin
Python binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
__all__ = ["binding", "inputs"]
