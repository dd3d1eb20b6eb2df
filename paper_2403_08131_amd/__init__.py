"""MI355X-native Gaussian-process surrogate fit and expected-improvement scoring.

``gpbo`` is the binding of the HIP library (``libgpbo.so``, C ABI in
``include/gpbo.h``); ``inputs`` generates the seeded synthetic workloads.
Nothing is loaded at import time.
"""
__all__ = ["gpbo", "inputs", "build"]
