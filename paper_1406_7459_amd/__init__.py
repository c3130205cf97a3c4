"""MI355X-native FFT-demagnetisation + LLG hot path (arXiv:1406.7459).

The compute lives in ``libmm.so`` (hand-written HIP for gfx950, C ABI in
``include/mm.h``); ``paper_1406_7459_amd.mm`` is the ctypes binding and
``paper_1406_7459_amd.workloads`` the seeded input generators.  Importing the
package loads nothing: the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["mm", "workloads"]
