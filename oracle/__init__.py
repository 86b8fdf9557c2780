"""FP64 CPU oracle for NS-RGS.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  See ``nsrgs.py``
for the method and ``quantize.py`` for the storage formats of A.
"""
from . import nsrgs, quantize  # noqa: F401
