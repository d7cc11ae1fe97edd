"""Float64 CPU oracle for guided linear upsampling: test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this package.  The product (the HIP library and its Python binding)
never imports it.
"""
from .glu_oracle import *  # noqa: F401,F403
from .glu_oracle import SearchResult, Decision  # noqa: F401
