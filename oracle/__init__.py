"""CPU oracle for QPE probabilities (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package. The product path never imports it.
"""
from .qpe_oracle import *  # noqa: F401,F403
from .qpe_oracle import __all__  # noqa: F401
