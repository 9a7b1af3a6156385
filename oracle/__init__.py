"""CPU oracle (test infrastructure): plain float64 numpy implementation of
the realfast search hot path.  Only tests, the smoke check and the
benchmark's CPU-baseline leg may import this package."""
from .rf_oracle import *  # noqa: F401,F403
from .rf_oracle import Plan  # noqa: F401
