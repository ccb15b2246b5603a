"""FP64 CPU oracle (test infrastructure only; see msl_oracle)."""
from .msl_oracle import *  # noqa: F401,F403
