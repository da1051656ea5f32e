"""FP64 CPU oracle (test infrastructure only; see sr_oracle)."""
from .sr_oracle import *  # noqa: F401,F403
