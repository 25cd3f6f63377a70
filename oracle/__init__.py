"""CPU FP64 oracle (test infrastructure only; see etc_oracle's header)."""
from .etc_oracle import *  # noqa: F401,F403
