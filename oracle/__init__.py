"""FP64 CPU oracle (test infrastructure only; never used by the device path)."""
from .pinv_oracle import *  # noqa: F401,F403
from .pinv_oracle import Build, NotPositiveDefinite  # noqa: F401
