"""FP64 CPU oracle (test infrastructure only; see rid_oracle.py)."""
from .rid_oracle import *  # noqa: F401,F403
from . import rid_oracle  # noqa: F401
