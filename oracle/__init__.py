"""FP64 CPU oracle (test infrastructure only; see core.py)."""
from .core import *  # noqa: F401,F403
