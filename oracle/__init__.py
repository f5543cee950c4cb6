"""FP64 CPU oracle (test infrastructure only; see qst_oracle's header)."""
from .qst_oracle import *  # noqa: F401,F403
from . import qst_oracle  # noqa: F401
