"""FP64 CPU oracle (test infrastructure only; see ``tbs_oracle``)."""
from .tbs_oracle import *  # noqa: F401,F403
from . import tbs_oracle  # noqa: F401
