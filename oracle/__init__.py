"""FP64 CPU oracle (test infrastructure only; never called by the product path)."""
from .fock_oracle import *  # noqa: F401,F403
from . import fock_oracle  # noqa: F401
