"""CPU oracle (test infrastructure only; see rbf_oracle.py)."""
from .rbf_oracle import *  # noqa: F401,F403
