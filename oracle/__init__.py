"""CPU oracle (test infrastructure only; see rbf_oracle.py and schwarz.py)."""
from .rbf_oracle import *  # noqa: F401,F403
from . import schwarz  # noqa: F401
