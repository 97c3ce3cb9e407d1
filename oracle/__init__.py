"""CPU oracle (test infrastructure only; see rbf_oracle.py, schwarz.py and mlp.py)."""
from .rbf_oracle import *  # noqa: F401,F403
from . import mlp, schwarz  # noqa: F401
