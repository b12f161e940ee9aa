"""CPU oracle (test infrastructure only; never used by the product path).

See ``oracle/oracle.py`` for what each function computes and which passage of
the paper it follows.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import O_INF, Tables  # noqa: F401
