"""CPU oracle for the LC covariance hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The
product path (``paper_2205_11852_amd``) never does, and the two share no
code: the oracle's pair counter is plain C compiled by gcc, its estimator,
multipole and covariance assembly is plain numpy in float64.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import build  # noqa: F401
