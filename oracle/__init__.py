"""CPU oracle for EMR-/LMR-RDHEI (arXiv 2302.07992) -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it.
The arithmetic lives in ``rdhei_oracle.c`` (plain C, single-threaded; it also
holds the bi-level map coder of the LMR variant); ``oracle.py`` only builds
the C file with gcc and marshals numpy arrays.  ``metrics.py`` holds the Sec. IV image
metrics in plain numpy (``from oracle import metrics``), ``dynamic_b.py`` the
per-tile choice of b of the dynamic-b variant (``from oracle import dynamic_b``).
"""
from .oracle import *  # noqa: F401,F403
