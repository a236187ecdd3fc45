"""High-precision CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library under
``paper_1302_7203_amd/`` never does.
"""
from .oracle import (  # noqa: F401
    build,
    arrow_eig,
    dpr1_eig,
    arrow_svd,
    herm_eig,
    tridiag_eig,
)
