"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps the plain C library built
from ``cns_oracle.c`` and, for gradients, a plain PyTorch CPU restatement of
the same discrete operator (``adjoint_ref``).  It shares no code with the HIP
library.
"""
from .oracle import *  # noqa: F401,F403
