"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never links or calls it.
"""
from .oracle import (Oracle, OracleParams, build_oracle, lib_path, num_threads,  # noqa: F401
                     set_threads, KIND_BITS)
