"""MI355X-native Eager K-truss (fine-grained per-edge supports + prune-to-fixpoint).

The compute path is the HIP library libktruss.so (C-ABI in include/ktruss.h);
`paper_2009_07929_amd.ktruss` is its thin ctypes binding.
"""
from . import ktruss  # noqa: F401
from .ktruss import (  # noqa: F401
    Graph, KtrussError, ktruss_build_csr, ktruss_prune, ktruss_run, ktruss_set_schedule,
    ktruss_support, ktruss_validate, ktruss_workspace_bytes,
)
