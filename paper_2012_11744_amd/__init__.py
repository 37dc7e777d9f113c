"""MI355X (gfx950) pressure projection for one-fluid multiphase flow.

The hot path lives in the HIP library libpp.so (C ABI: include/pp.h);
`solver` is its Python binding (import it explicitly: it needs torch and the
built library) and `workloads` holds the seeded synthetic inputs.
"""
from . import workloads  # noqa: F401  (pure numpy, no GPU needed)

__all__ = ["workloads"]
