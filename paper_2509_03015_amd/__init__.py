"""MI355X-native solver for SPD block-tridiagonal systems by recursive Schur-complement reduction.

The solver runs in the HIP library ``_lib/libbds.so`` (C ABI in include/bds.h);
``solver`` marshals torch tensors into it.  Importing this package does not load
the library; the first solver call does, and raises if it is not built.
"""


def __getattr__(name):
    if name in ("factor", "solve", "Factor", "BdsError", "PRECISIONS", "factor_batched", "BatchedFactor"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
