"""MI355X (gfx950) solver for electron-hole pair production in graphene by
split-operator propagation of the massless 2D Dirac equation in momentum
space (Fillion-Gourdeau et al., arXiv:1607.03062).

The compute path is libpd.so (HIP kernels behind the C ABI of include/pd.h);
this package only marshals arguments to it.  Importing the package does not
load the library; the first solver does, and fails loudly if it is not built.
"""
from ._lib import (  # noqa: F401
    LIB_PATH,
    PDError,
    Batch,
    Solver,
    load,
    set_fault,
)


def require_native():
    """Load libpd.so or raise: the package has no CPU fallback."""
    return load()


def version() -> str:
    return load().pd_version().decode()
