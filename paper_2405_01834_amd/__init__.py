"""libmderi: McMurchie-Davidson 3-/4-centre Coulomb integrals on MI355X.

Python binding over the C ABI of ``libmderi.so`` (``include/mderi.h``).  The
binding only marshals arguments: host inputs are numpy arrays, device
outputs are torch tensors (PyTorch supplies device memory and streams), and
every step of the computation runs in the library's HIP kernels.  There is
no CPU fallback: if the library is missing or no GPU is visible, the calls
raise.
"""
from __future__ import annotations

from .mderi import (  # noqa: F401
    Basis,
    Context,
    MderiError,
    lib_path,
    load_library,
)
