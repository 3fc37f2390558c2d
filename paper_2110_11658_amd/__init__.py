"""GPU Barnes-Hut distant (regular) forces and neighbour lists for the P3T
scheme of Arnold, Baumgardt & Wang (2021), on AMD Instinct MI355X (gfx950).

The work runs in libpbh (HIP kernels behind the C ABI of include/pbh.h); this
package binds it for torch tensors on the GPU. Importing the package is cheap:
the library is loaded on first use, and ``ic`` (seeded initial conditions)
needs no GPU.
"""
from __future__ import annotations

__all__ = ["Pbh", "ic"]


def __getattr__(name):
    if name == "Pbh":
        from .api import Pbh
        return Pbh
    raise AttributeError(name)
