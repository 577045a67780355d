"""MI355X-native Bahmani (2+2eps) densest-subgraph peeling.

The peeling passes run as hand-written HIP kernels for gfx950 in
``libdsg.so`` behind the C ABI declared in ``include/dsg.h``.  This package
is the thin Python binding over that ABI (argument marshalling only) plus the
seeded input generators in :mod:`paper_2103_00154_amd.inputs`.

The binding is imported lazily so that ``inputs`` can be used without
loading the HIP library.
"""
from __future__ import annotations

__all__ = ["peel", "PeelResult", "DsgError", "workspace_bytes", "lib"]


def __getattr__(name):
    if name in __all__:
        from . import dsg as _dsg
        return getattr(_dsg, name)
    raise AttributeError(name)
