"""Gini multidimensional scaling on AMD MI355X (gfx950).

The package is deliberately light at import time: the native library is only
loaded when :mod:`paper_2605_25124_amd.ginimds` is imported, and the seeded
input generators in :mod:`paper_2605_25124_amd.synth` need nothing but numpy.
"""

__all__ = ["ginimds", "synth"]
