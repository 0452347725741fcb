"""Batched MRI fast-stage solver for MI355X (gfx950).

The package is deliberately light at import time: `inputs` (seeded synthetic
workloads) has no GPU dependency, and `mri` (the ctypes binding of libmri.so)
is loaded only when imported explicitly.
"""
__all__ = ["inputs", "mri"]
