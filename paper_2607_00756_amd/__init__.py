"""BiP-PRISM core-loss STEM-EELS hot path for MI355X (gfx950).

The compute path is the HIP library behind the C ABI declared in
include/bip.h; `paper_2607_00756_amd.bip` is its thin Python binding.
Importing the package itself loads nothing native.
"""
__all__ = ["bip", "specimen"]
