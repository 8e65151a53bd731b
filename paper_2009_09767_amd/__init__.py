"""MI355X-native rank-safe column-block sparse SVD (Ranky, arXiv 2009.09767).

The compute path lives in the HIP library ``libranky.so`` (built from ``csrc/``)
behind the C-ABI declared in ``include/ranky.h``; ``ranky`` is its Python binding.
``gen`` draws the seeded synthetic inputs.  Importing this package loads nothing
native: the binding loads the library on first use and raises if it is missing.
"""
__all__ = ["gen", "ranky"]
