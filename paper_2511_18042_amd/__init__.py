"""MI355X-native hybrid LAD-GBR right-hand side (arxiv 2511.18042).

The compute path is the C-ABI library ``liblgbr.so`` built from ``csrc/`` (HIP for
gfx950); ``lgbr`` is its ctypes binding.  ``cases`` holds the seeded synthetic
inputs.  Importing the package loads nothing; ``lgbr.load()`` opens the library
and raises if it is missing.
"""
