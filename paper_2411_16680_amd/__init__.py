"""MI355X-native Update & Fuse + LDM composite (Quark, TOG 2024) on gfx950.

The compute path lives in the HIP library ``libquark.so`` behind the C-ABI
declared in ``include/quark.h``; ``paper_2411_16680_amd.lib`` is the thin
Python binding.  Importing this package loads nothing: the library is loaded
on first use, and every entry point fails loudly if it is missing.
"""

__version__ = "0.1.0"
