"""MI355X-native matrix permanents (Gray-code Ryser / Nijenhuis-Wilf sweep).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``libperm_mi355x.so``); ``paper_2502_16577_amd.api`` is the thin
Python binding over it.  Importing this package loads nothing native; the
library is loaded on first use and its absence is an error.
"""

__all__ = ["api", "workloads"]
__version__ = "0.1.0"
