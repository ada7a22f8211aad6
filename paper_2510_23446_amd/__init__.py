"""Tree-cotree-gauged dual-primal (IETI-DP) eddy-current time stepping on MI355X.

The solver lives in the HIP library ``libtcf.so`` (C-ABI declared in
``include/tcf.h``); ``paper_2510_23446_amd.tcf`` is its ctypes binding.
Importing the package does not load the library; ``tcf.lib()`` does, and
raises if it has not been built (``paper_2510_23446_amd.build.build()``).
"""
