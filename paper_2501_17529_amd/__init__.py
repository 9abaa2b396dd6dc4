"""MI355X-native batched DC loadflow screen over grid-topology candidates.

The solver lives in libdcflow.so (HIP, gfx950); ``dcflow`` is its thin
Python binding.  Build the library with ``python -m paper_2501_17529_amd.build_lib``.
"""
