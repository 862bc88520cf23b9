"""MI355X-native two-level deflation Helmholtz solver (arXiv 2308.06152).

The solver lives in the HIP library ``libhelmdefl.so`` behind a C-ABI
(``include/helmdefl.h``); ``paper_2308_06152_amd.helmdefl`` is its thin ctypes
binding.  ``paper_2308_06152_amd.inputs`` builds seeded synthetic inputs.
The binding is imported lazily so that the input module can be used without a
built library.
"""

__all__ = ["inputs", "helmdefl"]
