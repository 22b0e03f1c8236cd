"""Sort-Based Matching for Data Distribution Management on MI355X (gfx950).

The matching itself runs in ``libddm.so`` (hand-written HIP kernels behind a
C ABI declared in ``include/ddm.h``); ``paper_1703_06680_amd.ddm`` is the thin
Python binding.  Importing this package does not load the library, so the
input generators in ``workloads`` can be used without a GPU.
"""

__all__ = ["ddm", "workloads"]
