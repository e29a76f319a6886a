"""HashGraph (arXiv:1907.02900) hot path on AMD Instinct MI355X (gfx950).

The compute lives in ``libhashgraph.so`` (hand-written HIP kernels behind a C
ABI, declared in ``include/hashgraph.h``).  ``paper_1907_02900_amd.hg`` is the
thin ctypes binding; ``paper_1907_02900_amd.workloads`` holds the seeded input
generators.  Importing this package does not load the GPU library, so the
generators stay usable on machines without a GPU.
"""
__all__ = ["hg", "workloads"]
