"""MI355X-native CSPH-TVD shallow-water + Exner step (Khrapov & Khoperskov 2020).

The solver is the C-ABI library ``libcsph.so`` (hand-written HIP for gfx950);
``paper_2103_15196_amd.csph`` is its thin ctypes binding and
``paper_2103_15196_amd.workloads`` draws the seeded synthetic inputs.
Submodules are imported on demand so that input generation does not load
the GPU library.
"""
__all__ = ["csph", "workloads"]
