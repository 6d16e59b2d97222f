"""MI355X-native blip orbital evaluation (periodic cubic B-spline orbitals).

The evaluation runs in hand-written HIP kernels for gfx950 behind the C ABI
of ``libblip.so`` (see include/blip.h); :mod:`paper_1204_1121_amd.blip` is
its thin Python binding and :mod:`paper_1204_1121_amd.workloads` holds the
seeded synthetic inputs.
"""

__all__ = ["blip", "workloads", "build"]
