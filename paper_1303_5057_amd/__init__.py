"""MI355X-native Kerr photon-geodesic integrator (GRay scheme, arXiv:1303.5057).

The hot path lives in libgray.so (HIP kernels for gfx950 behind the C ABI of
include/gray.h). ``paper_1303_5057_amd.gray`` is its Python binding,
``paper_1303_5057_amd.workloads`` holds the seeded synthetic workloads, and
``paper_1303_5057_amd.build`` compiles the library in-tree.
"""
__all__ = ["gray", "workloads", "build"]
