"""MI355X-native tracer for the particle-based modified method of characteristics.

``mmoc``      -- Python binding of the C-ABI (``include/mmoc.h``, ``lib/libmmoc.so``)
``workloads`` -- seeded synthetic inputs (coarse meshes, analytic fields)
``build``     -- hipcc build of the library for gfx950
"""
__all__ = ["mmoc", "workloads", "build"]
