"""MI355X-native raycast-and-policy hot path (Riemannian Motion Policies over voxel maps).

Submodules:
  workloads -- seeded synthetic inputs (maps, states, scans); no method arithmetic
  binding   -- ctypes binding of the C-ABI library ``librmpcast.so`` (HIP kernels for gfx950)
  build     -- compiles the library with hipcc
"""
__all__ = ["workloads", "binding", "build"]
