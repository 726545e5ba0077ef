"""MI355X-native butterfly manifold harmonic transform.

Subpackages
  factor     host FP64 factor construction (trees, column IDs, factor files)
  workloads  seeded synthetic inputs (points, meshes, coefficients)
  runtime    ctypes binding of the C-ABI library libbfmht.so (HIP, gfx950)
"""
