"""MI355X-native butterfly manifold harmonic transform.

Contents
  bfmht      ctypes binding of the C-ABI library libbfmht.so (HIP, gfx950): Plan, Batch
  autograd   torch.autograd functions whose backward is the transposed apply
  autotune   per-stage tile-shape search
  grf        spectral densities for Gaussian random fields
  factor     FP64 factor construction (trees, column IDs on the host or the GPU, factor files)
  sphere     the perturbed-sphere problem (mesh, cotangent Laplacian, eigenpairs)
  workloads  seeded synthetic inputs (points, coefficients, workload sizes)
  build      compiles libbfmht.so from csrc/
"""
