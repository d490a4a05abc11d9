"""relpic: MI355X-native electromagnetic PIC step for relativistic beams.

Implements the PIC cycle analysed by Xu et al. (deposit, Yee or customized
finite-difference Maxwell advance, gather, relativistic Boris push) as HIP
kernels for gfx950 behind the C ABI in include/relpic.h.

  relpic   ctypes binding of librelpic.so (same names as the C ABI) and the
           `Sim` convenience wrapper
  inputs   seeded synthetic workloads (beams, plasma, single particles)
  build    compiles librelpic.so in-tree with hipcc
"""
