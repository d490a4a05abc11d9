"""FP64 CPU oracle for the relativistic-beam PIC step (TEST INFRASTRUCTURE ONLY).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import, call, link or execute anything in this directory.  It shares
no code with the GPU path; the two meet only through the seeded input
generators, which hold none of the method's arithmetic.

Contents
  pic_oracle.c / pic.py  plain FP64 PIC step (deposit, field advance, gather,
                         Boris push, J1 correction, moving window)
  fit.py                 App. C constrained least-squares fit of the axial
                         stencil coefficients, and the operator symbols
  kspace.py              the paper's k-space integral for E1 around a
                         streaming particle (Eq. 13 with Plemelj k2 integrals,
                         App. D) and the self-force (Eqs. 19, 25)
  steady.py              exact steady-state lattice fields of charges
                         streaming along x1 on a periodic 2D grid (the
                         Sec. 2.1 response in terms of the density, every
                         wavenumber and aliased frequency on the lattice)
  beam_init.py           self-consistent initial fields of charges streaming
                         along x1 (Sec. 2.1, ultra-relativistic limit)
  dispersion.py          closed-form vacuum dispersion of the discrete
                         Maxwell operators (Eq. 4)
  field_loss.py          field loss around a moving bunch on the oracle's
                         fields and its central-difference gradient in the
                         axial coefficients
"""
