"""FP64 CPU oracle for hierarchical homogenization (arXiv 2208.02320).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only ``tests/``, the smoke check
in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.  It
shares no code with the GPU implementation.

It is a plain, slow, obviously correct NumPy/SciPy implementation of what the
paper computes:

* ``galerkin``  -- the periodic Fourier-Galerkin elasticity solve of
  Appendix A (projection operator, FFT convolution, conjugate gradients), the
  isotropic/anisotropic constitutive laws of Sec. 4, and the averaged
  stiffness C = Sigma E^-1 of Sec. 4 (eq. for C^homo_R).
* ``brute``     -- a dense solve of the same discrete problem from explicit
  DFT derivative matrices (tiny grids only).
* ``hier``      -- partition, padding, intermediate image and second-level
  solve of Sec. 3/4, bulk/shear moduli and the n^-1 fit of Sec. 5.
* ``bounds``    -- Voigt/Reuss/Hashin-Shtrikman bounds and the laminate and
  uniform-shear closed forms used as pins.
"""
