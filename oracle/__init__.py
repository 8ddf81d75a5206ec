"""FP64 CPU oracle for the finite discrete shearlet transform (FFST).

TEST INFRASTRUCTURE ONLY. This package is the slow, plainly written reference
that the HIP path is checked against. Only the test-suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import or
call it; the product package (``paper_1202_1773_amd``) never does, and the two
share no code.

Everything here is float64 NumPy, written from the paper's definitions:

* ``windows``   -- the one-dimensional functions v, b, psi1-hat, psi2-hat and the
                   scaling function (Sec. 2.1, Sec. 2.4).
* ``grid``      -- number of scales, the frequency grid Xi and its spacing Delta
                   (Sec. 3.1, Sec. 3.5.1).
* ``spectra``   -- the index order (Sec. 3.5.2), every shearlet spectrum on the
                   grid, including the glued seam elements (Sec. 3.1), and the
                   Nyquist-line symmetrisation for real coefficients (Sec. 3.8.1).
* ``dft``       -- a direct DFT and a textbook mixed-radix FFT.
* ``transform`` -- forward transform, eq. (shearletTransform); adjoint/inverse,
                   eq. (inverseShearletTransform) (Sec. 3.1, Sec. 3.3).
* ``smooth``    -- the smooth-shearlet variant of Sec. 3.4, eq. (newPsi1).

Each module states in its header what pins it (the tests that check it against
values and identities fixed by the paper or by plain mathematics).
"""

from . import windows, grid, spectra, dft, transform  # noqa: F401
