"""Forward, adjoint and inverse finite shearlet transform (Sec. 3.1, 3.3).

Test infrastructure only (see the package header).

* Forward, eq. (shearletTransform): for every index i,
  SH(f)_i = ifft2(Psi_i * fft2(f)). With the Nyquist fix of Sec. 3.8.1 the
  result is real up to rounding; ``forward`` returns the real part and
  ``forward(..., return_complex=True)`` the complex array.
* Adjoint, eq. (inverseShearletTransform): f-hat = sum_i conj(Psi_i) *
  fft2(c_i), then f = ifft2(f-hat). The spectra are real, so conj changes
  nothing; it is written out because that is the adjoint of the forward.
* Inverse: the same computation, since the shearlets form a Parseval frame
  (Theorem in Sec. 3.2) and the inverse is the adjoint (Sec. 3.3).

``psi`` is either a float64 (eta, M, N) stack or a callable i -> (M, N)
plane, so that large grids can be streamed one plane at a time.

Pinned by tests/test_oracle_transform.py: reconstruction and energy
(Parseval frame), the adjoint dot-product identity, a brute-force frame
matrix U with U^T U = I on an 8x8 grid (eq. shearlet_transform_as_matrix),
plane waves (each coefficient plane is the wave times one spectrum value),
constant images, circular-shift equivariance and realness of the
coefficients with and without the Nyquist fix.
"""

import numpy as np

from .dft import dft2, idft2


def _count(psi):
    return psi.shape[0] if not callable(psi) else None


def _plane(psi, i):
    return psi(i) if callable(psi) else psi[i]


def forward(f, psi, planes=None, return_complex=False, eta=None):
    """Coefficients c[..., n, :, :] = ifft2(Psi_{planes[n]} * fft2(f))."""
    f = np.asarray(f, dtype=np.float64)
    M, N = f.shape[-2:]
    if planes is None:
        count = _count(psi) if eta is None else eta
        planes = range(count)
    planes = list(planes)
    F = dft2(f)
    dtype = np.complex128 if return_complex else np.float64
    c = np.empty(f.shape[:-2] + (len(planes), M, N), dtype=dtype)
    for n, i in enumerate(planes):
        plane = idft2(_plane(psi, i) * F)
        c[..., n, :, :] = plane if return_complex else plane.real
    return c


def adjoint(c, psi, return_complex=False):
    """f = ifft2(sum_i conj(Psi_i) * fft2(c_i)) over all eta planes of c."""
    c = np.asarray(c)
    eta = c.shape[-3]
    acc = None
    for i in range(eta):
        term = np.conj(_plane(psi, i)) * dft2(c[..., i, :, :])
        acc = term if acc is None else acc + term
    f = idft2(acc)
    return f if return_complex else f.real


def inverse(c, psi, return_complex=False):
    """Inverse transform; equal to the adjoint for this Parseval frame."""
    return adjoint(c, psi, return_complex)
