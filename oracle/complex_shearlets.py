"""Complex shearlets from one-sided spectra (Sec. 3.8.2).

Test infrastructure only (see the package header).

Sec. 3.8.2 obtains complex shearlets (and complex coefficients) by keeping
one side of each shearlet's spectrum, and states that the computations and
frame properties stay the same. Reading used here (the paper gives no
formula):

* Shearlet i >= 1 has the orientation vector d_i = (1, -k / 2^j) for the
  horizontal cone and the seam elements, and (-k / 2^j, 1) for the vertical
  cone (the centre ray of its wedge, Sec. 3.1). Its two spectral lobes lie on
  either side of the line <w, d_i> = 0.
* One-sided spectrum on the grid: Psi+_i(w) = sqrt(2) Psi_i(w) where
  <w, d_i> > 0, 0 where <w, d_i> < 0. A grid point and its DFT mirror
  (-r mod M, -c mod N) on a Nyquist line can fall on the same side (the
  mirror of -X is -X again); for such pairs, and on the line <w, d_i> = 0,
  Psi+_i = Psi_i. The low-pass has no orientation and stays Psi+_0 = Psi_0.
* Coefficients c+_i = ifft2(Psi+_i * fft2(f)) (complex).

For real f this is a Parseval frame: sum_i |Psi+_i(w)|^2 + |Psi+_i(-w)|^2 =
sum_i Psi_i(w)^2 + Psi_i(-w)^2 = 2 at every grid pair, so
sum_i ||c+_i||^2 = ||f||^2, and f = Re( sum_i ifft2(Psi+_i * fft2(c+_i)) ).

Pinned by tests/test_oracle_complex.py: Parseval and reconstruction on real
images, one-sidedness of every coefficient's spectrum, plane waves (a real
cosine in the positive half of shearlet i gives the analytic signal
Psi_i / sqrt(2) * exp(i theta), of constant modulus), and the relation of the
real part to the real transform away from the Nyquist lines.
"""

import numpy as np

from .dft import dft2, idft2
from .grid import frequencies
from .spectra import index_table, spectrum_plane


def orientation(kind, j, k):
    """Centre direction d of a shearlet's wedge (None for the low-pass)."""
    if kind == "lowpass":
        return None
    t = -k / 2.0 ** j
    return (t, 1.0) if kind == "v" else (1.0, t)


def one_sided_plane(M, N, J, i, max_scale="max", shearlet="meyer", aux=3):
    """Psi+_i on the (M, N) grid, float64, natural DFT order."""
    psi = spectrum_plane(M, N, J, i, max_scale, True, shearlet, aux)
    kind, j, k = index_table(J)[i]
    d = orientation(kind, j, k)
    if d is None:
        return psi
    w1, w2 = frequencies(M, N, J, max_scale)
    side = np.sign(w1 * d[0] + w2 * d[1])
    mirror = side[(-np.arange(M)) % M][:, (-np.arange(N)) % N]
    split = (side != 0) & (side == -mirror)
    return np.where(split, np.where(side > 0, np.sqrt(2.0) * psi, 0.0), psi)


def one_sided_spectra(M, N, J, max_scale="max", shearlet="meyer", aux=3):
    eta = len(index_table(J))
    return np.stack([one_sided_plane(M, N, J, i, max_scale, shearlet, aux) for i in range(eta)])


def forward(f, psi_plus):
    """c+_i = ifft2(Psi+_i * fft2(f)), complex (eta, M, N)."""
    F = dft2(np.asarray(f, dtype=np.float64))
    return np.stack([idft2(p * F) for p in psi_plus])


def adjoint_real(c, psi_plus):
    """Re( sum_i ifft2(Psi+_i * fft2(c_i)) ): the adjoint for real images."""
    acc = sum(np.conj(p) * dft2(ci) for p, ci in zip(psi_plus, c))
    return idft2(acc).real
