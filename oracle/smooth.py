"""Smooth shearlets of Sec. 3.4 (eq. Phi, eq. newPsi1, eq. smoothPsi).

Test infrastructure only (see the package header).

* Low-pass: the tensor scaling function Phi(w) = varphi(w1) varphi(w2), eq. (Phi).
* Radial part: the corona function Psi1(w) = sqrt(Phi^2(w / 4) - Phi^2(w)),
  eq. (newPsi1), taken at the dilated point 4^-j w (the same dilation
  a_j = 4^-j the discrete shearlets use, Sec. 3.1).
* Directional part, cones and seam gluing: as for the Meyer shearlets,
  "the construction of the horizontal, vertical and diagonal shearlets is the
  same as before" (Sec. 3.4), i.e. psi2(2^j w2/w1 + k) on the horizontal cone,
  psi2(2^j w1/w2 + k) on the vertical cone, both parts summed for |k| = 2^j.

Pinned by tests/test_oracle_smooth.py: Sec. 3.4 states that Phi^2 plus the sum
of the dilated Psi1^2 is one on the grid and that Psi1 lives in the Cartesian
corona [-4, 4]^2 minus [-1/2, 1/2]^2; the frame identity on several grids, the
direction pins and the symmetries of the Meyer case carry over.
"""

import numpy as np

from .windows import psi2, varphi


def tensor_lowpass(w1, w2, aux=3):
    """Phi(w) = varphi(w1) varphi(w2), eq. (Phi)."""
    return varphi(w1, aux) * varphi(w2, aux)


def corona(w1, w2, aux=3):
    """Psi1(w) = sqrt(Phi^2(w / 4) - Phi^2(w)), eq. (newPsi1)."""
    d = tensor_lowpass(w1 / 4.0, w2 / 4.0, aux) ** 2 - tensor_lowpass(w1, w2, aux) ** 2
    return np.sqrt(np.maximum(d, 0.0))


def _ratio(num, den):
    out = np.zeros_like(num)
    np.divide(num, den, out=out, where=den != 0)
    return out


def smooth_spectrum(kind, j, k, w1, w2, aux=3):
    """One smooth spectrum on the grid (before the Nyquist fix)."""
    a1, a2 = np.abs(w1), np.abs(w2)
    if kind == "lowpass":
        return tensor_lowpass(w1, w2, aux)
    radial = corona(w1 / 4.0 ** j, w2 / 4.0 ** j, aux)
    horiz = radial * psi2(2.0 ** j * _ratio(w2, w1) + k, aux)
    vert = radial * psi2(2.0 ** j * _ratio(w1, w2) + k, aux)
    if kind == "h":
        return np.where(a2 < a1, horiz, 0.0)
    if kind == "v":
        return np.where(a1 < a2, vert, 0.0)
    if kind == "hv":
        out = np.where((a2 <= a1) & (a1 > 0), horiz, 0.0)
        return np.where(a1 < a2, vert, out)
    raise ValueError(kind)
