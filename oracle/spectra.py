"""Shearlet spectra on the discrete grid and their index order.

Test infrastructure only (see the package header).

* Index order i (Sec. 3.5.2): i = 0 is the low-pass; scale j then contributes
  2^(j+2) spectra, visited counter-clockwise: horizontal cone k = 0, -1, ...,
  -2^j + 1; the glued seam element k = -2^j; the vertical cone
  k = -2^j + 1, ..., 2^j - 1; the seam element k = 2^j; the horizontal cone
  k = 2^j - 1, ..., 1. In total eta = 2^(J+2) - 3 spectra.
* Horizontal cone, |k| < 2^j (eq. horizontalShearlet, eq. discreteHorizontalTrans):
  psi1(4^-j w1) psi2(2^j w2 / w1 + k) where |w2| < |w1|.
* Vertical cone (eq. verticalShearlet, eq. discreteVerticalTrans):
  psi1(4^-j w2) psi2(2^j w1 / w2 + k) where |w1| < |w2|.
* Seam element |k| = 2^j (Sec. 3.1, eq. discreteSeamTrans): the sum of the
  horizontal part, the vertical part and the part on the seam line
  |w1| = |w2|; the seam-line part uses the horizontal formula.
* Low-pass (eq. phi): varphi(w1) where |w2| <= |w1|, varphi(w2) elsewhere.
* Real coefficients (Sec. 3.8.1): on a Nyquist line of an even-length axis
  each spectrum value and its mirror partner are both replaced by the root
  mean square of the two. This keeps every spectrum even on the grid and
  keeps the sum of squares; on the paper's toy row it reproduces the
  mirrored, 1/sqrt(2)-scaled row.

Pinned by tests/test_oracle_spectra.py: the counts of Sec. 3.5.2, the
Parseval identity sum_i Psi_i^2 = 1 at every grid point (Theorem in Sec. 3.2,
Sec. 3.6), points on the ray of a given slope where exactly one spectrum
equals 1 (fixing the index order and the sign of k), point symmetry,
transposition and mirror symmetries, and the toy row of Sec. 3.8.1
(tests/golden/realreal_toy.txt).
"""

import numpy as np

from .grid import default_scales, frequencies
from .windows import psi1, psi2, varphi


def num_spectra(J):
    """eta = 2^(J+2) - 3 (Sec. 3.5.2)."""
    return 2 ** (J + 2) - 3


def index_table(J):
    """(kind, j, k) for every index i in the order of Sec. 3.5.2.

    kind is 'lowpass', 'h', 'v' or 'hv' (glued seam element); the low-pass
    entry carries j = -1, k = 0."""
    table = [("lowpass", -1, 0)]
    for j in range(J):
        P = 2 ** j
        table.append(("h", j, 0))
        table += [("h", j, k) for k in range(-1, -P, -1)]
        table.append(("hv", j, -P))
        table += [("v", j, k) for k in range(-P + 1, P)]
        table.append(("hv", j, P))
        table += [("h", j, k) for k in range(P - 1, 0, -1)]
    return table


def _ratio(num, den):
    """num / den where den != 0, zero elsewhere (only read inside a cone
    where den is nonzero)."""
    out = np.zeros_like(num)
    np.divide(num, den, out=out, where=den != 0)
    return out


def horizontal_formula(j, k, w1, w2, aux=3):
    """psi1(4^-j w1) psi2(2^j w2 / w1 + k), the dilated and sheared shearlet of
    Sec. 3.1 (without the cone cut-off)."""
    return psi1(w1 / 4.0 ** j, aux) * psi2(2.0 ** j * _ratio(w2, w1) + k, aux)


def vertical_formula(j, k, w1, w2, aux=3):
    """Same with the roles of w1 and w2 interchanged (eq. verticalShearlet)."""
    return psi1(w2 / 4.0 ** j, aux) * psi2(2.0 ** j * _ratio(w1, w2) + k, aux)


def spectrum(kind, j, k, w1, w2, aux=3):
    """One spectrum Psi_i on the grid (w1, w2), before the Nyquist fix."""
    a1, a2 = np.abs(w1), np.abs(w2)
    if kind == "lowpass":
        return np.where(a2 <= a1, varphi(w1, aux), varphi(w2, aux))
    if kind == "h":
        return np.where(a2 < a1, horizontal_formula(j, k, w1, w2, aux), 0.0)
    if kind == "v":
        return np.where(a1 < a2, vertical_formula(j, k, w1, w2, aux), 0.0)
    if kind == "hv":
        horiz_and_seam_line = (a2 <= a1) & (a1 > 0)
        out = np.where(horiz_and_seam_line, horizontal_formula(j, k, w1, w2, aux), 0.0)
        return np.where(a1 < a2, vertical_formula(j, k, w1, w2, aux), out)
    raise ValueError(kind)


def symmetrize_nyquist(psi):
    """Real-coefficient fix of Sec. 3.8.1 on a (..., M, N) stack.

    Column N/2 (N even): the value at row r and the one at row (-r) mod M are
    both replaced by sqrt((a^2 + b^2) / 2). Row M/2 (M even): the same with
    columns c and (-c) mod N. Points that are their own partner are kept."""
    psi = np.asarray(psi, dtype=np.float64)
    M, N = psi.shape[-2], psi.shape[-1]
    out = psi.copy()
    if N % 2 == 0:
        c = N // 2
        partner = (-np.arange(M)) % M
        a = psi[..., :, c]
        b = psi[..., partner, c]
        out[..., :, c] = np.sqrt((a * a + b * b) / 2.0)
    if M % 2 == 0:
        r = M // 2
        partner = (-np.arange(N)) % N
        a = psi[..., r, :]
        b = psi[..., r, partner]
        out[..., r, :] = np.sqrt((a * a + b * b) / 2.0)
    return out


def symmetrize_line(line):
    """The same rule on one line of length L with partner (-p) mod L; used to
    replay the toy row of Sec. 3.8.1."""
    line = np.asarray(line, dtype=np.float64)
    partner = (-np.arange(line.shape[-1])) % line.shape[-1]
    return np.sqrt((line * line + line[..., partner] ** 2) / 2.0)


def spectrum_plane(M, N, J, i, max_scale="max", real_real=True, shearlet="meyer", aux=3):
    """Plane i of the spectra stack, float64 (M, N), natural DFT order; `aux`
    selects the auxiliary function v (see oracle.windows)."""
    w1, w2 = frequencies(M, N, J, max_scale)
    kind, j, k = index_table(J)[i]
    if shearlet == "meyer":
        plane = spectrum(kind, j, k, w1, w2, aux)
    elif shearlet == "smooth":
        from .smooth import smooth_spectrum
        plane = smooth_spectrum(kind, j, k, w1, w2, aux)
    else:
        raise ValueError(shearlet)
    return symmetrize_nyquist(plane) if real_real else plane


def spectra(M, N, J=None, max_scale="max", real_real=True, shearlet="meyer", aux=3):
    """All eta spectra as a float64 (eta, M, N) stack."""
    if J is None:
        J = default_scales(M, N)
    if J < 1:
        raise ValueError("need at least one scale")
    return np.stack([
        spectrum_plane(M, N, J, i, max_scale, real_real, shearlet, aux)
        for i in range(num_spectra(J))
    ])
