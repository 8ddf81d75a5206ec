"""One-dimensional window functions of the Meyer-type shearlet (Sec. 2.1, 2.4).

Test infrastructure only (see the package header).

Pinned by tests/test_oracle_windows.py: special values stated in the paper
(b(+-2) = 1, support of b and psi1-hat, psi2-hat(+-1) = 0), the symmetry
v(x) + v(1 - x) = 1 (Lemma in Sec. 2.1), v'(x) = -140 x^3 (x - 1)^3
(Remark on the construction of v), the closed form of psi1-hat printed in
Sec. 3.4, and the partitions of unity of Lemma (propertySumbj),
Theorem (PropertyPsi1), Theorem (PropertyPsi2) and eq. (overlapPsi1Phi).
"""

import numpy as np

HALF_PI = np.pi / 2.0


def v(x):
    """Auxiliary function v, eq. (v): 0 for x < 0, 1 for x > 1 and the
    degree-7 polynomial 35x^4 - 84x^5 + 70x^6 - 20x^7 on [0, 1]."""
    x = np.asarray(x, dtype=np.float64)
    t = np.clip(x, 0.0, 1.0)
    poly = 35.0 * t**4 - 84.0 * t**5 + 70.0 * t**6 - 20.0 * t**7
    return np.where(x < 0.0, 0.0, np.where(x > 1.0, 1.0, poly))


def b(w):
    """Function b, eq. (b): sin(pi/2 v(|w| - 1)) on 1 <= |w| <= 2,
    cos(pi/2 v(|w|/2 - 1)) on 2 < |w| <= 4, zero elsewhere."""
    a = np.abs(np.asarray(w, dtype=np.float64))
    rising = np.sin(HALF_PI * v(a - 1.0))
    falling = np.cos(HALF_PI * v(a / 2.0 - 1.0))
    out = np.where((a >= 1.0) & (a <= 2.0), rising, 0.0)
    return np.where((a > 2.0) & (a <= 4.0), falling, out)


def psi1(w):
    """psi1-hat, eq. (Psi1): the square root of b(2w)^2 + b(w)^2."""
    w = np.asarray(w, dtype=np.float64)
    return np.sqrt(b(2.0 * w) ** 2 + b(w) ** 2)


def psi2(w):
    """psi2-hat, eq. (Psi2): sqrt(v(1 + w)) for w <= 0 and sqrt(v(1 - w)) for
    w > 0."""
    w = np.asarray(w, dtype=np.float64)
    return np.where(w <= 0.0, np.sqrt(v(1.0 + w)), np.sqrt(v(1.0 - w)))


def varphi(w):
    """One-dimensional scaling function of Sec. 2.4: 1 for |w| <= 1/2,
    cos(pi/2 v(2|w| - 1)) for 1/2 < |w| < 1, zero otherwise."""
    a = np.abs(np.asarray(w, dtype=np.float64))
    ramp = np.cos(HALF_PI * v(2.0 * a - 1.0))
    out = np.where((a > 0.5) & (a < 1.0), ramp, 0.0)
    return np.where(a <= 0.5, 1.0, out)
