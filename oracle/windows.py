"""One-dimensional window functions of the Meyer-type shearlet (Sec. 2.1, 2.4).

Test infrastructure only (see the package header).

Pinned by tests/test_oracle_windows.py: special values stated in the paper
(b(+-2) = 1, support of b and psi1-hat, psi2-hat(+-1) = 0), the symmetry
v(x) + v(1 - x) = 1 (Lemma in Sec. 2.1), v'(x) = -140 x^3 (x - 1)^3
(Remark on the construction of v), the closed form of psi1-hat printed in
Sec. 3.4, and the partitions of unity of Lemma (propertySumbj),
Theorem (PropertyPsi1), Theorem (PropertyPsi2) and eq. (overlapPsi1Phi).

Other auxiliary functions (Remark on the construction of v): `aux` = k >= 1
selects the v with v'(x) = c x^k (x - 1)^k and v(1) = 1 (shearlets in C^k;
k = 3 is eq. (v)); `aux` = "inf" selects v(x) = s(x-1) / (s(x-1) + s(x)) with
s(x) = exp(-(1/(1+x)^2 + 1/(1-x)^2)) (C-infinity). Every window below takes
the same `aux`. Pinned by tests/test_oracle_aux.py.
"""

from math import comb

import numpy as np

HALF_PI = np.pi / 2.0


def _v_poly(t, k):
    """The integral of c t^k (t - 1)^k from 0 to t, with c such that the
    value at t = 1 is 1. That is the regularised incomplete Beta function
    I_t(k+1, k+1), evaluated as the binomial tail
    sum_{m=k+1}^{2k+1} C(2k+1, m) t^m (1-t)^(2k+1-m), whose terms are all
    nonnegative (no cancellation)."""
    n = 2 * k + 1
    return sum(comb(n, m) * t**m * (1.0 - t) ** (n - m) for m in range(k + 1, n + 1))


def _v_inf(t):
    """s(t - 1) / (s(t - 1) + s(t)) with s(x) = exp(-(1/(1+x)^2 + 1/(1-x)^2)),
    for 0 <= t <= 1 (s vanishes at +-1)."""
    def s(x):
        with np.errstate(divide="ignore"):
            e = 1.0 / (1.0 + x) ** 2 + 1.0 / (1.0 - x) ** 2
        return np.exp(-e)
    a, b_ = s(t - 1.0), s(t)
    return a / (a + b_)


def v(x, aux=3):
    """Auxiliary function v: 0 for x < 0, 1 for x > 1, and on [0, 1] the
    degree-7 polynomial 35x^4 - 84x^5 + 70x^6 - 20x^7 of eq. (v) (aux = 3),
    the C^k polynomial (aux = k) or the C-infinity function (aux = "inf")."""
    x = np.asarray(x, dtype=np.float64)
    t = np.clip(x, 0.0, 1.0)
    if aux == 3:
        mid = 35.0 * t**4 - 84.0 * t**5 + 70.0 * t**6 - 20.0 * t**7
    elif aux == "inf":
        mid = _v_inf(t)
    elif isinstance(aux, int) and aux >= 1:
        mid = _v_poly(t, aux)
    else:
        raise ValueError("aux must be a positive int or 'inf'")
    return np.where(x < 0.0, 0.0, np.where(x > 1.0, 1.0, mid))


def b(w, aux=3):
    """Function b, eq. (b): sin(pi/2 v(|w| - 1)) on 1 <= |w| <= 2,
    cos(pi/2 v(|w|/2 - 1)) on 2 < |w| <= 4, zero elsewhere."""
    a = np.abs(np.asarray(w, dtype=np.float64))
    rising = np.sin(HALF_PI * v(a - 1.0, aux))
    falling = np.cos(HALF_PI * v(a / 2.0 - 1.0, aux))
    out = np.where((a >= 1.0) & (a <= 2.0), rising, 0.0)
    return np.where((a > 2.0) & (a <= 4.0), falling, out)


def psi1(w, aux=3):
    """psi1-hat, eq. (Psi1): the square root of b(2w)^2 + b(w)^2."""
    w = np.asarray(w, dtype=np.float64)
    return np.sqrt(b(2.0 * w, aux) ** 2 + b(w, aux) ** 2)


def psi2(w, aux=3):
    """psi2-hat, eq. (Psi2): sqrt(v(1 + w)) for w <= 0 and sqrt(v(1 - w)) for
    w > 0."""
    w = np.asarray(w, dtype=np.float64)
    return np.where(w <= 0.0, np.sqrt(v(1.0 + w, aux)), np.sqrt(v(1.0 - w, aux)))


def varphi(w, aux=3):
    """One-dimensional scaling function of Sec. 2.4: 1 for |w| <= 1/2,
    cos(pi/2 v(2|w| - 1)) for 1/2 < |w| < 1, zero otherwise."""
    a = np.abs(np.asarray(w, dtype=np.float64))
    ramp = np.cos(HALF_PI * v(2.0 * a - 1.0, aux))
    out = np.where((a > 0.5) & (a < 1.0), ramp, 0.0)
    return np.where(a <= 0.5, 1.0, out)
