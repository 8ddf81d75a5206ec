"""Shared helpers for the GPU parity tests: oracle references (cached per
process) and error measures. Inputs come from the seeded generator; the
oracle always receives float64 of the exact float32 arrays the GPU gets."""

import functools
import sys

import numpy as np

from oracle import spectra as ospec
from oracle import transform as otr


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=8)
def oracle_spectra(M, N, J, max_scale="max", shearlet="meyer"):
    return ospec.spectra(M, N, J, max_scale=max_scale, shearlet=shearlet)


def oracle_forward(f32, M, N, J, planes=None, max_scale="max", shearlet="meyer"):
    if planes is None:
        psi = oracle_spectra(M, N, J, max_scale, shearlet)
        return otr.forward(np.asarray(f32, dtype=np.float64), psi)
    plane = lambda i: ospec.spectrum_plane(M, N, J, i, max_scale, True, shearlet)  # noqa: E731
    return otr.forward(np.asarray(f32, dtype=np.float64), plane, planes=planes)


def oracle_adjoint(c32, M, N, J, max_scale="max", shearlet="meyer"):
    psi = oracle_spectra(M, N, J, max_scale, shearlet)
    return otr.adjoint(np.asarray(c32, dtype=np.float64), psi)


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)


def per_plane_rel_l2(got, ref):
    """Relative L2 error of every coefficient plane (last two axes)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.sqrt(((got - ref) ** 2).sum(axis=(-2, -1)))
    den = np.sqrt((ref ** 2).sum(axis=(-2, -1)))
    return num / np.where(den > 0, den, 1.0)
