"""Every FFT length the library is compiled for, once as the column length M
and once as the row length N (odd N through the odd-row kernels), with real
and complex shearlets, against the FP64 oracle: each kernel instantiation
runs at least once with its own data. Planes whose oracle norm is
negligible (<= 1e-12 ||f||, spectra that vanish on small grids) are not
compared relatively; the GPU must write (numerically) zero there instead."""

import numpy as np
import pytest
import torch

from oracle import complex_shearlets as ocs
from paper_1202_1773_amd import Plan
from paper_1202_1773_amd.synthetic import gaussian

from gpu_helpers import log, oracle_forward, per_plane_rel_l2, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-5

POW2 = [4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
THREE = [6, 12, 24, 48, 96, 192, 384, 768, 1536, 3072]
NINE = [9, 18, 36, 72, 144, 288, 576, 1152, 2304]
# 27 and higher powers of 3: groups that are not a power of two lanes wide
HIGHER = [27, 54, 108, 216, 432, 864, 1728, 3456, 81, 162, 324, 648, 1296, 2592,
          243, 486, 972, 1944, 3888, 729, 1458, 2916, 2187]
LENGTHS = POW2 + THREE + NINE + HIGHER


def _check(M, N, J, complex_shearlets, batch=1):
    fs = [gaussian(M, N, seed=M * 7 + N + b) for b in range(batch)]
    x = torch.from_numpy(np.stack(fs)).to(DEV)
    plan = Plan(M, N, J, complex_shearlets=complex_shearlets)
    c = plan.forward(x)
    y = plan.adjoint(c).cpu().numpy()
    err = rec = 0.0
    for b, f in enumerate(fs):
        if complex_shearlets:
            pp = ocs.one_sided_spectra(M, N, J)
            ref = ocs.forward(f.astype(np.float64), pp)
            got = c[b].cpu().numpy()
            num = np.sqrt((np.abs(got - ref) ** 2).sum(axis=(-2, -1)))
            den = np.sqrt((np.abs(ref) ** 2).sum(axis=(-2, -1)))
            big = den > 1e-12 * np.linalg.norm(f)
            err = max(err, float((num[big] / den[big]).max()))
            # planes the oracle gives as (numerically) zero must be ~0 on the GPU
            assert np.abs(got[~big]).max(initial=0.0) <= 1e-11 * np.linalg.norm(f), (M, N, b)
        else:
            ref = oracle_forward(f, M, N, J)
            den = np.sqrt((ref ** 2).sum(axis=(-2, -1)))
            big = den > 1e-12 * np.linalg.norm(f)
            got = c[b].cpu().numpy()
            err = max(err, float(per_plane_rel_l2(got[big], ref[big]).max()))
            assert np.abs(got[~big]).max(initial=0.0) <= 1e-11 * np.linalg.norm(f), (M, N, b)
        rec = max(rec, rel_l2(y[b], f))
    plan.close()
    return err, rec


@pytest.mark.parametrize("complex_shearlets", [False, True])
@pytest.mark.parametrize("L", LENGTHS)
def test_every_length(L, complex_shearlets):
    cases = [(L, 64), (32, L)]
    for M, N in cases:
        J = min(2, (max(M, N).bit_length() - 1) // 2)
        err, rec = _check(M, N, J, complex_shearlets)
        log(f"  {M}x{N} J={J} complex={complex_shearlets}: fwd {err:.2e} rec {rec:.2e}")
        assert err <= TOL and rec <= TOL, (M, N)


@pytest.mark.parametrize("complex_shearlets", [False, True])
@pytest.mark.parametrize("M,N", [(4, 4), (6, 6), (4, 6), (6, 4), (4, 8), (12, 6), (9, 4), (9, 9), (4, 9)])
def test_tiny_images(M, N, complex_shearlets):
    # the smallest sides: J = 1 (5 spectra), every line a single FFT stage
    err, rec = _check(M, N, 1, complex_shearlets)
    log(f"  {M}x{N} J=1 complex={complex_shearlets}: fwd {err:.2e} rec {rec:.2e}")
    assert err <= TOL and rec <= TOL, (M, N)


@pytest.mark.parametrize("complex_shearlets", [False, True])
@pytest.mark.parametrize("M,N,J", [(216, 216, 3), (324, 162, 3), (243, 486, 3), (108, 864, 3), (81, 54, 2),
                                   (27, 81, 2), (96, 243, 3), (243, 729, 3)])
def test_higher_powers_of_three(M, N, J, complex_shearlets):
    # both sides with 27 or more as a factor, two images per call
    err, rec = _check(M, N, J, complex_shearlets, batch=2)
    log(f"  {M}x{N} J={J} complex={complex_shearlets} batch 2: fwd {err:.2e} rec {rec:.2e}")
    assert err <= TOL and rec <= TOL, (M, N)
