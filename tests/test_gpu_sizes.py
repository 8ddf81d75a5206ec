"""Every FFT length the library is compiled for, once as the column length M
and once as the row length N (real and complex shearlets), against the FP64
oracle: each kernel instantiation runs at least once with its own data."""

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
LENGTHS = POW2 + THREE + NINE


def _check(M, N, J, complex_shearlets):
    f = gaussian(M, N, seed=M * 7 + N)
    x = torch.from_numpy(f).to(DEV)
    plan = Plan(M, N, J, complex_shearlets=complex_shearlets)
    c = plan.forward(x)
    if complex_shearlets:
        pp = ocs.one_sided_spectra(M, N, J)
        ref = ocs.forward(f.astype(np.float64), pp)
        got = c.cpu().numpy()
        num = np.sqrt((np.abs(got - ref) ** 2).sum(axis=(-2, -1)))
        den = np.sqrt((np.abs(ref) ** 2).sum(axis=(-2, -1)))
        big = den > 1e-12 * np.linalg.norm(f)
        err = float((num[big] / den[big]).max())
    else:
        ref = oracle_forward(f, M, N, J)
        den = np.sqrt((ref ** 2).sum(axis=(-2, -1)))
        big = den > 1e-12 * np.linalg.norm(f)
        err = float(per_plane_rel_l2(c.cpu().numpy()[big], ref[big]).max())
    rec = rel_l2(plan.adjoint(c).cpu().numpy(), f)
    plan.close()
    return err, rec


@pytest.mark.parametrize("complex_shearlets", [False, True])
@pytest.mark.parametrize("L", LENGTHS)
def test_every_length(L, complex_shearlets):
    cases = [(L, 64)]
    if L % 2 == 0:
        cases.append((32, L))
    for M, N in cases:
        J = min(2, (max(M, N).bit_length() - 1) // 2)
        err, rec = _check(M, N, J, complex_shearlets)
        log(f"  {M}x{N} J={J} complex={complex_shearlets}: fwd {err:.2e} rec {rec:.2e}")
        assert err <= TOL and rec <= TOL, (M, N)


@pytest.mark.parametrize("complex_shearlets", [False, True])
@pytest.mark.parametrize("M,N", [(4, 4), (6, 6), (4, 6), (6, 4), (4, 8), (12, 6), (9, 4)])
def test_tiny_images(M, N, complex_shearlets):
    # the smallest sides: J = 1 (5 spectra), every line a single FFT stage
    err, rec = _check(M, N, 1, complex_shearlets)
    log(f"  {M}x{N} J=1 complex={complex_shearlets}: fwd {err:.2e} rec {rec:.2e}")
    assert err <= TOL and rec <= TOL, (M, N)
