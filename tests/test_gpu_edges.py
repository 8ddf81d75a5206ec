"""Edge cases on the GPU through the C ABI, against the FP64 oracle:
all-zero spectra (J above the default, so that coarse scales fall between
grid points), the largest supported sides (4096 and 3 * 2^10) on sampled
planes, and a mixed-radix 1536 x 1536 image."""

import numpy as np
import pytest
import torch

from oracle import complex_shearlets as ocs
from paper_1202_1773_amd import Plan
from paper_1202_1773_amd.synthetic import cartoon, gaussian

from gpu_helpers import (log, oracle_adjoint, oracle_forward, oracle_spectra, per_plane_rel_l2,
                         rel_l2)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-5


@pytest.mark.parametrize("M,N,J", [(64, 64, 6), (32, 48, 4), (16, 16, 5)])
def test_zero_spectra(M, N, J):
    # Delta = 2^(2J) / L grows with J; at these sizes whole scales have no grid
    # point in their support, so many spectra are identically zero
    log(f"zero spectra {M}x{N} J={J}")
    psi = oracle_spectra(M, N, J)
    # "zero": every value below 1e-12 (the oracle keeps rounding residues such
    # as cos(pi/2) = 6e-17 at window breakpoints, the device's closed form 0)
    peak = np.abs(psi).reshape(psi.shape[0], -1).max(axis=1)
    zero = int((peak < 1e-12).sum())
    assert zero > 0
    plan = Plan(M, N, J)
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - psi)) <= 1.2e-7
    lo, hi = plan.windows()
    assert sum(1 for a in lo if a == -1) >= zero
    f = gaussian(M, N, seed=M + J)
    c = plan.forward(torch.from_numpy(f).to(DEV)).cpu().numpy()
    ref = oracle_forward(f, M, N, J)
    nz = peak >= 1e-12
    assert per_plane_rel_l2(c[nz], ref[nz]).max() <= TOL
    assert np.max(np.abs(c[~nz])) <= 1e-12 * np.linalg.norm(f)
    d = np.random.default_rng(J).standard_normal(c.shape).astype(np.float32)
    y = plan.adjoint(torch.from_numpy(d).to(DEV)).cpu().numpy()
    assert rel_l2(y, oracle_adjoint(d, M, N, J)) <= TOL
    assert rel_l2(plan.adjoint(torch.from_numpy(c).to(DEV)).cpu().numpy(), f) <= TOL
    plan.close()
    cplan = Plan(M, N, J, complex_shearlets=True)
    pp = ocs.one_sided_spectra(M, N, J)
    cc = cplan.forward(torch.from_numpy(f).to(DEV))
    cref = ocs.forward(f.astype(np.float64), pp)
    num = np.sqrt((np.abs(cc.cpu().numpy() - cref) ** 2).sum(axis=(-2, -1)))
    den = np.sqrt((np.abs(cref) ** 2).sum(axis=(-2, -1)))
    big = den > 1e-12 * np.linalg.norm(f)
    assert (num[big] / den[big]).max() <= TOL and np.max(num[~big], initial=0.0) <= 1e-11 * np.linalg.norm(f)
    assert rel_l2(cplan.adjoint(cc).cpu().numpy(), f) <= TOL
    cplan.close()


# The FP64 oracle's textbook FFTs of a 4096 x 4096 image take about two
# minutes of host time, more than the per-test limit of the GPU runs.
@pytest.mark.timeout(400)
@pytest.mark.parametrize("M,N,J,planes", [(4096, 4096, 6, [0, 252]), (3072, 3072, 5, [3, 124]),
                                          (1536, 1536, 5, [0, 11, 50, 124])])
def test_largest_sides_sampled(M, N, J, planes):
    log(f"largest sides {M}x{N} J={J}, planes {planes}")
    plan = Plan(M, N, J)
    f = cartoon(M, N, 40, 10, 0.1, seed=777)
    x = torch.from_numpy(f).to(DEV)
    c = plan.forward(x)
    log("  GPU done; oracle planes (FP64 FFTs of the full image on the host)")
    ref = oracle_forward(f, M, N, J, planes=planes)
    err = per_plane_rel_l2(c[planes].cpu().numpy(), ref)
    log(f"  sampled max plane relL2 {err.max():.2e}")
    assert err.max() <= TOL
    y = plan.adjoint(c)
    assert float(torch.linalg.norm(y - x) / torch.linalg.norm(x)) <= TOL
    energy = sum(float((c[i].double() ** 2).sum()) for i in range(plan.eta)) / float((x.double() ** 2).sum())
    assert abs(energy - 1.0) <= 1e-5
    del c, y
    plan.close()
    torch.cuda.empty_cache()
