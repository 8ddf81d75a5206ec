"""Spectra with the other auxiliary functions v (Remark on the construction
of v: C^k polynomials and the C-infinity function) on the GPU, against the
FP64 oracle, for Meyer, smooth and complex shearlets."""

import numpy as np
import pytest
import torch

from oracle import complex_shearlets as ocs
from oracle import spectra as ospec
from oracle import transform as otr
from paper_1202_1773_amd import Plan
from paper_1202_1773_amd.synthetic import cartoon

from gpu_helpers import log, per_plane_rel_l2, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("aux", [1, 5, 10, "inf"])
@pytest.mark.parametrize("shearlet", ["meyer", "smooth"])
@pytest.mark.parametrize("M,N,J", [(64, 64, 2), (256, 512, 3)])
def test_spectra_match_oracle(aux, shearlet, M, N, J):
    log(f"aux={aux} {shearlet} {M}x{N} J={J}")
    plan = Plan(M, N, J, shearlet=shearlet, aux=aux)
    ref = ospec.spectra(M, N, J, shearlet=shearlet, aux=aux)
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1.2e-7
    plan.close()


@pytest.mark.parametrize("aux", [2, "inf"])
def test_transforms_match_oracle(aux):
    log(f"aux={aux} transforms 128x128 J=3")
    M = N = 128
    f = cartoon(M, N, 8, 3, 0.1, seed=13)
    x = torch.from_numpy(f).to(DEV)
    plan = Plan(M, N, 3, aux=aux)
    psi = ospec.spectra(M, N, 3, aux=aux)
    c = plan.forward(x)
    assert per_plane_rel_l2(c.cpu().numpy(), otr.forward(f.astype(np.float64), psi)).max() <= 1e-5
    assert rel_l2(plan.adjoint(c).cpu().numpy(), f) <= 1e-5
    plan.close()
    cplan = Plan(M, N, 3, complex_shearlets=True, aux=aux)
    pp = ocs.one_sided_spectra(M, N, 3, aux=aux)
    got = cplan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - pp)) <= 1.2e-7
    cc = cplan.forward(x)
    ref = ocs.forward(f.astype(np.float64), pp)
    num = np.sqrt((np.abs(cc.cpu().numpy() - ref) ** 2).sum(axis=(-2, -1)))
    den = np.sqrt((np.abs(ref) ** 2).sum(axis=(-2, -1)))
    assert (num / np.where(den > 0, den, 1)).max() <= 1e-5
    assert rel_l2(cplan.adjoint(cc).cpu().numpy(), f) <= 1e-5
    cplan.close()
