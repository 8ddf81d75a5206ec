"""Image sides 3 * 2^k and 9 * 2^k (mixed-radix FFTs with radix 12 = 3 * 4
and 18 = 2 * 9) on the GPU through the C ABI, against the FP64 oracle:
spectra, forward, adjoint for real and complex shearlets, including the sizes
of the uneven-batch workload (384 x 512 and 768 x 1024)."""

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

CASES = [(12, 12, 1), (24, 48, 2), (48, 24, 2), (96, 96, 2), (96, 64, 3), (64, 96, 3), (192, 192, 3),
         (384, 512, 3), (512, 384, 3), (384, 384, 3),
         # 9 * 2^k (radix-9 / radix-18 stages), odd M = 9 included
         (9, 18, 1), (18, 36, 2), (72, 144, 3), (144, 144, 3), (288, 576, 4), (576, 288, 4), (1152, 128, 4)]


@pytest.mark.parametrize("M,N,J", CASES)
def test_real_shearlets(M, N, J):
    log(f"radix-3 real {M}x{N} J={J}")
    plan = Plan(M, N, J)
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - oracle_spectra(M, N, J))) <= 1.2e-7
    f = cartoon(M, N, 10, 4, 0.1, seed=M + N) if min(M, N) >= 24 else gaussian(M, N, seed=M)
    x = torch.from_numpy(f).to(DEV)
    c = plan.forward(x).cpu().numpy()
    err = per_plane_rel_l2(c, oracle_forward(f, M, N, J))
    log(f"  fwd max plane relL2 {err.max():.2e}")
    assert err.max() <= TOL
    rng = np.random.default_rng(M * N)
    d = rng.standard_normal((plan.eta, M, N)).astype(np.float32)
    y = plan.adjoint(torch.from_numpy(d).to(DEV)).cpu().numpy()
    assert rel_l2(y, oracle_adjoint(d, M, N, J)) <= TOL
    assert rel_l2(plan.adjoint(torch.from_numpy(c).to(DEV)).cpu().numpy(), f) <= TOL
    # batched equals separate
    xb = torch.stack([x, x.flip(0)])
    cb = plan.forward(xb)
    assert torch.equal(cb[0].cpu(), torch.from_numpy(c))
    plan.close()


@pytest.mark.parametrize("M,N,J", [(768, 1024, 4), (1024, 768, 4), (2304, 2304, 5)])
def test_large_sampled(M, N, J):
    log(f"radix-3 {M}x{N} J={J}, sampled planes")
    plan = Plan(M, N, J)
    f = cartoon(M, N, 20, 10, 0.1, seed=403)
    x = torch.from_numpy(f).to(DEV)
    c = plan.forward(x)
    planes = [0, 1, 7, 20, 33, 45, 60] if plan.eta < 100 else [0, 13, 124]
    ref = oracle_forward(f, M, N, J, planes=planes)
    err = per_plane_rel_l2(c[planes].cpu().numpy(), ref)
    log(f"  fwd sampled max plane relL2 {err.max():.2e}")
    assert err.max() <= TOL
    assert rel_l2(plan.adjoint(c).cpu().numpy(), f) <= TOL
    plan.close()


@pytest.mark.parametrize("M,N,J", [(96, 48, 2), (384, 512, 3), (48, 96, 2), (144, 288, 3), (9, 36, 1)])
def test_complex_shearlets(M, N, J):
    log(f"radix-3 complex {M}x{N} J={J}")
    plan = Plan(M, N, J, complex_shearlets=True)
    pp = ocs.one_sided_spectra(M, N, J)
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - pp)) <= 1.2e-7
    f = cartoon(M, N, 10, 4, 0.1, seed=5 * M + N)
    c = plan.forward(torch.from_numpy(f).to(DEV))
    ref = ocs.forward(f.astype(np.float64), pp)
    num = np.sqrt((np.abs(c.cpu().numpy() - ref) ** 2).sum(axis=(-2, -1)))
    den = np.sqrt((np.abs(ref) ** 2).sum(axis=(-2, -1)))
    assert (num / np.where(den > 0, den, 1)).max() <= TOL
    assert rel_l2(plan.adjoint(c).cpu().numpy(), f) <= TOL
    plan.close()
