"""Plans whose spectra are cut into several plane groups: the column passes
then run once per group over its own CSR, the adjoint adds the groups'
partial sums (its accumulate path) and images go one per unit. This happens
on its own only for very large images (a compact buffer above 1 GiB per
image, e.g. 4096 x 4096, J = 6); FFST_CHUNK_MB, read at plan creation, forces
it here at small sizes, for real and complex shearlets, against the FP64
oracle: forward per plane, adjoint of N(0, 1) coefficients, reconstruction."""

import os

import numpy as np
import pytest
import torch

from oracle import complex_shearlets as ocs
from paper_1202_1773_amd import Plan
from paper_1202_1773_amd.synthetic import cartoon

from gpu_helpers import log, oracle_adjoint, oracle_forward, per_plane_rel_l2, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-5


def _plan_with_chunk(M, N, J, mb, **kw):
    old = os.environ.get("FFST_CHUNK_MB")
    os.environ["FFST_CHUNK_MB"] = str(mb)
    try:
        return Plan(M, N, J, **kw)
    finally:
        if old is None:
            del os.environ["FFST_CHUNK_MB"]
        else:
            os.environ["FFST_CHUNK_MB"] = old


def _compact_mb(plan):
    # bytes of one image's compact intermediate, from the windows
    first, last = plan.windows()
    w = [(l - f) % (plan.N if plan.complex_shearlets else plan.N // 2 + 1) + 1 if f >= 0 else 0
         for f, l in zip(first, last)]
    pitch = plan.M + 16 if plan.M >= 64 else plan.M
    return sum(w) * pitch * 8 / 2 ** 20


@pytest.mark.parametrize("M,N,J", [(256, 256, 3), (192, 256, 3)])
def test_real_plane_groups(M, N, J):
    plan = _plan_with_chunk(M, N, J, 1)
    groups = _compact_mb(plan)
    log(f"real {M}x{N} J={J} with 1 MiB plane groups (compact buffer {groups:.1f} MiB per image)")
    assert groups > 2
    B = 3
    imgs = np.stack([cartoon(M, N, 8, 3, 0.1, seed=900 + b) for b in range(B)])
    x = torch.from_numpy(imgs).to(DEV)
    c = plan.forward(x).cpu().numpy()
    for b in range(B):
        assert per_plane_rel_l2(c[b], oracle_forward(imgs[b], M, N, J)).max() <= TOL, b
    g = torch.Generator(device=DEV).manual_seed(M + N)
    r = torch.randn((B, plan.eta, M, N), device=DEV, generator=g)
    y = plan.adjoint(r).cpu().numpy()
    rn = r.cpu().numpy()
    for b in range(B):
        assert rel_l2(y[b], oracle_adjoint(rn[b], M, N, J)) <= TOL, b
    assert rel_l2(plan.adjoint(torch.from_numpy(c).to(DEV)).cpu().numpy(), imgs) <= TOL
    plan.close()


@pytest.mark.parametrize("M,N,J", [(256, 256, 3), (192, 256, 3)])
def test_complex_plane_groups(M, N, J):
    plan = _plan_with_chunk(M, N, J, 1, complex_shearlets=True)
    groups = _compact_mb(plan)
    log(f"complex {M}x{N} J={J} with 1 MiB plane groups (compact buffer {groups:.1f} MiB per image)")
    assert groups > 2
    pp = ocs.one_sided_spectra(M, N, J)
    B = 2
    imgs = np.stack([cartoon(M, N, 8, 3, 0.1, seed=950 + b) for b in range(B)])
    x = torch.from_numpy(imgs).to(DEV)
    cc = plan.forward(x)
    cn = cc.cpu().numpy()
    for b in range(B):
        ref = ocs.forward(imgs[b].astype(np.float64), pp)
        num = np.sqrt((np.abs(cn[b] - ref) ** 2).sum(axis=(-2, -1)))
        den = np.sqrt((np.abs(ref) ** 2).sum(axis=(-2, -1)))
        big = den > 1e-12 * np.linalg.norm(imgs[b])
        assert (num[big] / den[big]).max() <= TOL, b
    g = torch.Generator(device=DEV).manual_seed(3 * M + N)
    re = torch.randn((B, plan.eta, M, N), device=DEV, generator=g)
    im = torch.randn((B, plan.eta, M, N), device=DEV, generator=g)
    d = torch.complex(re, im).contiguous()
    y = plan.adjoint(d).cpu().numpy()
    dn = d.cpu().numpy()
    for b in range(B):
        assert rel_l2(y[b], ocs.adjoint_real(dn[b].astype(np.complex128), pp)) <= TOL, b
    assert rel_l2(plan.adjoint(cc).cpu().numpy(), imgs) <= TOL
    plan.close()
