"""The adjoint (eq. inverseShearletTransform, Sec. 3.3) in every launch form
the library can pick, on coefficients OUTSIDE the range of the forward map.

Reconstruction only tests coefficients c = SH f; an adjoint error that
vanishes on that range would pass it unseen. Here the coefficients are
i.i.d. N(0, 1) (a random coefficient array has almost all of its energy
outside the range of SH), and every sampled image's adjoint is compared with
the FP64 oracle adjoint of the same float32 coefficients. Each case forces
one form of the adjoint's sum over the spectra through the plan's tuning:
nparts = 1 (the column pass ends with its own inverse FFT) and nparts = 4
(partial sums added in a fixed order by a separate inverse column pass), at
the benchmark's shape (16 x 512^2, J = 3), at B = 8, for the largest class
of the uneven batch (1024^2, J = 4) and for complex shearlets. The
dot-product identity <SH x, r> = <x, SH* r> is checked at B = 16 as well.
"""

import numpy as np
import pytest
import torch

from oracle import complex_shearlets as ocs
from paper_1202_1773_amd import BatchPlan, Plan, _lib
from paper_1202_1773_amd.synthetic import config2_batch, uneven_sizes

from gpu_helpers import log, oracle_adjoint, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-5


def _random_coefficients(shape, seed):
    g = torch.Generator(device=DEV).manual_seed(seed)
    return torch.randn(shape, device=DEV, generator=g, dtype=torch.float32)


@pytest.mark.parametrize("B", [16, 8])
@pytest.mark.parametrize("nparts", [1, 4, 0])
def test_adjoint_of_random_coefficients_512(B, nparts):
    # nparts = 0 is the library's own choice for this batch (the benchmark's
    # plan before tuning).
    log(f"adjoint of N(0,1) coefficients, {B}x512x512 J=3, nparts={nparts}")
    plan = Plan(512, 512, 3)
    plan.set_tuning(nparts, 0)
    c = _random_coefficients((B, plan.eta, 512, 512), seed=1000 + 10 * B + nparts)
    y = plan.adjoint(c)
    torch.cuda.synchronize()
    for b in sorted({0, B // 2 + 1, B - 1}):
        ref = oracle_adjoint(c[b].cpu().numpy(), 512, 512, 3)
        err = rel_l2(y[b].cpu().numpy(), ref)
        log(f"  image {b}: adjoint relL2 {err:.2e}")
        assert err <= TOL, (b, err)
    plan.close()


def test_dot_product_identity_16_images():
    # <SH x, r> = <x, SH* r> for the 16 benchmark images and random r, in the
    # benchmark's launch form (the library's own choice for B = 16)
    log("dot-product identity, 16x512x512 J=3")
    plan = Plan(512, 512, 3)
    x = torch.from_numpy(config2_batch(16)).to(DEV)
    r = _random_coefficients((16, plan.eta, 512, 512), seed=77)
    cd = plan.forward(x).double()
    lhs = (cd * r.double()).sum().item()
    rhs = (x.double() * plan.adjoint(r).double()).sum().item()
    scale = float(torch.linalg.norm(cd) * torch.linalg.norm(r.double()))
    log(f"  <SHx,r> {lhs:.9e} <x,SH*r> {rhs:.9e} rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-6 * scale
    plan.close()


@pytest.mark.parametrize("nparts", [1, 4])
def test_adjoint_uneven_batch_largest_class(nparts):
    # The 64-image uneven batch; its 1024 x 1024 (J = 4) class is forced to
    # one adjoint form and a sampled image of it is checked against the
    # oracle adjoint of random coefficients.
    log(f"uneven batch, 1024x1024 J=4 class, adjoint of N(0,1) coefficients, nparts={nparts}")
    sizes, Js = uneven_sizes()
    bp = BatchPlan(sizes, Js)
    cls = None
    for k in range(bp.classes):
        h, n = _lib.ffst_batch_class(bp._h, k)
        if _lib.ffst_plan_info(h)[:3] == (1024, 1024, 4):
            cls = (h, n)
    assert cls is not None
    _lib.ffst_set_tuning(cls[0], nparts, 0)
    c = _random_coefficients((bp.coef_total,), seed=500 + nparts)
    y = bp.adjoint(c)
    torch.cuda.synchronize()
    big = [b for b, s in enumerate(sizes) if s == (1024, 1024)]
    views, imgs = bp.coefficients(c), bp.images(y)
    for b in (big[0], big[-1]):
        ref = oracle_adjoint(views[b].cpu().numpy(), 1024, 1024, 4)
        err = rel_l2(imgs[b].cpu().numpy(), ref)
        log(f"  image {b}: adjoint relL2 {err:.2e}")
        assert err <= TOL, (b, err)
    # one image of another class (its own default form)
    other = next(b for b, s in enumerate(sizes) if s == (384, 512))
    ref = oracle_adjoint(views[other].cpu().numpy(), 384, 512, 3)
    assert rel_l2(imgs[other].cpu().numpy(), ref) <= TOL
    bp.close()


@pytest.mark.parametrize("M,N,J", [(64, 64, 2), (96, 128, 3), (256, 256, 3)])
@pytest.mark.parametrize("nparts", [1, 4])
def test_adjoint_complex_random_coefficients(M, N, J, nparts):
    log(f"complex adjoint of N(0,1) coefficients, {M}x{N} J={J}, nparts={nparts}")
    plan = Plan(M, N, J, complex_shearlets=True)
    plan.set_tuning(nparts, 0)
    B = 3
    re = _random_coefficients((B, plan.eta, M, N), seed=M + N + nparts)
    im = _random_coefficients((B, plan.eta, M, N), seed=M + N + nparts + 1)
    c = torch.complex(re, im).contiguous()
    y = plan.adjoint(c)
    torch.cuda.synchronize()
    pp = ocs.one_sided_spectra(M, N, J)
    for b in range(B):
        ref = ocs.adjoint_real(c[b].cpu().numpy().astype(np.complex128), pp)
        err = rel_l2(y[b].cpu().numpy(), ref)
        assert err <= TOL, (b, err)
    plan.close()


@pytest.mark.parametrize("M,N,J", [(64, 64, 2), (48, 96, 2), (1024, 1024, 4)])
@pytest.mark.parametrize("nparts", [1, 4])
def test_adjoint_real_forced_forms(M, N, J, nparts):
    log(f"real adjoint of N(0,1) coefficients, {M}x{N} J={J}, nparts={nparts}")
    plan = Plan(M, N, J)
    plan.set_tuning(nparts, 0)
    B = 2
    c = _random_coefficients((B, plan.eta, M, N), seed=3 * M + N + nparts)
    y = plan.adjoint(c)
    torch.cuda.synchronize()
    for b in range(B):
        ref = oracle_adjoint(c[b].cpu().numpy(), M, N, J)
        assert rel_l2(y[b].cpu().numpy(), ref) <= TOL, b
    plan.close()
