"""Differentiable FFST and the smooth-shearlet spectra on the GPU (through the
C ABI), checked against the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import spectra as ospec
from oracle import transform as otr
from paper_1202_1773_amd import Plan
from paper_1202_1773_amd.autograd import l1_denoise, l1_loss, shearlet_adjoint, shearlet_transform
from paper_1202_1773_amd.synthetic import cartoon, config2_batch

from gpu_helpers import log, per_plane_rel_l2, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def test_backward_is_the_oracle_adjoint():
    log("autograd backward vs oracle adjoint, 64x64 J=2")
    plan = Plan(64, 64, 2)
    rng = np.random.default_rng(21)
    x = torch.from_numpy(rng.standard_normal((64, 64)).astype(np.float32)).to(DEV).requires_grad_(True)
    w = rng.standard_normal((13, 64, 64)).astype(np.float32)
    out = (shearlet_transform(x, plan) * torch.from_numpy(w).to(DEV)).sum()
    (g,) = torch.autograd.grad(out, x)
    ref = otr.adjoint(w.astype(np.float64), ospec.spectra(64, 64, 2))
    assert rel_l2(g.cpu().numpy(), ref) <= 1e-5
    # adjoint's backward is the forward transform
    c = torch.from_numpy(w).to(DEV).requires_grad_(True)
    v = torch.from_numpy(rng.standard_normal((64, 64)).astype(np.float32)).to(DEV)
    (gc,) = torch.autograd.grad((shearlet_adjoint(c, plan) * v).sum(), c)
    refc = otr.forward(v.cpu().numpy().astype(np.float64), ospec.spectra(64, 64, 2))
    assert per_plane_rel_l2(gc.cpu().numpy(), refc).max() <= 1e-5
    plan.close()


def test_backward_complex_shearlets():
    # L = Re sum conj(W) c for complex W: the gradient is Re SH^H W, the
    # oracle's real-part adjoint of the one-sided system
    log("autograd backward, complex shearlets 64x64 J=2")
    from oracle import complex_shearlets as ocs
    plan = Plan(64, 64, 2, complex_shearlets=True)
    rng = np.random.default_rng(23)
    x = torch.from_numpy(rng.standard_normal((64, 64)).astype(np.float32)).to(DEV).requires_grad_(True)
    w = (rng.standard_normal((13, 64, 64)) + 1j * rng.standard_normal((13, 64, 64))).astype(np.complex64)
    c = shearlet_transform(x, plan)
    loss = (torch.conj(torch.from_numpy(w).to(DEV)) * c).real.sum()
    (g,) = torch.autograd.grad(loss, x)
    ref = ocs.adjoint_real(w.astype(np.complex128), ocs.one_sided_spectra(64, 64, 2))
    assert rel_l2(g.cpu().numpy(), ref) <= 1e-5
    plan.close()


def test_l1_gradient_matches_fp64_finite_differences():
    # 32x32 crops, J = 2 (13 spectra), lambda = 0.05, central differences with
    # h = 1e-6 on the FP64 oracle loss.
    log("l1 loss gradient vs FP64 central differences, 32x32 J=2")
    M = N = 32
    J = 2
    lam = 0.05
    imgs = config2_batch(1)[0]
    rng = np.random.default_rng(31)
    y = imgs[100:132, 200:232].astype(np.float64)
    x = (y + 0.1 * rng.standard_normal((M, N))).astype(np.float32).astype(np.float64)
    psi = ospec.spectra(M, N, J)

    def loss64(z):
        return 0.5 * np.sum((z - y) ** 2) + lam * np.sum(np.abs(otr.forward(z, psi)))

    plan = Plan(M, N, J)
    xt = torch.from_numpy(x.astype(np.float32)).to(DEV).requires_grad_(True)
    yt = torch.from_numpy(y.astype(np.float32)).to(DEV)
    (g,) = torch.autograd.grad(l1_loss(xt, yt, plan, lam), xt)
    g = g.cpu().numpy().astype(np.float64)
    # The sign of each coefficient is decided in the kernel's precision on
    # both sides: the oracle gradient (x - y) + lam SH*(s) uses the GPU's signs.
    s_gpu = np.sign(shearlet_transform(xt.detach(), plan).cpu().numpy()).astype(np.float64)
    g_or = (x - y) + lam * otr.adjoint(s_gpu, psi)
    assert rel_l2(g, g_or) <= 1e-5
    # The oracle's analytic gradient against FP64 central differences, at
    # pixels where no coefficient changes sign within +-h (the l1 term is
    # linear there).
    c64 = otr.forward(x, psi)
    g64 = (x - y) + lam * otr.adjoint(np.sign(c64), psi)
    h = 1e-6
    checked = 0
    for p in rng.permutation(M * N):
        e = np.zeros(M * N)
        e[p] = 1.0
        e = e.reshape(M, N)
        a = otr.forward(e, psi)
        if np.min(np.abs(c64) - h * np.abs(a)) <= 0:
            continue
        fd = (loss64(x + h * e) - loss64(x - h * e)) / (2 * h)
        assert abs(fd - g64.reshape(-1)[p]) <= 1e-6 * max(1.0, abs(fd)), (p, fd, g64.reshape(-1)[p])
        checked += 1
        if checked == 48:
            break
    assert checked == 48
    plan.close()


def test_l1_descent_16_images_200_steps():
    # 16 images 512x512, J = 3, y = cartoon + N(0, 0.1^2), lambda = 0.05.
    log("200 steps of l1 gradient descent, 16x512x512 J=3")
    plan = Plan(512, 512, 3)
    y = torch.from_numpy(np.stack([cartoon(512, 512, 20, 10, 0.1, seed=301 + b) for b in range(16)])).to(DEV)
    x, losses = l1_denoise(y, plan, lam=0.05, steps=200, lr=0.25)
    torch.cuda.synchronize()
    ls = losses.cpu().numpy()
    log(f"  loss {ls[0]:.6g} -> {ls[-1]:.6g}")
    assert np.all(np.isfinite(ls)) and torch.isfinite(x).all()
    assert ls[1] < ls[0] and ls[-1] < ls[0]
    plan.close()


def test_l1_descent_iterates_match_fp64_descent():
    # The first three iterates of l1 gradient descent on a 32x32 crop (J = 2,
    # lambda = 0.05, step 0.25) against the same descent in FP64 on the
    # oracle: x_{k+1} = x_k - lr ((x_k - y) + lam SH*(sign(SH x_k))). The sign
    # of each coefficient is decided in the kernel's precision on both sides
    # (the oracle takes the GPU's signs at the GPU's iterate), so the two
    # trajectories differ only by the transforms' rounding.
    log("l1 descent iterates vs FP64 oracle descent, 32x32 J=2")
    M = N = 32
    J = 2
    lam, lr = 0.05, 0.25
    rng = np.random.default_rng(37)
    clean = config2_batch(1)[0][300:332, 64:96].astype(np.float64)
    y = (clean + 0.1 * rng.standard_normal((M, N))).astype(np.float32)
    psi = ospec.spectra(M, N, J)
    plan = Plan(M, N, J)
    yt = torch.from_numpy(y).to(DEV)
    x_gpu = yt.clone()
    x_or = y.astype(np.float64)
    y64 = y.astype(np.float64)
    for k in range(3):
        s_gpu = np.sign(plan.forward(x_gpu).cpu().numpy()).astype(np.float64)
        x_gpu, _ = l1_denoise(yt, plan, lam=lam, steps=1, lr=lr, x0=x_gpu)
        x_or = x_or - lr * ((x_or - y64) + lam * otr.adjoint(s_gpu, psi))
        err = rel_l2(x_gpu.cpu().numpy(), x_or)
        log(f"  iterate {k + 1}: relL2 {err:.2e}")
        assert err <= 1e-5, (k, err)
    # the descent moved the iterate (the test is not vacuous)
    assert rel_l2(x_or, y64) > 1e-3
    plan.close()


@pytest.mark.parametrize("M,N,J", [(64, 64, 2), (512, 512, 3), (256, 512, 3)])
def test_smooth_spectra_and_transform(M, N, J):
    log(f"smooth shearlets {M}x{N} J={J}")
    plan = Plan(M, N, J, shearlet="smooth")
    ref = ospec.spectra(M, N, J, shearlet="smooth")
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1.2e-7
    f = cartoon(M, N, 12, 4, 0.1, seed=5)
    x = torch.from_numpy(f).to(DEV)
    c = plan.forward(x)
    err = per_plane_rel_l2(c.cpu().numpy(), otr.forward(f.astype(np.float64), ref))
    assert err.max() <= 1e-5
    y = plan.adjoint(c)
    assert rel_l2(y.cpu().numpy(), f) <= 1e-5
    plan.close()


def test_min_scale_option():
    log("maxScale 'min', 128x128 J=3")
    plan = Plan(128, 128, 3, max_scale="min")
    ref = ospec.spectra(128, 128, 3, max_scale="min")
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1.2e-7
    f = cartoon(128, 128, 8, 3, 0.1, seed=9)
    c = plan.forward(torch.from_numpy(f).to(DEV))
    assert per_plane_rel_l2(c.cpu().numpy(), otr.forward(f.astype(np.float64), ref)).max() <= 1e-5
    plan.close()
