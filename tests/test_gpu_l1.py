"""The adjoint of the l1 subgradient, SH*(s sign(c)), with the sign applied
inside the adjoint kernels: equal up to rounding to the plain adjoint of
s * sign(c), and the l1 loss built on it against the FP64 oracle."""

import ctypes

import numpy as np
import pytest
import torch

from oracle import spectra as ospec
from oracle import transform as otr
from paper_1202_1773_amd import Plan, _lib
from paper_1202_1773_amd.autograd import l1_loss, shearlet_l1
from paper_1202_1773_amd.synthetic import cartoon

from gpu_helpers import log, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("M,N,J,B", [(64, 64, 2, 1), (512, 512, 3, 2), (27, 81, 2, 3), (144, 288, 3, 2),
                                     (8, 8, 1, 4)])
def test_adjoint_sign_equals_adjoint_of_scaled_signs(M, N, J, B):
    log(f"adjoint_sign {M}x{N} J={J} B={B}")
    plan = Plan(M, N, J)
    x = torch.from_numpy(np.stack([cartoon(M, N, 8, 3, 0.1, seed=400 + b) for b in range(B)])).to(DEV)
    c = plan.forward(x)
    c[:, :, 0, 0] = 0.0          # exact zeros: sign 0
    s = torch.tensor([0.037], dtype=torch.float32, device=DEV)
    got = plan.adjoint_sign(c, s)
    ref = plan.adjoint((torch.sign(c) * s).contiguous())
    # the same kernels on the same values, compiled as a separate
    # instantiation (the compiler may contract or order the FFT's float
    # operations differently): equal up to rounding
    err = rel_l2(got.cpu().numpy(), ref.cpu().numpy())
    log(f"  rel L2 {err:.2e}, bit-identical {bool(torch.equal(got, ref))}")
    assert err <= 1e-6
    plan.close()


def test_adjoint_sign_rejects_complex_plans_and_null_scale():
    plan = Plan(16, 16, 2)
    c = torch.zeros((13, 16, 16), dtype=torch.float32, device=DEV)
    f = torch.empty((16, 16), dtype=torch.float32, device=DEV)
    lib = _lib.load()
    P = ctypes.c_void_p
    st = lib.ffst_adjoint_sign(P(plan._h), P(c.data_ptr()), P(f.data_ptr()), 1, None, P(plan.workspace(1)), None)
    assert st == _lib.FFST_EINVAL
    plan.close()
    cplan = Plan(16, 16, 2, complex_shearlets=True)
    with pytest.raises(ValueError):
        cplan.adjoint_sign(torch.zeros((13, 16, 16), dtype=torch.complex64, device=DEV),
                           torch.ones(1, device=DEV))
    cc = torch.zeros((13, 16, 16), dtype=torch.complex64, device=DEV)
    s = torch.ones(1, device=DEV)
    st = lib.ffst_adjoint_sign(P(cplan._h), P(cc.data_ptr()), P(f.data_ptr()), 1, P(s.data_ptr()),
                               P(cplan.workspace(1)), None)
    assert st == _lib.FFST_EINVAL
    cplan.close()


def test_l1_term_value_and_gradient_against_the_oracle():
    # lam ||SH x||_1 and its gradient lam SH*(sign(SH x)), the sign taken from
    # the GPU coefficients (the decision in the kernel's precision)
    log("l1 term and gradient vs oracle, 64x48 J=2, batch 2")
    M, N, J, lam = 64, 48, 2, 0.05
    plan = Plan(M, N, J)
    psi = ospec.spectra(M, N, J)
    xs = np.stack([cartoon(M, N, 8, 3, 0.1, seed=440 + b) for b in range(2)])
    x = torch.from_numpy(xs).to(DEV).requires_grad_(True)
    val = shearlet_l1(x, plan, lam)
    (g,) = torch.autograd.grad(val, x)
    c_gpu = plan.forward(x.detach()).cpu().numpy().astype(np.float64)
    for b in range(2):
        c64 = otr.forward(xs[b].astype(np.float64), psi)
        ref_g = lam * otr.adjoint(np.sign(c_gpu[b]), psi)
        assert rel_l2(g[b].cpu().numpy(), ref_g) <= 1e-5
    ref_val = lam * sum(np.abs(otr.forward(xs[b].astype(np.float64), psi)).sum() for b in range(2))
    assert abs(float(val.detach()) - ref_val) <= 1e-5 * ref_val
    # the loss as the descent uses it: same gradient as the unfused formula
    y = torch.from_numpy(xs[::-1].copy()).to(DEV)
    (g1,) = torch.autograd.grad(l1_loss(x, y, plan, lam), x)
    cx = plan.forward(x.detach())
    g2 = (x.detach() - y) + plan.adjoint((lam * torch.sign(cx)).contiguous())
    assert rel_l2(g1.cpu().numpy(), g2.cpu().numpy()) <= 1e-6
    plan.close()
