"""Complex shearlets (one-sided spectra, Sec. 3.8.2) on the GPU through the
C ABI, against the FP64 oracle.

Bar: relative L2 error <= 1e-5 on every complex coefficient plane and for
the adjoint / reconstruction; one-sided spectra within one float32 rounding
(1.2e-7) of the oracle's float64 values.
"""

import ctypes
import functools

import numpy as np
import pytest
import torch

from oracle import complex_shearlets as ocs
from paper_1202_1773_amd import Plan, _lib
from paper_1202_1773_amd.synthetic import cartoon, config1_image, config2_batch, gaussian

from gpu_helpers import log, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-5


@functools.lru_cache(maxsize=6)
def oracle_plus(M, N, J, shearlet="meyer"):
    return ocs.one_sided_spectra(M, N, J, shearlet=shearlet)


def plane_rel_l2(got, ref):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    num = np.sqrt((np.abs(got - ref) ** 2).sum(axis=(-2, -1)))
    den = np.sqrt((np.abs(ref) ** 2).sum(axis=(-2, -1)))
    return num / np.where(den > 0, den, 1.0)


def images(kind, M, N, B=1):
    if kind == "config1":
        return config1_image()[None]
    if kind == "config2":
        return config2_batch(B)
    if kind == "gauss":
        return np.stack([gaussian(M, N, seed=102 + b) for b in range(B)])
    return np.stack([cartoon(M, N, 12, 4, 0.1, seed=7 + b) for b in range(B)])


SPECTRA_CASES = [(8, 8, 1), (16, 16, 2), (64, 64, 2), (128, 64, 3), (512, 512, 3), (256, 512, 3),
                 (512, 256, 3), (1024, 1024, 5)]


@pytest.mark.parametrize("M,N,J", SPECTRA_CASES)
def test_one_sided_spectra_and_windows(M, N, J):
    log(f"one-sided spectra {M}x{N} J={J}")
    plan = Plan(M, N, J, complex_shearlets=True)
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    ref = oracle_plus(M, N, J)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1.2e-7
    # frame identity over grid pairs (w, -w)
    mir = got[:, (-np.arange(M)) % M][:, :, (-np.arange(N)) % N]
    assert np.max(np.abs((got ** 2 + mir ** 2).sum(0) - 2.0)) < 2e-6
    # cyclic windows: hold every nonzero column of the device's spectra (the
    # value check above bounds what lies outside), and start and end on one
    lo, last = plan.windows()
    for i in range(plan.eta):
        nz = set(np.nonzero(np.any(got[i] != 0.0, axis=0))[0].tolist())
        if not nz:
            assert lo[i] == -1 and last[i] == -1
            continue
        w = (last[i] - lo[i]) % N + 1
        cols = {(lo[i] + m) % N for m in range(w)}
        assert nz <= cols and lo[i] in nz and last[i] in nz, i
    with pytest.raises(_lib.FfstError):
        plan.spectra(full_plane=False)
    plan.close()


FWD_CASES = [(64, 64, 2, "config1"), (512, 512, 3, "config2"), (256, 512, 3, "cartoon"),
             (512, 256, 3, "cartoon"), (8, 8, 1, "gauss"), (16, 16, 2, "gauss"), (128, 64, 3, "cartoon"),
             (64, 128, 2, "gauss")]


@pytest.mark.parametrize("M,N,J,kind", FWD_CASES)
def test_forward_adjoint_match_oracle(M, N, J, kind):
    log(f"complex forward/adjoint {M}x{N} J={J} {kind}")
    f = images(kind, M, N)[0]
    plan = Plan(M, N, J, complex_shearlets=True)
    pp = oracle_plus(M, N, J)
    c = plan.forward(torch.from_numpy(f).to(DEV))
    assert c.dtype == torch.complex64 and c.shape == (plan.eta, M, N)
    cg = c.cpu().numpy()
    ref = ocs.forward(f.astype(np.float64), pp)
    err = plane_rel_l2(cg, ref)
    log(f"  fwd max plane relL2 {err.max():.2e}")
    assert err.max() <= TOL, (int(err.argmax()), err.max())
    # Parseval and reconstruction
    energy = float((np.abs(cg.astype(np.complex128)) ** 2).sum() / (f.astype(np.float64) ** 2).sum())
    assert abs(energy - 1.0) < 1e-5
    y = plan.adjoint(c).cpu().numpy()
    assert rel_l2(y, f) <= TOL
    # adjoint of arbitrary complex coefficients
    rng = np.random.default_rng(M * 7 + N)
    d = (rng.standard_normal((plan.eta, M, N)) + 1j * rng.standard_normal((plan.eta, M, N))).astype(np.complex64)
    g = plan.adjoint(torch.from_numpy(d).to(DEV)).cpu().numpy()
    gref = ocs.adjoint_real(d.astype(np.complex128), pp)
    e2 = rel_l2(g, gref)
    log(f"  adj relL2 {e2:.2e}")
    assert e2 <= TOL
    plan.close()


def test_smooth_complex():
    log("complex smooth shearlets 128x128 J=3")
    M = N = 128
    plan = Plan(M, N, 3, shearlet="smooth", complex_shearlets=True)
    pp = oracle_plus(M, N, 3, "smooth")
    got = plan.spectra(full_plane=True).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - pp)) <= 1.2e-7
    f = cartoon(M, N, 8, 3, 0.1, seed=11)
    c = plan.forward(torch.from_numpy(f).to(DEV))
    assert plane_rel_l2(c.cpu().numpy(), ocs.forward(f.astype(np.float64), pp)).max() <= TOL
    assert rel_l2(plan.adjoint(c).cpu().numpy(), f) <= TOL
    plan.close()


def test_batched_equals_separate():
    log("complex batched vs separate, 3 x 128x128 J=3")
    M = N = 128
    plan = Plan(M, N, 3, complex_shearlets=True)
    imgs = images("cartoon", M, N, B=3)
    x = torch.from_numpy(imgs).to(DEV)
    cb = plan.forward(x)
    yb = plan.adjoint(cb)
    for b in range(3):
        c1 = plan.forward(x[b])
        assert torch.equal(c1, cb[b])
        y1 = plan.adjoint(c1)
        assert float((y1 - yb[b]).abs().max()) <= 1e-6
    # deterministic
    assert torch.equal(plan.forward(x), cb)
    plan.close()


def test_bench_shape_sampled():
    # 16 images 512x512, J = 3 in one call; planes of images 0 and 15 checked
    # against the oracle, reconstruction of all 16.
    log("complex 16x512x512 J=3, sampled")
    M = N = 512
    plan = Plan(M, N, 3, complex_shearlets=True)
    imgs = config2_batch(16)
    x = torch.from_numpy(imgs).to(DEV)
    c = plan.forward(x)
    pp = oracle_plus(M, N, 3)
    for b in (0, 15):
        err = plane_rel_l2(c[b].cpu().numpy(), ocs.forward(imgs[b].astype(np.float64), pp))
        assert err.max() <= TOL, (b, err.max())
    y = plan.adjoint(c).cpu().numpy()
    for b in range(16):
        assert rel_l2(y[b], imgs[b]) <= TOL
    plan.close()


def test_kind_mismatch_is_rejected():
    log("complex/real call mismatch")
    lib = _lib.load()
    real = Plan(16, 16, 2)
    cplx = Plan(16, 16, 2, complex_shearlets=True)
    x = torch.zeros((16, 16), dtype=torch.float32, device=DEV)
    cr = torch.zeros((real.eta, 16, 16), dtype=torch.float32, device=DEV)
    cc = torch.zeros((cplx.eta, 16, 16), dtype=torch.complex64, device=DEV)
    ws = cplx.workspace(1)
    P = ctypes.c_void_p
    assert lib.ffst_forward(P(cplx._h), P(x.data_ptr()), P(cc.data_ptr()), 1, P(ws), None) == _lib.FFST_EINVAL
    assert "complex" in _lib.ffst_last_error()
    assert lib.ffst_adjoint(P(cplx._h), P(cc.data_ptr()), P(x.data_ptr()), 1, P(ws), None) == _lib.FFST_EINVAL
    wr = real.workspace(1)
    assert lib.ffst_forward_complex(P(real._h), P(x.data_ptr()), P(cr.data_ptr()), 1, P(wr), None) == _lib.FFST_EINVAL
    assert lib.ffst_inverse_complex(P(real._h), P(cr.data_ptr()), P(x.data_ptr()), 1, P(wr), None) == _lib.FFST_EINVAL
    with pytest.raises(ValueError):
        cplx.forward(x, out=cr)
    real.close()
    cplx.close()
