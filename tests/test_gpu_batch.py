"""Uneven batches (images of several sizes, one HIP graph launch per
direction) and the autotuner, through the C ABI: every image against the
FP64 oracle, graph replays against the eager per-size calls."""

import ctypes

import numpy as np
import pytest
import torch

from oracle import complex_shearlets as ocs
from paper_1202_1773_amd import BatchPlan, Plan, _lib
from paper_1202_1773_amd.synthetic import cartoon, uneven_images, uneven_sizes

from gpu_helpers import log, oracle_forward, per_plane_rel_l2, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-5

SMALL = [(64, 64), (48, 96), (64, 64), (128, 128), (96, 48), (128, 128), (64, 64)]
SMALL_J = [2, 2, 2, 3, 2, 3, 2]


def small_images():
    return [cartoon(m, n, 8, 3, 0.1, seed=900 + b) for b, (m, n) in enumerate(SMALL)]


def eager_reference(bp, imgs, direction, coeffs=None):
    """Per-size Plan calls on the same images, in class order (what the graph
    replays): forward coefficients or adjoint images per image."""
    out = [None] * len(imgs)
    for key in dict.fromkeys(zip(bp.sizes, bp.J)):
        (M, N), J = key
        idx = [b for b in range(len(imgs)) if (bp.sizes[b], bp.J[b]) == key]
        plan = Plan(M, N, J, complex_shearlets=bp.complex_shearlets)
        if direction == "forward":
            x = torch.from_numpy(np.stack([imgs[b] for b in idx])).to(DEV)
            res = plan.forward(x)
        else:
            res = plan.adjoint(torch.stack([coeffs[b] for b in idx]).contiguous())
        for k, b in enumerate(idx):
            out[b] = res[k].clone()
        plan.close()
    return out


def test_small_uneven_batch_graph_replays():
    log("uneven batch of 7 small images: oracle parity and graph replays")
    imgs = small_images()
    bp = BatchPlan(SMALL, SMALL_J)
    assert bp.count == 7 and bp.classes == 4
    f = bp.pack([torch.from_numpy(i) for i in imgs])
    c = bp.forward(f)
    torch.cuda.synchronize()
    first = c.clone()
    views = bp.coefficients(c)
    for b, img in enumerate(imgs):
        M, N = SMALL[b]
        err = per_plane_rel_l2(views[b].cpu().numpy(), oracle_forward(img, M, N, SMALL_J[b]))
        assert err.max() <= TOL, (b, err.max())
    ref = eager_reference(bp, imgs, "forward")
    for b in range(len(imgs)):
        assert torch.equal(views[b], ref[b]), b
    # replays of the captured graph, with eager work and syncs between them
    for rep in range(3):
        junk = torch.randn(1 << 20, device=DEV) * 3.0
        torch.cuda.synchronize()
        c2 = bp.forward(f, out=c)
        torch.cuda.synchronize()
        assert torch.equal(c2, first), rep
        del junk
    # adjoint: reconstruction and equality with the eager per-size adjoint
    y = bp.adjoint(c)
    torch.cuda.synchronize()
    yfirst = y.clone()
    for b, img in enumerate(bp.images(y)):
        assert rel_l2(img.cpu().numpy(), imgs[b]) <= TOL, b
    yref = eager_reference(bp, imgs, "adjoint", coeffs=views)
    for b, img in enumerate(bp.images(y)):
        assert torch.equal(img, yref[b]), b
    for rep in range(3):
        torch.cuda.synchronize()
        y2 = bp.adjoint(c, out=y)
        torch.cuda.synchronize()
        assert torch.equal(y2, yfirst), rep
    # a new output buffer makes a new graph; results are the same
    c3 = bp.forward(f, out=torch.empty_like(c))
    assert torch.equal(c3, first)
    bp.close()


def test_complex_uneven_batch():
    log("complex uneven batch")
    sizes = [(64, 64), (96, 48), (64, 64)]
    imgs = [cartoon(m, n, 8, 3, 0.1, seed=950 + b) for b, (m, n) in enumerate(sizes)]
    bp = BatchPlan(sizes, 2, complex_shearlets=True)
    c = bp.forward(bp.pack([torch.from_numpy(i) for i in imgs]))
    assert c.dtype == torch.complex64
    for b, (M, N) in enumerate(sizes):
        pp = ocs.one_sided_spectra(M, N, 2)
        ref = ocs.forward(imgs[b].astype(np.float64), pp)
        got = bp.coefficients(c)[b].cpu().numpy()
        num = np.sqrt((np.abs(got - ref) ** 2).sum(axis=(-2, -1)))
        den = np.sqrt((np.abs(ref) ** 2).sum(axis=(-2, -1)))
        assert (num / np.where(den > 0, den, 1)).max() <= TOL
    y = bp.adjoint(c)
    for b, img in enumerate(bp.images(y)):
        assert rel_l2(img.cpu().numpy(), imgs[b]) <= TOL
    bp.close()


def test_uneven_batch_odd_and_27_sides():
    log("uneven batch with odd widths and sides with a factor 27")
    sizes = [(27, 54), (81, 9), (27, 54), (243, 64), (9, 9), (108, 81)]
    Js = [2, 2, 2, 3, 1, 3]
    imgs = [cartoon(m, n, 8, 3, 0.1, seed=980 + b) for b, (m, n) in enumerate(sizes)]
    bp = BatchPlan(sizes, Js)
    assert bp.classes == 5
    f = bp.pack([torch.from_numpy(i) for i in imgs])
    c = bp.forward(f)
    views = bp.coefficients(c)
    for b, (M, N) in enumerate(sizes):
        err = per_plane_rel_l2(views[b].cpu().numpy(), oracle_forward(imgs[b], M, N, Js[b]))
        assert err.max() <= TOL, (b, err.max())
    y = bp.adjoint(c)
    for b, img in enumerate(bp.images(y)):
        assert rel_l2(img.cpu().numpy(), imgs[b]) <= TOL, b
    bp.close()


@pytest.mark.timeout(400)
@pytest.mark.parametrize("tuned", [False, True])
def test_uneven_workload_64_images(tuned):
    # the uneven workload: 64 images drawn from 256^2 .. 1024^2 (seed 401),
    # J = 3 up to 512, else 4; one image per size checked on sampled planes,
    # reconstruction of all 64; with the built-in launch settings and after
    # the batch autotuner (the settings the benchmark times)
    log(f"uneven workload, 64 images, tuned={tuned}")
    sizes, Js = uneven_sizes()
    imgs = uneven_images(sizes)
    bp = BatchPlan(sizes, Js)
    assert bp.classes == 5
    f = bp.pack([torch.from_numpy(i) for i in imgs])
    if tuned:
        bp.tune(f)
        log(f"  class settings {bp.class_tuning()}")
    c = bp.forward(f)
    views = bp.coefficients(c)
    done = set()
    for b, (M, N) in enumerate(sizes):
        if (M, N) in done:
            continue
        done.add((M, N))
        eta = bp.etas[b]
        planes = sorted({0, 1, eta // 3, eta // 2, eta - 1})
        ref = oracle_forward(imgs[b], M, N, Js[b], planes=planes)
        err = per_plane_rel_l2(views[b][planes].cpu().numpy(), ref)
        log(f"  {M}x{N} J={Js[b]} sampled max plane relL2 {err.max():.2e}")
        assert err.max() <= TOL
    y = bp.adjoint(c)
    for b, img in enumerate(bp.images(y)):
        assert rel_l2(img.cpu().numpy(), imgs[b]) <= TOL, b
    bp.close()


def test_autotuner():
    log("autotuner: single plan and uneven batch")
    M = N = 128
    plan = Plan(M, N, 3)
    x = torch.from_numpy(np.stack([cartoon(M, N, 8, 3, 0.1, seed=70 + b) for b in range(4)])).to(DEV)
    c0 = plan.forward(x)
    best = plan.tune(x)
    t = plan.tuning_ex()
    log(f"  best {best:.4f} ms at {t}")
    assert best > 0 and 1 <= t["nparts"] <= 8 and t["blocks_per_cu"] in (0, 1, 2, 4, 8, 16)
    assert t["col_values"] in (8, 16) and t["row_block"] in (1, 2) and 1 <= t["fwd_nparts"] <= 8
    c1 = plan.forward(x)
    # the forward does not depend on the splits, blocks per CU or the row
    # block height; another column lane width only changes the rounding order
    if t["col_values"] == 8:
        assert torch.equal(c0, c1)
    assert rel_l2(c1.cpu().numpy(), c0.cpu().numpy()) <= 1e-6
    assert rel_l2(plan.adjoint(c1).cpu().numpy(), x.cpu().numpy()) <= TOL
    plan.set_tuning(0, 0)
    assert plan.tuning() == (0, 0)
    assert plan.tuning_ex() == {"nparts": 0, "blocks_per_cu": 0, "col_values": 8, "row_block": 1, "fwd_nparts": 0}
    plan.close()
    imgs = small_images()
    bp = BatchPlan(SMALL, SMALL_J)
    f = bp.pack([torch.from_numpy(i) for i in imgs])
    bp.tune(f)
    # the classes keep their tuned settings only if the whole batch got
    # faster with them; otherwise every class is back at the defaults
    tuned = bp.class_tuning()
    log(f"  batch class settings {tuned}")
    defaults = all(t["nparts"] == 0 and t["blocks_per_cu"] == 0 and t["row_block"] == 1 and t["fwd_nparts"] == 0
                   for t in tuned)
    assert defaults or all(1 <= t["nparts"] <= 8 and t["blocks_per_cu"] in (0, 1, 2, 4, 8, 16)
                           and 1 <= t["fwd_nparts"] <= 8 for t in tuned)
    y = bp.adjoint(bp.forward(f))
    for b, img in enumerate(bp.images(y)):
        assert rel_l2(img.cpu().numpy(), imgs[b]) <= TOL
    bp.close()


def test_batch_argument_checks():
    log("uneven batch argument checks")
    lib = _lib.load()
    bp = BatchPlan([(16, 16), (32, 32)], 2)
    P = ctypes.c_void_p
    f = bp.empty_images()
    c = bp.empty_coefficients()
    ws = bp.workspace()
    assert lib.ffst_batch_forward(P(bp._h), P(f.data_ptr()), P(f.data_ptr()), P(ws), None) == _lib.FFST_EINVAL
    assert lib.ffst_batch_forward(P(bp._h), P(f.data_ptr()), P(c.data_ptr()), P(ws + 8), None) == _lib.FFST_EINVAL
    assert lib.ffst_batch_forward(P(bp._h), None, P(c.data_ptr()), P(ws), None) == _lib.FFST_EINVAL
    with pytest.raises(ValueError):
        bp.forward(f[:-1])
    bp.close()


def test_graphs_of_several_output_buffers_are_kept():
    # Alternating between output buffers (and fresh outputs from the binding)
    # replays the graphs kept for each (input, output, workspace) triple; every
    # result equals the first.
    log("uneven batch: graphs of several output buffers")
    imgs = small_images()
    bp = BatchPlan(SMALL, SMALL_J)
    f = bp.pack([torch.from_numpy(i) for i in imgs])
    outs = [bp.empty_coefficients() for _ in range(3)]
    first = bp.forward(f, out=outs[0]).clone()
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
            torch.cuda.synchronize()
            assert torch.equal(bp.forward(f, out=o), first), rep
    fresh = [bp.forward(f) for _ in range(10)]   # more triples than the cache holds
    torch.cuda.synchronize()
    for c in fresh:
        assert torch.equal(c, first)
    ys = [bp.adjoint(first) for _ in range(3)]
    torch.cuda.synchronize()
    assert torch.equal(ys[0], ys[1]) and torch.equal(ys[1], ys[2])
    bp.close()
