"""ffst_forward_noalloc (GPU only): the forward transform with its workspace
in the library's static device scratch, through the C ABI, against
ffst_forward with a caller workspace (same kernels: bitwise equal) and the
FP64 oracle; two calls in a row, the second with a smaller input, and the
rejection of a batch whose workspace exceeds the static scratch."""

import numpy as np
import pytest
import torch

from paper_1202_1773_amd import Plan, _lib
from paper_1202_1773_amd.synthetic import cartoon

from gpu_helpers import log, oracle_forward, per_plane_rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
LIMIT = 64 << 20


def _call(plan, x, out):
    _lib.ffst_forward_noalloc(plan._h, x.data_ptr(), out.data_ptr(), x.shape[0],
                              torch.cuda.current_stream(DEV).cuda_stream)


def test_forward_noalloc_two_calls_second_smaller():
    results = []
    for (M, N, J, B) in [(256, 256, 3, 3), (128, 96, 2, 1)]:
        log(f"ffst_forward_noalloc {M}x{N} J={J} B={B}")
        plan = Plan(M, N, J)
        assert plan.workspace_size(B) <= LIMIT
        imgs = np.stack([cartoon(M, N, 10, 4, 0.1, seed=70 + b + M) for b in range(B)])
        x = torch.from_numpy(imgs).to(DEV)
        ref = plan.forward(x)
        out = torch.full_like(ref, float("nan"))
        held = _lib.ffst_device_bytes()
        torch.cuda.synchronize()
        _call(plan, x, out)
        torch.cuda.synchronize()
        assert _lib.ffst_device_bytes() == held
        assert torch.equal(out, ref)
        err = per_plane_rel_l2(out[0].cpu().numpy(), oracle_forward(imgs[0], M, N, J))
        assert err.max() <= 1e-5
        results.append((plan, x, out.clone()))
    # the first plan again after the smaller call: the scratch kept the second
    # call's contents, the result must not depend on them
    plan, x, first = results[0]
    out = torch.full_like(first, float("nan"))
    _call(plan, x, out)
    torch.cuda.synchronize()
    assert torch.equal(out, first)
    for plan, _, _ in results:
        plan.close()


def test_forward_noalloc_rejects_batches_beyond_the_scratch():
    plan = Plan(512, 512, 3)
    B = 1
    while plan.workspace_size(B) <= LIMIT:
        B += 1
    x = torch.zeros((B, 512, 512), device=DEV)
    out = torch.full((B, plan.eta, 512, 512), 7.0, device=DEV)
    with pytest.raises(_lib.FfstError) as e:
        _call(plan, x, out)
    assert e.value.status == _lib.FFST_EINVAL
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())        # nothing ran
    # the largest batch that fits runs
    y = torch.from_numpy(np.stack([cartoon(512, 512, 8, 3, 0.1, seed=90 + b) for b in range(B - 1)])).to(DEV)
    got = torch.empty((B - 1, plan.eta, 512, 512), device=DEV)
    _call(plan, y, got)
    assert torch.equal(got, plan.forward(y))
    plan.close()
