"""Allocation failures during plan and batch creation (GPU only).

With FFST_FAULT_ALLOC=n the n-th device allocation inside one creation call
fails as if the device were out of memory; the call must return FFST_ENOMEM
and release everything it had allocated (ffst_device_bytes back to its value
before the call). n runs from 1 until creation succeeds, so every allocation
of the path, and every cleanup path behind it, is exercised once. Nothing is
launched after a failed allocation, so no kernel sees a partial plan.
"""

import os

import pytest
import torch

from paper_1202_1773_amd import _lib

from gpu_helpers import log

pytestmark = pytest.mark.gpu


def _sweep(create, destroy, what):
    torch.cuda.init()
    before = _lib.ffst_device_bytes()
    failures = 0
    try:
        for n in range(1, 200):
            os.environ["FFST_FAULT_ALLOC"] = str(n)
            try:
                h = create()
            except _lib.FfstError as e:
                assert e.status == _lib.FFST_ENOMEM, (what, n, str(e))
                assert _lib.ffst_device_bytes() == before, (what, n)
                failures += 1
                continue
            os.environ.pop("FFST_FAULT_ALLOC", None)
            assert _lib.ffst_device_bytes() > before
            destroy(h)
            assert _lib.ffst_device_bytes() == before
            break
        else:
            pytest.fail(f"{what}: creation never succeeded")
    finally:
        os.environ.pop("FFST_FAULT_ALLOC", None)
    log(f"  {what}: {failures} injected failures, no device memory left behind")
    assert failures >= 3


@pytest.mark.parametrize("complex_shearlets", [False, True])
def test_plan_creation_releases_memory_on_every_failure(complex_shearlets):
    log(f"allocation faults in ffst_spectra_ex, 64x96 J=2, complex={complex_shearlets}")
    _sweep(lambda: _lib.ffst_spectra(64, 96, 2, complex_shearlets=complex_shearlets), _lib.ffst_destroy,
           f"plan complex={complex_shearlets}")


def test_batch_creation_releases_memory_on_every_failure():
    log("allocation faults in ffst_batch_create, 3 classes")
    sizes = [(64, 64), (32, 48), (64, 64), (96, 64)]
    _sweep(lambda: _lib.ffst_batch_create([m for m, _ in sizes], [n for _, n in sizes], [2, 1, 2, 2]),
           _lib.ffst_batch_destroy, "batch")


def test_plan_after_injected_failures_still_works():
    # a plan created after the sweep computes what a fresh one computes
    import numpy as np
    from paper_1202_1773_amd import Plan
    x = torch.randn(64, 64, device="cuda")
    os.environ["FFST_FAULT_ALLOC"] = "2"
    try:
        with pytest.raises(_lib.FfstError):
            Plan(64, 64, 2)
    finally:
        os.environ.pop("FFST_FAULT_ALLOC", None)
    p = Plan(64, 64, 2)
    y = p.adjoint(p.forward(x))
    assert float(torch.linalg.norm(y - x) / torch.linalg.norm(x)) <= 1e-5
    p.close()
    assert np.isfinite(_lib.ffst_device_bytes())
