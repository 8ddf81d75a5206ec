"""Every launch-shape variant the autotuner can pick (ffst_tuning in
include/ffst.h), against the FP64 oracle: the default and the alternative
values per lane of the column FFTs, default and doubled row blocks, and both
forms of the adjoint's sum over spectra (nparts = 1 and 4), and the forward's
column pass with a column's spectra on 1, 3 and 8 lines (bitwise the same
coefficients: every spectrum line is computed once, by the same code, whatever
the split). Sizes cover every
alternative lane width (16 and 8 for powers of two, 6 for 3 * 2^k, with
groups inside one wave and groups spanning several waves) and the doubled
row blocks of short, medium and the longest rows. Forward: relative L2 per
coefficient plane; adjoint: random N(0, 1) coefficients (outside the range
of the forward map); both within 1e-5."""

import numpy as np
import pytest
import torch

from paper_1202_1773_amd import Plan, _lib
from paper_1202_1773_amd.synthetic import cartoon

from gpu_helpers import log, oracle_adjoint, oracle_forward, per_plane_rel_l2, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = 1e-5

# (M, N, J, alternative col_values, row_block 2 available)
CASES = [(512, 512, 3, 16, True), (384, 768, 3, 6, True), (1024, 256, 4, 8, True), (96, 2048, 3, 6, True),
         (64, 4096, 2, 16, True), (3072, 64, 2, 6, True), (4096, 32, 2, 8, False), (192, 24, 2, 6, False)]


@pytest.mark.parametrize("M,N,J,alt,rb2", CASES)
def test_every_launch_shape_matches_the_oracle(M, N, J, alt, rb2):
    log(f"launch-shape variants {M}x{N} J={J}")
    plan = Plan(M, N, J)
    f = cartoon(M, N, 10, 4, 0.1, seed=M + 3 * N)
    x = torch.from_numpy(f).to(DEV)
    ref_f = oracle_forward(f, M, N, J)
    g = torch.Generator(device=DEV).manual_seed(M * N)
    r = torch.randn((plan.eta, M, N), device=DEV, generator=g)
    ref_a = oracle_adjoint(r.cpu().numpy(), M, N, J)
    shapes = [(0, 0), (alt, 0)] + ([(0, 2), (alt, 2)] if rb2 else [])
    for col_values, row_block in shapes:
        c_first = None
        for nparts, fwd_nparts in ((1, 1), (4, 3), (1, 8)):
            plan.set_tuning(nparts, 0, col_values, row_block, fwd_nparts)
            t = plan.tuning_ex()
            assert t["row_block"] == (2 if row_block == 2 else 1) and t["fwd_nparts"] == fwd_nparts
            if col_values:
                assert t["col_values"] == col_values
            c = plan.forward(x)
            if c_first is None:
                c_first = c
            assert torch.equal(c, c_first), t
            e_f = per_plane_rel_l2(c.cpu().numpy(), ref_f).max()
            e_a = rel_l2(plan.adjoint(r).cpu().numpy(), ref_a)
            log(f"  {t}: forward {e_f:.2e} adjoint {e_a:.2e}")
            assert e_f <= TOL and e_a <= TOL, (t, e_f, e_a)
    plan.close()


def test_tuning_rejects_shapes_that_are_not_compiled():
    plan = Plan(512, 512, 3)
    with pytest.raises(_lib.FfstError) as e:
        plan.set_tuning(0, 0, col_values=12)
    assert e.value.status == _lib.FFST_EINVAL
    for bad in (-1, 9):
        with pytest.raises(_lib.FfstError) as e:
            plan.set_tuning(0, 0, fwd_nparts=bad)
        assert e.value.status == _lib.FFST_EINVAL
    plan.close()
    plan = Plan(64, 16, 1)          # row length 16: no doubled row blocks
    with pytest.raises(_lib.FfstError):
        plan.set_tuning(0, 0, row_block=2)
    plan.set_tuning(0, 0, row_block=1)
    plan.close()
