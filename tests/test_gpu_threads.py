"""Several host threads using the library at once, as a serving process
would: each thread owns a plan (or shares one with its own workspace) and a
stream of its own, and runs forward + adjoint repeatedly. Every result must
equal, bit for bit, the same call made alone on one thread."""

import threading

import numpy as np
import pytest
import torch

from paper_1202_1773_amd import Plan
from paper_1202_1773_amd.synthetic import cartoon

from gpu_helpers import log

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _images(M, N, B, seed):
    return torch.from_numpy(np.stack([cartoon(M, N, 8, 3, 0.1, seed=seed + b) for b in range(B)])).to(DEV)


def _worker(plan, x, ws, reps, results, errors, key):
    try:
        stream = torch.cuda.Stream(device=DEV)  # default priority
        outs = []
        with torch.cuda.stream(stream):
            for _ in range(reps):
                c = plan.forward(x, ws=ws)
                y = plan.adjoint(c, ws=ws)
                outs.append((c, y))
        stream.synchronize()
        results[key] = outs
    except Exception as e:  # reported by the main thread
        errors.append(repr(e))


def test_threads_own_plans_and_shared_plan():
    log("4 host threads: two own plans, two share a plan with separate workspaces")
    cases = {"a": (128, 128, 3, 4, 10), "b": (96, 192, 2, 3, 20)}
    plans = {k: Plan(M, N, J) for k, (M, N, J, B, s) in cases.items()}
    shared = Plan(64, 64, 2)
    inputs = {k: _images(M, N, B, s) for k, (M, N, J, B, s) in cases.items()}
    inputs["s1"] = _images(64, 64, 2, 30)
    inputs["s2"] = _images(64, 64, 2, 40)
    plan_of = {"a": plans["a"], "b": plans["b"], "s1": shared, "s2": shared}
    # reference: each call alone, on the default stream
    ref = {}
    for k, plan in plan_of.items():
        c = plan.forward(inputs[k])
        ref[k] = (c, plan.adjoint(c))
    torch.cuda.synchronize()
    # separate workspaces for the threads (the shared plan's calls run at the
    # same time, so they must not share one)
    ws_bufs = {}
    for k, plan in plan_of.items():
        n = plan.workspace_size(inputs[k].shape[0])
        buf = torch.empty(n + 256, dtype=torch.uint8, device=DEV)
        ws_bufs[k] = (buf, buf.data_ptr() + (-buf.data_ptr()) % 256)
    results, errors = {}, []
    threads = [threading.Thread(target=_worker, args=(plan_of[k], inputs[k], ws_bufs[k][1], 5, results, errors, k))
               for k in plan_of]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a worker thread did not finish"
    assert not errors, errors
    for k in plan_of:
        for rep, (c, y) in enumerate(results[k]):
            assert torch.equal(c, ref[k][0]), (k, rep)
            assert torch.equal(y, ref[k][1]), (k, rep)
    for p in list(plans.values()) + [shared]:
        p.close()
