"""GPU: the resident kernel (a whole small grid in one workgroup, all steps of
a call in one launch) gives bitwise the state of the one-sweep-per-launch
kernel, alone and inside batches, from the smallest grid (one point per
colour) to the largest that fits one workgroup's LDS."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu

LDS_MAX = 160 * 1024


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def lds_limit():
    import torch

    props = torch.cuda.get_device_properties(0)
    return min(LDS_MAX, getattr(props, "shared_memory_per_block", 64 * 1024))


def tuning(kernel):
    t = kgs.KgsTuning()
    t.kernel = kernel
    t.block = 256
    return t


def run(p, chunks, kernel):
    sim = kgs.simulation_from_problem(p, tuning=tuning(kernel))
    try:
        assert sim.info().kernel == kernel
        for c in chunks:
            sim.step(c)
        return sim.read_state(), sim.energy()
    finally:
        sim.close()


CASES = [
    # dim, n, precision
    (1, 2, workloads.FP64), (1, 4, workloads.FP32), (1, 130, workloads.FP64),
    (1, 256, workloads.FP32), (1, 1030, workloads.FP64), (1, 2050, workloads.FP32),
    (1, 6826, workloads.FP64), (1, 8192, workloads.FP32),
    (2, 2, workloads.FP64), (2, 34, workloads.FP32), (2, 64, workloads.FP64),
    (2, 82, workloads.FP64), (2, 90, workloads.FP32),
    (3, 2, workloads.FP32), (3, 12, workloads.FP64), (3, 16, workloads.FP32),
    (3, 18, workloads.FP64), (3, 20, workloads.FP32),
]


def lds_bytes(dim, n, prec):
    return 6 * (n ** dim // 2) * (8 if prec == workloads.FP64 else 4)


@pytest.mark.parametrize("dim,n,prec", CASES)
def test_resident_equals_sweep_bitwise(dim, n, prec):
    if lds_bytes(dim, n, prec) > lds_limit():
        pytest.skip(f"needs {lds_bytes(dim, n, prec)} bytes of LDS per workgroup")
    p = workloads.random_problem(dim, n, seed=dim * 1000 + n, tau=0.02, amp=0.5, precision=prec)
    say("resident vs sweep", dim, n, prec)
    (a, ea) = run(p, [2, 3], kgs.KGS_KERNEL_RESIDENT)
    (b, eb) = run(p, [5], kgs.KGS_KERNEL_SWEEP)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert ea == eb


def test_resident_is_default_for_small_grids_and_matches_oracle():
    p = workloads.config_1d()
    sim = kgs.simulation_from_problem(p)
    assert sim.info().kernel == kgs.KGS_KERNEL_RESIDENT
    sim.close()
    p = workloads.random_problem(2, 24, seed=5, tau=0.02, amp=0.5)
    say("resident 2-D vs oracle")
    ((psi, u, v), _) = run(p, [30], kgs.KGS_KERNEL_RESIDENT)
    oracle_check.check(p, (psi, u, v), 30)


def test_resident_rejects_grids_that_do_not_fit():
    p = workloads.random_problem(1, 8194, seed=1, precision=workloads.FP32)
    sim = kgs.simulation_from_problem(p)
    assert sim.info().kernel == kgs.KGS_KERNEL_SWEEP
    with pytest.raises(kgs.KgsError):
        sim.tuning = tuning(kgs.KGS_KERNEL_RESIDENT)
    assert sim.info().kernel == kgs.KGS_KERNEL_SWEEP
    sim.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_with_resident_and_sweep_members(graph):
    specs = [(1, 256, 0), (1, 8194, 1), (1, 130, 1), (2, 64, 0), (2, 200, 0), (3, 12, 1),
             (3, 40, 0), (2, 2, 0)]
    probs = [workloads.random_problem(d, n, seed=70 + i, tau=0.02, amp=0.5, precision=pr)
             for i, (d, n, pr) in enumerate(specs)]
    say("batch resident+sweep, graph =", graph)
    ref = []
    for p in probs:
        s = kgs.simulation_from_problem(p, tuning=tuning(kgs.KGS_KERNEL_SWEEP))
        s.step(9)
        ref.append(s.read_state())
        s.close()
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims, graph=graph)
    for _ in range(3):
        b.step(3)  # graph replays with eager reads in between
        sims[0].energy()
    got = [s.read_state() for s in sims]
    b.close()
    for s in sims:
        s.close()
    for g, r in zip(got, ref):
        for x, y in zip(g, r):
            assert np.array_equal(x, y)
    for i, (p, g) in enumerate(zip(probs, got)):
        oracle_check.check(p, g, 9, label=f"member {i} (graph={graph})", cache=True)


def test_batch_step_each_with_resident_members():
    specs = [(1, 256, 0, 5), (1, 300, 1, 0), (2, 40, 0, 8), (2, 130, 1, 3), (3, 14, 0, 1)]
    probs = [workloads.random_problem(d, n, seed=90 + i, tau=0.02, amp=0.5, precision=pr)
             for i, (d, n, pr, _) in enumerate(specs)]
    steps = [k for (_, _, _, k) in specs]
    say("batch step_each with resident members")
    ref = []
    for p, k in zip(probs, steps):
        s = kgs.simulation_from_problem(p, tuning=tuning(kgs.KGS_KERNEL_SWEEP))
        s.step(2 * k)
        ref.append(s.read_state())
        s.close()
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims)
    b.step_each(steps)
    b.step_each(steps)
    got = [s.read_state() for s in sims]
    b.close()
    for s in sims:
        s.close()
    for g, r in zip(got, ref):
        for x, y in zip(g, r):
            assert np.array_equal(x, y)
    for i, (p, g, k) in enumerate(zip(probs, got, steps)):
        oracle_check.check(p, g, 2 * k, label=f"member {i}")
