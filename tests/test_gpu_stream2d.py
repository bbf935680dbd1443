"""GPU: the 2-D streaming kernel (one wave per tile of 64 lanes streaming
along y, 1 or 2 DP-AVF2 steps per launch, ping-pong buffers) gives bitwise
the state of the one-sweep-per-launch kernel, for rows that fit one wave
(periodic lanes) and rows split into tiles with halos, and matches the
oracle."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def tuning(kernel, chunk=16, spl=2):
    t = kgs.KgsTuning()
    t.kernel = kernel
    t.block = 256
    t.chunk, t.steps_per_launch = chunk, spl
    return t


def run(p, chunks, t):
    sim = kgs.simulation_from_problem(p, tuning=t)
    try:
        assert sim.info().kernel == t.kernel
        for c in chunks:
            sim.step(c)
        return sim.read_state(), sim.energy()
    finally:
        sim.close()


CASES = [
    # n, chunk, steps per launch, step calls
    (2, 1, 2, [3]), (4, 3, 1, [2, 1]), (30, 7, 2, [5]), (128, 16, 2, [3, 4]),
    (130, 5, 2, [3]), (130, 64, 1, [4]), (250, 13, 2, [2, 3]), (256, 1000, 2, [5]),
    (1024, 64, 2, [3]),
]


@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
@pytest.mark.parametrize("n,chunk,spl,calls", CASES)
def test_stream2d_equals_sweep_bitwise(n, chunk, spl, calls, prec):
    p = workloads.random_problem(2, n, seed=300 + n + chunk, tau=0.02, amp=0.5, precision=prec)
    say("stream2d vs sweep", n, chunk, spl, calls, prec)
    (a, ea) = run(p, calls, tuning(kgs.KGS_KERNEL_STREAM, chunk, spl))
    (b, eb) = run(p, [sum(calls)], tuning(kgs.KGS_KERNEL_SWEEP))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert ea == eb


def test_stream2d_matches_oracle():
    p = workloads.config_2d(n=160, steps=60)
    say("stream2d vs oracle")
    ((psi, u, v), _) = run(p, [p.steps], tuning(kgs.KGS_KERNEL_STREAM, 32, 2))
    oracle_check.check(p, (psi, u, v), p.steps)


def test_stream2d_rejects_bad_shapes():
    p = workloads.random_problem(2, 64, seed=1)
    sim = kgs.simulation_from_problem(p)
    for bad in (tuning(kgs.KGS_KERNEL_STREAM, 0, 2), tuning(kgs.KGS_KERNEL_STREAM, 8, 3)):
        with pytest.raises(kgs.KgsError):
            sim.tuning = bad
    sim.close()
    p1 = workloads.random_problem(1, 64, seed=1)
    sim = kgs.simulation_from_problem(p1)
    with pytest.raises(kgs.KgsError):
        sim.tuning = tuning(kgs.KGS_KERNEL_STREAM, 8, 2)
    sim.close()
