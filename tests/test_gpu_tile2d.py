"""GPU: the 2-D tiled kernel (a tile plus halo of both colours in LDS, 1, 2 or 4
DP-AVF2 steps per launch, ping-pong buffers) gives bitwise the state of the
one-sweep-per-launch kernel for tiles that divide the grid, ragged edge
tiles, tiles wider or taller than the grid, every points-per-thread class,
and matches the oracle."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def tuning(kernel, ty=32, tx=16, spl=2):
    t = kgs.KgsTuning()
    t.kernel = kernel
    t.block = 256
    t.tile_y, t.tile_x, t.steps_per_launch = ty, tx, spl
    t.chunk = 16
    return t


def run(p, calls, t):
    sim = kgs.simulation_from_problem(p, tuning=t)
    try:
        assert sim.info().kernel == t.kernel
        for c in calls:
            sim.step(c)
        return sim.read_state(), sim.energy()
    finally:
        sim.close()


CASES = [
    # n, tile rows, tile points of one colour, steps per launch, step calls
    (2, 1, 1, 2, [3]),          # tile and halo wrap around a 2x2 grid
    (4, 3, 1, 1, [2, 1]),
    (30, 7, 5, 2, [5]),         # ragged in both directions
    (64, 32, 16, 2, [3, 4]),    # 256 threads, 2 points each
    (64, 16, 16, 1, [3]),
    (130, 32, 16, 2, [3]),      # odd number of points per row and colour
    (250, 48, 24, 2, [2, 3]),   # 256 threads, 4 points each
    (256, 40, 32, 2, [5]),      # 1584-point block: 512 threads, 4 points each
    (256, 64, 32, 2, [2]),      # too many points for one workgroup: rejected
    (1024, 32, 16, 2, [3]),
    # 4 steps (8 sweeps) per launch: 8 halo rows, 4 compressed positions
    (2, 1, 1, 4, [6]),
    (30, 7, 5, 4, [5]),         # one launch of 4 steps, then 1
    (64, 16, 16, 4, [4, 3]),    # the tail of a call: 2 steps, then 1
    (130, 32, 16, 4, [9]),
    (256, 24, 24, 4, [8]),
]


@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
@pytest.mark.parametrize("n,ty,tx,spl,calls", CASES)
def test_tile2d_equals_sweep_bitwise(n, ty, tx, spl, calls, prec):
    p = workloads.random_problem(2, n, seed=700 + n + ty, tau=0.02, amp=0.5, precision=prec)
    say("tile2d vs sweep", n, ty, tx, spl, calls, prec)
    sim = kgs.simulation_from_problem(p)
    try:
        sim.tuning = tuning(kgs.KGS_KERNEL_TILE, ty, tx, spl)
    except kgs.KgsError:
        # the block does not fit one workgroup (LDS or points per thread)
        assert (ty + 4 * spl) * (tx + 2 * spl) > 2048 or \
            6 * (ty + 4 * spl) * (tx + 2 * spl) * (8 if prec == workloads.FP64 else 4) > 160 * 1024
        sim.close()
        return
    sim.close()
    (a, ea) = run(p, calls, tuning(kgs.KGS_KERNEL_TILE, ty, tx, spl))
    (b, eb) = run(p, [sum(calls)], tuning(kgs.KGS_KERNEL_SWEEP))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert ea == eb


def test_tile2d_matches_oracle():
    p = workloads.config_2d(n=160, steps=60)
    say("tile2d vs oracle")
    ((psi, u, v), _) = run(p, [p.steps], tuning(kgs.KGS_KERNEL_TILE, 32, 16, 2))
    oracle_check.check(p, (psi, u, v), p.steps)


def test_tile2d_rejects_bad_shapes():
    p = workloads.random_problem(2, 64, seed=1)
    sim = kgs.simulation_from_problem(p)
    for bad in (tuning(kgs.KGS_KERNEL_TILE, 0, 16, 2), tuning(kgs.KGS_KERNEL_TILE, 16, 0, 2),
                tuning(kgs.KGS_KERNEL_TILE, 16, 16, 3), tuning(kgs.KGS_KERNEL_TILE, 200, 100, 2)):
        with pytest.raises(kgs.KgsError):
            sim.tuning = bad
    sim.close()
    for dim in (1, 3):
        q = workloads.random_problem(dim, 8, seed=1)
        sim = kgs.simulation_from_problem(q)
        with pytest.raises(kgs.KgsError):
            sim.tuning = tuning(kgs.KGS_KERNEL_TILE, 4, 4, 1)
        sim.close()


def test_autotune_2d_keeps_state_and_results():
    # the 2-D candidates (sweeps, y-streaming chunks, tiles) all give the
    # same state; tuning leaves the state as it was
    p = workloads.random_problem(2, 200, seed=9, tau=0.02, amp=0.5)
    say("2-D autotune")
    sim = kgs.simulation_from_problem(p)
    before = sim.read_state()
    best = sim.autotune(steps=2, use_cache=False)
    for x, y in zip(before, sim.read_state()):
        assert np.array_equal(x, y)
    assert best.kernel in (kgs.KGS_KERNEL_SWEEP, kgs.KGS_KERNEL_STREAM, kgs.KGS_KERNEL_TILE)
    assert sim.tuning.kernel == best.kernel
    sim.step(3)
    tuned = sim.read_state()
    sim.close()
    (ref, _) = run(p, [3], tuning(kgs.KGS_KERNEL_SWEEP))
    for x, y in zip(tuned, ref):
        assert np.array_equal(x, y)
