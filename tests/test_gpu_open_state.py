"""GPU: kgs_step may leave the adjoint red sweep that closes its last step
pending (Algorithm 3: a step ends with the adjoint half's red points); the
next call fuses it with its first red sweep and every call that reads or
replaces the state applies it first.  Whatever a caller observes must be
bitwise the state of one uninterrupted run, across kernels, tunings, energy
evaluations, writes and autotuning."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def tun(kernel, **kw):
    t = kgs.KgsTuning()
    t.kernel = kernel
    t.block = 256
    for k, v in kw.items():
        setattr(t, k, v)
    return t


SWEEP = tun(kgs.KGS_KERNEL_SWEEP)
STREAM3 = tun(kgs.KGS_KERNEL_STREAM, tile_x=16, tile_y=16, chunk=16, steps_per_launch=2)
STREAM3_1 = tun(kgs.KGS_KERNEL_STREAM, tile_x=8, tile_y=8, chunk=8, steps_per_launch=1)
TILE2 = tun(kgs.KGS_KERNEL_TILE, tile_x=16, tile_y=16, steps_per_launch=2)
STREAM2 = tun(kgs.KGS_KERNEL_STREAM, chunk=16, steps_per_launch=2)
RESIDENT = tun(kgs.KGS_KERNEL_RESIDENT)


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def straight(p, steps):
    s = kgs.simulation_from_problem(p)
    s.step(steps)
    out = s.read_state()
    s.close()
    return out


@pytest.mark.parametrize("dim,n,tunings", [
    (3, 40, [STREAM3, SWEEP, STREAM3_1, STREAM3]),
    (3, 12, [RESIDENT, STREAM3_1, RESIDENT, SWEEP]),
    (2, 130, [TILE2, STREAM2, SWEEP, TILE2]),
    (2, 40, [STREAM2, RESIDENT, TILE2, RESIDENT]),
])
@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
def test_calls_across_kernels_equal_one_run(dim, n, tunings, prec):
    p = workloads.random_problem(dim, n, seed=90 + n, tau=0.03, amp=0.5, precision=prec)
    counts = [3, 2, 1, 4]
    say("open state across kernels", dim, n, prec)
    s = kgs.simulation_from_problem(p)
    for t, k in zip(tunings, counts):
        s.tuning = t
        s.step(k)
    got = s.read_state()
    s.close()
    assert same(got, straight(p, sum(counts)))
    oracle_check.check(p, got, sum(counts), label=f"open state {dim}-D n={n}", cache=True)


def test_energy_and_reads_in_the_middle_of_a_run():
    p = workloads.random_problem(3, 96, seed=5, tau=0.02, amp=0.5)
    say("energy / read between calls")
    s = kgs.simulation_from_problem(p)
    assert s.tuning.kernel == kgs.KGS_KERNEL_STREAM
    s.step(3)
    e3 = s.energy()
    mid = s.read_state()
    s.step(4)
    got = s.read_state()
    e7 = s.energy()
    s.close()
    assert same(mid, straight(p, 3))
    assert same(got, straight(p, 7))
    r = kgs.simulation_from_problem(p)
    r.step(3)
    assert r.energy() == e3
    r.step(4)
    assert r.energy() == e7
    r.close()


def test_write_state_replaces_an_open_state():
    p = workloads.random_problem(3, 96, seed=6, tau=0.02, amp=0.5)
    q = workloads.random_problem(3, 96, seed=7, tau=0.02, amp=0.5)
    say("write over an open state")
    s = kgs.simulation_from_problem(p)
    s.step(3)  # leaves the closing sweep pending
    s.write_state(q.psi, q.u, q.v)
    s.step(2)
    got = s.read_state()
    s.close()
    # the handle keeps p's parameters; only the fields are q's
    assert same(got, straight(dataclasses.replace(p, psi=q.psi, u=q.u, v=q.v), 2))


def test_autotune_on_an_open_state_keeps_it():
    p = workloads.random_problem(3, 64, seed=8, tau=0.02, amp=0.5)
    say("autotune after an open step")
    s = kgs.simulation_from_problem(p)
    s.tuning = STREAM3
    s.step(3)
    s.autotune(steps=2, use_cache=False)
    s.step(4)
    got = s.read_state()
    s.close()
    assert same(got, straight(p, 7))


def test_sync_completes_the_steps():
    # kgs_sync applies the pending closing sweep: a run of calls with syncs
    # in between ends where one uninterrupted run does
    p = workloads.random_problem(3, 96, seed=10, tau=0.02, amp=0.5)
    say("sync between calls")
    s = kgs.simulation_from_problem(p)
    for k in (3, 2, 4):
        s.step(k)
        s.sync()
    got = s.read_state()
    s.close()
    assert same(got, straight(p, 9))


def test_repeated_calls_as_in_the_bench():
    # the bench times repeated calls of K steps followed by one energy
    p = workloads.random_problem(3, 96, seed=9, tau=0.02, amp=0.5)
    say("repeated K-step calls + energy")
    s = kgs.simulation_from_problem(p)
    energies = []
    for _ in range(3):
        s.step(4)
        energies.append(s.energy())
    got = s.read_state()
    s.close()
    assert same(got, straight(p, 12))
    r = kgs.simulation_from_problem(p)
    for i in range(3):
        r.step(4)
        assert r.energy() == energies[i]
    r.close()


@pytest.mark.parametrize("dim,n", [(3, 96), (3, 34), (2, 130), (2, 2050)])
@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
def test_energy_that_closes_the_step_equals_sweep_then_energy(dim, n, prec):
    # kgs_energy on an open state applies the closing sweep in its own pass;
    # reading the state first closes it with the sweep kernel instead
    p = workloads.random_problem(dim, n, seed=70 + n, tau=0.02, amp=0.5, precision=prec)
    say("closing energy", dim, n, prec)
    a = kgs.simulation_from_problem(p)
    b = kgs.simulation_from_problem(p)
    for x in (a, b):
        x.tuning = STREAM3 if dim == 3 else TILE2
        x.step(3)
    ea = a.energy()          # fused: closing sweep + energy
    sa = a.read_state()
    sb = b.read_state()      # closing sweep alone
    eb = b.energy()          # energy of the closed state
    a.close()
    b.close()
    assert same(sa, sb)
    assert ea == eb
    oracle_check.check(p, sa, 3, label=f"closing energy {dim}-D n={n}", cache=True)
    # the energy of the GPU's own final state, by the oracle's definition
    psi, u, v = sa
    ref = oracle.energy(oracle_check.grid_of(p), oracle.State.from_fields(psi, u, v))
    assert abs(ea - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("dim,n", [(1, 8192), (2, 2), (2, 6), (3, 2), (3, 4), (3, 10)])
@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
def test_closing_energy_on_small_and_1d_grids(dim, n, prec):
    # one colour sweep per launch: n = 2 (each neighbour along an axis is
    # the same point twice), odd chunkings of tiny planes, and 1-D grids,
    # whose energy closes the step with the sweep kernel first
    p = workloads.random_problem(dim, n, seed=80 + n + dim, tau=0.02, amp=0.5, precision=prec)
    say("closing energy, sweeps", dim, n, prec)
    a = kgs.simulation_from_problem(p, tuning=SWEEP)
    b = kgs.simulation_from_problem(p, tuning=SWEEP)
    a.step(3)
    b.step(3)
    ea = a.energy()
    sa = a.read_state()
    sb = b.read_state()
    eb = b.energy()
    a.close()
    b.close()
    assert same(sa, sb)
    assert ea == eb
    oracle_check.check(p, sa, 3, label=f"closing energy (sweeps) {dim}-D n={n}", cache=True)
    psi, u, v = sa
    ref = oracle.energy(oracle_check.grid_of(p), oracle.State.from_fields(psi, u, v))
    assert abs(ea - ref) <= 1e-13 * abs(ref)
