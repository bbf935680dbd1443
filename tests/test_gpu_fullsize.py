"""GPU, full sizes in the launch configurations bench.py times.

After 4 steps of a 3-D 256^3 grid, samples are checked against the oracle
run on sub-blocks (an output depends only on points at most 2K+1 away).
After 200 steps the cone covers the whole grid, so that run is checked by
properties that hold at any size: the discrete energy is conserved, and the
symmetric composition is time-reversible (200 steps with -tau return to the
initial state).  The batched configuration (64 uneven 2-D grids x 500 steps)
is checked member by member against runs of the same grids alone, and its
members up to n = 256 against the oracle over all 500 steps."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_3d_256_200_steps_conserves_energy_and_reverses():
    import torch

    p = workloads.config_3d()  # 256^3, tau = 0.002, 200 steps, float64
    say("3-D 256^3 x 200 steps forward and back")
    sim = kgs.simulation_from_problem(p)
    assert sim.info().kernel == kgs.KGS_KERNEL_STREAM
    e0 = sim.energy()
    sim.step(p.steps)
    e1 = sim.energy()
    assert abs(e1 - e0) <= 1e-12 * abs(e0), (e0, e1)
    psi, u, v = sim.read_state(as_torch=True)
    sim.close()
    back = kgs.Simulation(kgs.config_of(p.with_(tau=-p.tau)), psi, u, v)
    del psi, u, v
    back.step(p.steps)
    psi0, u0, v0 = back.read_state(as_torch=True)
    back.close()
    ref_psi = torch.from_numpy(p.psi).to("cuda")
    ref_u = torch.from_numpy(p.u).to("cuda")
    scale = max(float(ref_psi.abs().max()), float(ref_u.abs().max()))
    err = max(float((psi0 - ref_psi).abs().max()), float((u0 - ref_u).abs().max()),
              float(v0.abs().max()))  # v0 = 0
    print("  max deviation after 200 steps there and back:", err / scale, flush=True)
    assert err <= 1e-11 * scale


def test_batched_config_full_size_equals_runs_alone():
    probs = workloads.batched_instances(count=64, steps=500)
    say("batched: 64 2-D instances x 500 steps, hipGraph")
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims, graph=True)
    b.step(500)
    picks = (0, 17, 31, 63)
    got = [sims[i].read_state() for i in picks]
    small_got = {i: sims[i].read_state() for i, p in enumerate(probs) if p.n <= 256}
    b.close()
    for s in sims:
        s.close()
    for i, g in zip(picks, got):
        s = kgs.simulation_from_problem(probs[i])
        s.step(500)
        ref = s.read_state()
        s.close()
        for x, y in zip(g, ref):
            assert np.array_equal(x, y), i
    # every member up to n = 256 (the oracle needs about a second each) and
    # the picks of n <= 512 against the oracle over the whole 500 steps
    small = [i for i, p in enumerate(probs) if p.n <= 256]
    say("batched: oracle on", len(small), "members of n <= 256")
    for i in small:
        oracle_check.check(probs[i], small_got[i], 500, label=f"member {i} (n={probs[i].n})")


@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
def test_3d_256_sampled_points_match_the_oracle(prec):
    """A full 256^3 grid after 4 steps (two 4-sweep streaming launches and
    the closing sweep, the launch configuration bench.py times), checked
    against the oracle point by point on samples.  After K steps (2K+1 colour sweeps) a value
    depends only on points at most 2K+1 away along the axes, so the oracle
    run on a 24^3 periodic sub-block that starts from the same data is exact
    in its central 4^3 points: what its wrong periodic wrap spoils travels
    at most 9 points inward.  The blocks start at even offsets, so that
    their local colours are the global ones."""
    import oracle

    steps, B, lo_i, hi_i = 4, 24, 10, 14
    # the launch configuration depends on n and the precision only; random
    # fields make every sampled block count (the configuration's Gaussian
    # is below 1e-20 away from the centre)
    p = workloads.random_problem(3, 256, seed=17, tau=0.002, amp=0.5, lo=-8.0, hi=8.0,
                                 precision=prec)
    say("3-D 256^3 x 4 steps, sampled oracle", prec)
    sim = kgs.simulation_from_problem(p)
    assert sim.info().kernel == kgs.KGS_KERNEL_STREAM
    sim.step(steps)
    psi, u, v = sim.read_state()
    sim.close()
    h = (p.hi - p.lo) / p.n
    rng = np.random.default_rng(7)
    starts = [(0, 0, 0), (244, 120, 250)] + [tuple(int(x) for x in 2 * rng.integers(0, 128, size=3))
                                              for _ in range(4)]
    for st in starts:
        idx = np.ix_(*[(np.arange(B) + s) % p.n for s in st])
        g = oracle.Grid(3, B, 0.0, B * h, p.kappa1, p.kappa2, p.mu, p.gamma)
        c = (slice(lo_i, hi_i),) * 3
        refs = sub_block_refs(g, p.tau, steps, prec, (p.psi[idx], p.u[idx], p.v[idx]), c)
        got = (psi[idx][c], u[idx][c], v[idx][c])
        oracle_check.compare(prec, got, *refs, label=f"block at {st}")


@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
def test_3d_256_whole_grid_after_the_bench_sequence_matches_the_oracle(prec):
    """The sequence bench.py times, at full size: kgs_step (4-sweep streaming
    launches; the sweep that closes the last step is left pending), then
    kgs_energy (that sweep and the reduction in one pass).  Every point of
    the 256^3 grid after 4 steps against the all-cores oracle (bitwise the
    one-core oracle), and the energy against the oracle's energy of the
    state the GPU holds."""
    import os

    import oracle

    steps = 4
    p = workloads.random_problem(3, 256, seed=19, tau=0.002, amp=0.5, lo=-8.0, hi=8.0,
                                 precision=prec)
    say("3-D 256^3 x 4 steps + closing energy, whole grid vs oracle", prec)
    sim = kgs.simulation_from_problem(p)
    assert sim.info().kernel == kgs.KGS_KERNEL_STREAM
    sim.step(steps)
    e = sim.energy()
    got = sim.read_state()
    sim.close()
    threads = max(1, min(16, os.cpu_count() or 1))
    g = oracle_check.grid_of(p)
    refs = []
    for bits in ((64,) if prec == workloads.FP64 else (64, 32)):
        r = oracle.State.from_fields(p.psi, p.u, p.v)
        oracle.step_passes(g, p.tau, r, steps, storage_bits=bits, threads=threads)
        refs.append((r.psi, r.U, r.V))
    oracle_check.compare(prec, got, *refs, label="256^3 whole grid")
    e_ref = oracle.energy(g, oracle.State.from_fields(*got))
    assert abs(e - e_ref) <= 1e-13 * abs(e_ref), (e, e_ref)


def sub_block_refs(g, tau, steps, prec, initial, c):
    """The float64 oracle (and, for a float32 state, its float32-storage
    mode) on a periodic sub-block from `initial` = (psi, u, v), restricted to
    the central points c where the sub-block is exact."""
    import oracle

    out = []
    for bits in ((64,) if prec == workloads.FP64 else (64, 32)):
        s0 = oracle.State.from_fields(*initial)
        if bits == 64:
            oracle.step(g, tau, s0, steps)
        else:
            oracle.step_passes(g, tau, s0, steps, storage_bits=32)
        out.append((s0.psi[c], s0.U[c], s0.V[c]))
    return out + [None] * (2 - len(out))


@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
@pytest.mark.parametrize("dim,n", [(3, 1024), (2, 32768), (1, 1 << 30)])
def test_largest_grids_sampled_points_match_the_oracle(dim, n, prec):
    """Grids of 2^30 points (3-D 1024^3, 2-D 32768^2, 1-D 2^30): a colour's
    pair plane is 8.6 GB in float64, so every state offset is beyond 32
    bits.  Random fields made on the device go in through the device
    boundary; after 4 steps (the library's default launches: tiles for
    2-D float64, streaming otherwise in 2-D and 3-D, colour sweeps in 1-D)
    six 24^dim sub-blocks, two of them
    across the periodic edges, match the oracle in their central 4^dim
    points, and the float64 energy is conserved."""
    import torch

    import oracle

    steps, B, lo_i, hi_i = 4, 24, 10, 14
    lo, hi, tau = -8.0, 8.0, 0.002
    say(f"{dim}-D {n}^{dim} x {steps} steps, sampled oracle", prec)
    cfg = kgs.make_config(dim, n, lo, hi, tau, 1.0, 1.0, 1.0, 1.0, prec)
    fields = workloads.random_fields_torch(dim, n, seed=23)
    rng = np.random.default_rng(11)
    starts = [(0,) * dim, tuple(n - 12 if a % 2 == 0 else n // 2 - 12 for a in range(dim))] + [
        tuple(int(x) for x in 2 * rng.integers(0, n // 2, size=dim)) for _ in range(4)]
    index = [[torch.from_numpy((np.arange(B) + s) % n).to("cuda") for s in st] for st in starts]

    def block(t, ix):
        for a, sel in enumerate(ix):
            t = t.index_select(a, sel)
        return t.cpu().numpy()

    initial = [[block(f, ix) for f in fields] for ix in index]
    stream = torch.cuda.current_stream()
    h = kgs.kgs_init(cfg, *[f.data_ptr() for f in fields], kgs.KGS_DEVICE, stream.cuda_stream)
    try:
        del fields
        torch.cuda.synchronize()
        expected = (kgs.KGS_KERNEL_SWEEP if dim == 1 else
                    kgs.KGS_KERNEL_TILE if dim == 2 and prec == workloads.FP64 else
                    kgs.KGS_KERNEL_STREAM)
        assert kgs.kgs_get_info(h).kernel == expected
        e0 = kgs.kgs_energy(h)
        kgs.kgs_step(h, steps)
        e1 = kgs.kgs_energy(h)
        out = [torch.empty((n,) * dim, dtype=torch.float64, device="cuda") for _ in range(4)]
        kgs.kgs_read_state(h, *[o.data_ptr() for o in out], kgs.KGS_DEVICE)
    finally:
        kgs.kgs_free(h)
    print("  energy", e0, "->", e1, flush=True)
    if prec == workloads.FP64:
        assert abs(e1 - e0) <= 1e-12 * abs(e0), (e0, e1)
    hgrid = (hi - lo) / n
    g = oracle.Grid(dim, B, 0.0, B * hgrid, 1.0, 1.0, 1.0, 1.0)
    c = (slice(lo_i, hi_i),) * dim
    for st, ix, (P0, Q0, U0, V0) in zip(starts, index, initial):
        refs = sub_block_refs(g, tau, steps, prec, (P0 + 1j * Q0, U0, V0), c)
        P, Q, U, V = (block(o, ix)[c] for o in out)
        oracle_check.compare(prec, (P + 1j * Q, U, V), *refs, label=f"block at {st}")


@pytest.mark.parametrize("which,n", [("2d", 2048), ("3d", 256)])
def test_paper_timing_examples_full_size_conserve_energy(which, n):
    """The paper's own GPU timing examples (Tab. time-2d at its largest grid,
    Tab. gpu3d_list at 256^3 with kappa1 < 0) over their 100 steps: the
    discrete energy is conserved in the launch configuration the library
    picks for them."""
    p = (workloads.timing_2d if which == "2d" else workloads.timing_3d)(n)
    say("paper timing example", which, n, p.steps, "steps")
    sim = kgs.simulation_from_problem(p)
    try:
        e0 = sim.energy()
        sim.step(p.steps)
        e1 = sim.energy()
    finally:
        sim.close()
    print("  energy", e0, "->", e1, flush=True)
    assert abs(e1 - e0) <= 1e-12 * abs(e0), (e0, e1)
