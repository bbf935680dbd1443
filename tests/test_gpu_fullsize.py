"""GPU, full sizes in the launch configurations bench.py times.

After 200 steps of the 3-D 256^3 grid the oracle cannot be evaluated point
by point (every output depends on the whole grid), so the run is checked by
properties that hold at any size: the discrete energy is conserved, and the
symmetric composition is time-reversible (200 steps with -tau return to the
initial state).  The batched configuration (64 uneven 2-D grids x 500 steps)
is checked member by member against runs of the same grids alone."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads

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
