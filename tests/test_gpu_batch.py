"""GPU: batches of uneven simulations (one batched launch per colour sweep and
class, optional hipGraph replay) end bitwise where individual runs end, and
every member matches the oracle (float64 <= 1e-12; float32 as in
tests/oracle_check.py): points of one colour are independent (sec. 4.2,
Algorithm 3), so how the members share launches does not change a result."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def mixed_problems(seed=0):
    specs = [(1, 1030, 0), (1, 64, 1), (2, 70, 0), (2, 34, 1), (2, 16, 0), (3, 18, 0), (3, 12, 1),
             (3, 64, 0), (2, 2, 0), (3, 2, 1)]
    out = []
    for i, (d, n, prec) in enumerate(specs):
        out.append(workloads.random_problem(d, n, seed=seed * 100 + i, tau=0.03, amp=0.5,
                                            precision=prec))
    return out


def states(sims):
    return [s.read_state() for s in sims]


def match_oracle(probs, got, steps, what):
    steps = [steps] * len(probs) if isinstance(steps, int) else steps
    for i, (p, g, k) in enumerate(zip(probs, got, steps)):
        oracle_check.check(p, g, k, label=f"{what} member {i} ({p.dim}-D n={p.n}, {k} steps)",
                           cache=True)


def same(a, b):
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            if not np.array_equal(u, v):
                return False
    return True


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_individual_runs_bitwise(graph):
    probs = mixed_problems(1)
    say("batch uniform, graph =", graph)
    ref = []
    for p in probs:
        s = kgs.simulation_from_problem(p)
        s.step(7)
        ref.append(s.read_state())
        s.close()
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims, graph=graph)
    b.step(3)
    b.step(4)
    got = states(sims)
    b.close()
    for s in sims:
        s.close()
    assert same(got, ref)
    match_oracle(probs, got, 7, f"uniform batch (graph={graph})")


def test_graph_replays_match_eager_every_time():
    probs = mixed_problems(2)
    say("graph replays")
    eager = [kgs.simulation_from_problem(p) for p in probs]
    graphed = [kgs.simulation_from_problem(p) for p in probs]
    be = kgs.Batch(eager, graph=False)
    bg = kgs.Batch(graphed, graph=True)
    for rep in range(4):
        be.step(5)
        bg.step(5)  # captured on the first call, replayed afterwards
        # eager work between replays: energies and a read-back
        e1 = [s.energy() for s in graphed]
        e0 = [s.energy() for s in eager]
        assert e1 == e0, rep
        got = states(graphed)
        assert same(got, states(eager)), rep
        match_oracle(probs, got, 5 * (rep + 1), f"graph replay {rep}")
    be.close()
    bg.close()
    for s in eager + graphed:
        s.close()


def test_step_each_uneven_counts():
    probs = mixed_problems(3)
    counts = [0, 5, 3, 1, 6, 2, 4, 0, 3, 7]
    say("uneven counts", counts)
    ref = []
    for p, k in zip(probs, counts):
        s = kgs.simulation_from_problem(p)
        s.step(k)
        ref.append(s.read_state())
        s.close()
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims)
    b.step_each(counts)
    got = states(sims)
    # a second uneven run reuses the schedule buffers
    counts2 = [2, 0, 1, 3, 0, 1, 1, 2, 0, 1]
    b.step_each(counts2)
    got2 = states(sims)
    b.close()
    for s in sims:
        s.close()
    assert same(got, ref)
    match_oracle(probs, got, counts, "step_each")
    ref2 = []
    for p, k, k2 in zip(probs, counts, counts2):
        s = kgs.simulation_from_problem(p)
        s.step(k)
        s.step(k2)
        ref2.append(s.read_state())
        s.close()
    assert same(got2, ref2)
    match_oracle(probs, got2, [a + b for a, b in zip(counts, counts2)], "step_each twice")


def test_members_stepped_alone_in_between():
    # a 3-D float64 member (n >= 96) steps alone with the ping-pong streaming
    # kernel between batched runs: the batch follows its current buffer
    probs = [workloads.random_problem(3, 96, seed=5, tau=0.03, amp=0.5),
             workloads.random_problem(2, 40, seed=6, tau=0.03, amp=0.5)]
    say("alone + batched")
    sims = [kgs.simulation_from_problem(p) for p in probs]
    assert sims[0].tuning.kernel == kgs.KGS_KERNEL_STREAM
    b = kgs.Batch(sims)
    b.step(2)
    sims[0].step(3)
    sims[1].step(3)
    b.step(2)
    got = states(sims)
    b.close()
    for s in sims:
        s.close()
    ref = []
    for p in probs:
        s = kgs.simulation_from_problem(p)
        s.step(7)
        ref.append(s.read_state())
        s.close()
    assert same(got, ref)
    match_oracle(probs, got, 7, "alone + batched")


def test_batch_rejects_bad_input():
    p = workloads.random_problem(2, 8, seed=1)
    say("batch errors")
    s = kgs.simulation_from_problem(p)
    with pytest.raises(kgs.KgsError):
        kgs.Batch([s, s])
    b = kgs.Batch([s])
    with pytest.raises(kgs.KgsError):
        b.step(-1)
    with pytest.raises(kgs.KgsError):
        b.step_each([-2])
    b.close()
    s.close()


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
@pytest.mark.parametrize("sizes", [[130, 200, 256, 1030, 66 * 2, 90 * 2], [2048, 130, 514]],
                         ids=["tiled", "streamed"])
def test_2d_batches_stream_and_equal_individual_runs(graph, prec, sizes):
    # uneven 2-D members beyond one workgroup: uniform runs use 2 steps per
    # launch (an even number of launches) of the tiled kernel when every
    # member is below n = 2048, else of the y-streaming kernel
    probs = [workloads.random_problem(2, n, seed=500 + n, tau=0.02, amp=0.5, precision=prec)
             for n in sizes]
    say("2-D batch streaming, graph =", graph, "prec", prec)
    for k_run in ([1, 2, 3], [7, 7]):
        ref = []
        for p in probs:
            t = kgs.KgsTuning()
            t.kernel = kgs.KGS_KERNEL_SWEEP
            t.block = 256
            s = kgs.simulation_from_problem(p, tuning=t)
            s.step(sum(k_run))
            ref.append(s.read_state())
            s.close()
        sims = [kgs.simulation_from_problem(p) for p in probs]
        b = kgs.Batch(sims, graph=graph)
        for k in k_run:
            b.step(k)
            sims[0].energy()  # eager work between (replayed) runs
        got = states(sims)
        b.close()
        for s in sims:
            s.close()
        assert same(got, ref), k_run
        match_oracle(probs, got, sum(k_run), f"2-D group {k_run} (graph={graph})")


def test_2d_members_stepped_alone_between_streamed_batch_runs():
    probs = [workloads.random_problem(2, 512, seed=61, tau=0.02, amp=0.5),
             workloads.random_problem(2, 150, seed=62, tau=0.02, amp=0.5)]
    say("2-D alone + batched")
    sims = [kgs.simulation_from_problem(p) for p in probs]
    # both run the ping-pong tiled kernel alone: each swaps its buffers
    assert [s.tuning.kernel for s in sims] == [kgs.KGS_KERNEL_TILE] * 2
    b = kgs.Batch(sims)
    b.step(4)
    sims[0].step(3)
    sims[1].step(3)
    b.step(5)
    got = states(sims)
    b.close()
    for s in sims:
        s.close()
    ref = []
    for p in probs:
        s = kgs.simulation_from_problem(p)
        s.step(12)
        ref.append(s.read_state())
        s.close()
    assert same(got, ref)
    match_oracle(probs, got, 12, "2-D alone + batched")


def stream3d_problems(seed=0):
    # 3-D members all large enough for the z-streaming kernel's member-list
    # launch (one class per precision), ragged against the 16x16 tile and the
    # plane chunks
    specs = [(32, 0), (40, 0), (66, 0), (96, 0), (34, 0), (128, 0), (32, 1), (50, 1), (72, 1)]
    return [workloads.random_problem(3, n, seed=seed * 100 + i, tau=0.03, amp=0.5, precision=prec)
            for i, (n, prec) in enumerate(specs)]


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("calls", [(2,), (3,), (4, 5), (7,)])
def test_batch_3d_streaming_equals_individual_runs_and_oracle(graph, calls):
    probs = stream3d_problems(4)
    total = sum(calls)
    say("3-D streaming batch, graph =", graph, "calls", calls)
    ref = []
    for p in probs:
        s = kgs.simulation_from_problem(p)
        s.step(total)
        ref.append(s.read_state())
        s.close()
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims, graph=graph)
    for k in calls:
        b.step(k)
    got = states(sims)
    if graph:
        # a replay of the captured run on top, against the eager path
        b.step(calls[0])
        again = states(sims)
    b.close()
    for s in sims:
        s.close()
    assert same(got, ref)
    match_oracle(probs, got, total, f"3-D streaming batch (graph={graph})")
    if graph:
        ref2 = []
        for p in probs:
            s = kgs.simulation_from_problem(p)
            s.step(total + calls[0])
            ref2.append(s.read_state())
            s.close()
        assert same(again, ref2)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_3d_wide_tile_group_equals_individual_runs_and_oracle(graph):
    """A float64 group (n = 66, 98, 130, 162) whose member-list launches the
    planner gives the 12-wave 32x13 tile (chunk 32): ragged tiles along x,
    y and z in every member; run alone, each member streams with 16x16
    tiles or sweeps."""
    probs = [workloads.random_problem(3, n, seed=700 + n, tau=0.03, amp=0.5)
             for n in (66, 98, 130, 162)]
    say("3-D wide-tile batch, graph =", graph)
    ref = []
    for p in probs:
        s = kgs.simulation_from_problem(p)
        s.step(5)
        ref.append(s.read_state())
        s.close()
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims, graph=graph)
    b.step(2)
    b.step(3)
    got = states(sims)
    b.close()
    for s in sims:
        s.close()
    assert same(got, ref)
    match_oracle(probs, got, 5, f"3-D wide-tile batch (graph={graph})")


def tuner_problems(seed=0):
    # a 2-D streaming group, a 3-D member-list group, a resident member and a
    # 3-D member below the list kernel's size (its class sweeps)
    specs = [(2, 96, 0), (2, 130, 0), (2, 200, 0), (3, 32, 0), (3, 40, 0), (3, 66, 0),
             (2, 34, 0), (3, 20, 1), (2, 90, 1), (2, 160, 1)]
    return [workloads.random_problem(d, n, seed=seed * 100 + i, tau=0.03, amp=0.5, precision=prec)
            for i, (d, n, prec) in enumerate(specs)]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_autotune_keeps_states_and_results(graph, tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KGS_TUNE_CACHE", str(path))
    probs = tuner_problems(5 + int(graph))
    say("batch autotune, graph =", graph)
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims, graph=graph)
    b.step(3)  # captured first when graph=True
    before = states(sims)
    b.autotune(steps=2, use_cache=False)
    assert same(states(sims), before)
    b.step(3)  # recaptured with the tuned launches
    b.step(3)
    got = states(sims)
    b.close()
    for s in sims:
        s.close()
    ref = []
    for p in probs:
        s = kgs.simulation_from_problem(p)
        s.step(9)
        ref.append(s.read_state())
        s.close()
    assert same(got, ref)
    match_oracle(probs, got, 9, f"tuned batch (graph={graph})")
    lines = [l.split() for l in path.read_text().splitlines() if l.startswith("kgs-group-v1")]
    assert sorted(int(l[2]) for l in lines) == [2, 2, 3]  # fp64 2-D, fp32 2-D, fp64 3-D groups
    # a second batch of the same groups reuses the winners without timing
    sims = [kgs.simulation_from_problem(p) for p in probs]
    b = kgs.Batch(sims)
    b.autotune(steps=2, use_cache=True)
    b.step(9)
    again = states(sims)
    b.close()
    for s in sims:
        s.close()
    assert same(again, ref)
    assert len([l for l in path.read_text().splitlines() if l.startswith("kgs-group-v1")]) == 3
