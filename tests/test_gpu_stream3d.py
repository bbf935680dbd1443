"""GPU: the 3-D z-streaming kernel (1 or 2 DP-AVF2 steps per launch, ping-pong
buffers) gives bitwise the same state as the one-sweep-per-launch kernel, for
every tile/chunk shape, and matches the oracle."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def tuning(tile_x, tile_y, chunk, spl):
    t = kgs.KgsTuning()
    t.kernel = kgs.KGS_KERNEL_STREAM
    t.block = 256
    t.tile_x, t.tile_y, t.chunk, t.steps_per_launch = tile_x, tile_y, chunk, spl
    return t


def sweep_tuning():
    t = kgs.KgsTuning()
    t.kernel = kgs.KGS_KERNEL_SWEEP
    t.block = 256
    return t


def run(p, steps, t=None):
    sim = kgs.simulation_from_problem(p, tuning=t if t is not None else sweep_tuning())
    try:
        sim.step(steps)
        e = sim.energy()
        return sim.read_state(), e
    finally:
        sim.close()


SHAPES = [
    # n, steps, tile_x, tile_y, chunk, steps per launch
    (26, 5, 8, 6, 5, 1),
    (26, 5, 8, 6, 5, 2),
    (32, 4, 16, 32, 32, 1),
    (32, 3, 16, 17, 32, 2),
    (6, 3, 16, 16, 16, 1),
    (6, 3, 2, 3, 2, 2),
    (2, 2, 1, 1, 1, 2),
    (40, 2, 20, 12, 7, 1),
    (40, 3, 16, 16, 13, 2),   # the compiled-in float64 tile, ragged tiles and chunks
    (36, 4, 16, 16, 128, 2),  # chunk longer than the grid
    (58, 3, 16, 28, 20, 2),   # 720 threads (3 waves per SIMD), ragged
    (30, 2, 20, 20, 9, 2),    # a 768-thread runtime shape
    (70, 3, 32, 13, 20, 2),   # the wide float64 tile (756 threads), ragged along x, y and z
    (66, 2, 32, 13, 30, 2),   # the same, tiles wider than the grid's 33 positions
]


@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
@pytest.mark.parametrize("n,steps,tx,ty,chunk,spl", SHAPES)
def test_stream_equals_sweep_bitwise(n, steps, tx, ty, chunk, spl, prec):
    p = workloads.random_problem(3, n, seed=31 + n, tau=0.04, amp=0.5, precision=prec)
    say("stream vs sweep", n, steps, tx, ty, chunk, spl, prec)
    (a, ea) = run(p, steps)
    (b, eb) = run(p, steps, tuning(tx, ty, chunk, spl))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert ea == eb


# float32 shapes beyond 12 waves per workgroup: the four-sweep float32
# pipeline fits 128 VGPRs, so up to 16 waves (float64 stops at 12)
F32_SHAPES = [
    (70, 3, 16, 32, 20, 2),   # the float32 default tile (832 threads), ragged tiles and chunks
    (66, 3, 32, 16, 64, 2),   # 896 threads, chunk longer than the grid
    (40, 5, 16, 40, 7, 2),    # 960 threads
    (34, 4, 16, 32, 9, 1),    # the default tile with 2 sweeps per launch
]


@pytest.mark.parametrize("n,steps,tx,ty,chunk,spl", F32_SHAPES)
def test_fp32_wide_workgroups_equal_sweep_bitwise(n, steps, tx, ty, chunk, spl):
    p = workloads.random_problem(3, n, seed=41 + n, tau=0.04, amp=0.5, precision=workloads.FP32)
    say("fp32 stream vs sweep", n, steps, tx, ty, chunk, spl)
    (a, ea) = run(p, steps)
    (b, eb) = run(p, steps, tuning(tx, ty, chunk, spl))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert ea == eb


def test_wide_workgroups_are_float32_only():
    say("16x32 tile: float32 only")
    for prec, ok in ((workloads.FP32, True), (workloads.FP64, False)):
        p = workloads.random_problem(3, 64, seed=2, precision=prec)
        sim = kgs.simulation_from_problem(p)
        try:
            if ok:
                sim.tuning = tuning(16, 32, 32, 2)
                assert (sim.tuning.tile_x, sim.tuning.tile_y) == (16, 32)
            else:
                with pytest.raises(kgs.KgsError):
                    sim.tuning = tuning(16, 32, 32, 2)
        finally:
            sim.close()


@pytest.mark.parametrize("n,tile", [(96, (16, 16)), (128, (16, 32)), (256, (16, 32))])
def test_default_fp32_3d_tile(n, tile):
    p = workloads.random_problem(3, n, seed=3, precision=workloads.FP32)
    say("fp32 default tile", n)
    sim = kgs.simulation_from_problem(p)
    try:
        t = sim.tuning
        assert t.kernel == kgs.KGS_KERNEL_STREAM
        assert (t.tile_x, t.tile_y) == tile
    finally:
        sim.close()


@pytest.mark.parametrize("prec", [workloads.FP64, workloads.FP32])
def test_default_chunk_on_a_grid_between_whole_rounds(prec):
    # at 224^3 the items of 64-plane (float64) or 32-plane (float32) chunks
    # fill 1.5 rounds of the CUs: the default takes equal splits of 45
    # planes (4 x 45 + 44) and a ragged last one, bitwise the same state
    p = workloads.random_problem(3, 224, seed=7, tau=0.02, amp=0.5, precision=prec)
    say("default chunk 224^3", prec)
    sim = kgs.simulation_from_problem(p)
    try:
        t = sim.tuning
    finally:
        sim.close()
    assert t.kernel == kgs.KGS_KERNEL_STREAM and t.chunk == 45
    (a, ea) = run(p, 2)
    (b, eb) = run(p, 2, t)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert ea == eb


def test_default_fp64_wide_tile_at_full_size_equals_sweep():
    """At 384^3 the float64 default is the 12-wave 32x13 tile with 96-plane
    chunks (180 tiles x 4 chunks), at 200^3 the same tile with the equal
    split of 50 planes (4 x 16 tiles x 4 chunks); two steps give bitwise the
    state of the colour sweeps.  At 256^3 the default stays 16x16 x 128
    planes."""
    import torch

    say("float64 default tile 256^3 / 384^3 / 200^3")
    for n, want in ((256, (16, 16, 128)), (384, (32, 13, 96)), (200, (32, 13, 50))):
        cfg = kgs.make_config(3, n, -8.0, 8.0, 0.002)
        f = workloads.random_fields_torch(3, n, seed=29)
        psi = torch.complex(f[0], f[1])
        states = []
        for t in (None, sweep_tuning()):
            sim = kgs.Simulation(cfg, psi, f[2], f[3], tuning=t)
            try:
                if t is None:
                    d = sim.tuning
                    assert d.kernel == kgs.KGS_KERNEL_STREAM
                    assert (d.tile_x, d.tile_y, d.chunk) == want
                    if n == 256:
                        break
                sim.step(2)
                states.append(sim.read_state(as_torch=True))
            finally:
                sim.close()
        if n != 256:
            for x, y in zip(*states):
                assert torch.equal(x, y)
        del f, psi, states
        torch.cuda.empty_cache()


def test_stream_matches_oracle_3d_config_reduced():
    p = workloads.config_3d(n=32, steps=200)
    say("stream vs oracle 32^3 x 200")
    (psi, u, v), e = run(p, p.steps, tuning(16, 17, 32, 2))
    oracle_check.check(p, (psi, u, v), p.steps)


def test_stream_rejects_bad_shapes():
    p = workloads.random_problem(3, 8, seed=1)
    say("bad shapes")
    sim = kgs.simulation_from_problem(p)
    for bad in (tuning(0, 4, 4, 1), tuning(4, 4, 4, 3), tuning(64, 64, 4, 1), tuning(4, 4, 0, 1)):
        with pytest.raises(kgs.KgsError):
            sim.tuning = bad
    sim.close()
    # 1-D grids have no streaming kernel
    p1 = workloads.random_problem(1, 8, seed=1)
    sim = kgs.simulation_from_problem(p1)
    with pytest.raises(kgs.KgsError):
        sim.tuning = tuning(4, 4, 4, 1)
    sim.close()


def test_default_3d_fp64_uses_streaming_kernel_and_matches_sweep_at_full_size():
    p = workloads.config_3d(n=256)
    say("full-size default (streaming) vs sweep, 2 steps")
    sim = kgs.simulation_from_problem(p)
    assert sim.tuning.kernel == kgs.KGS_KERNEL_STREAM
    sim.step(2)
    a = sim.read_state()
    sim.close()
    (b, _) = run(p, 2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_autotune_keeps_state_and_results():
    p = workloads.random_problem(3, 66, seed=8, tau=0.03, amp=0.5)
    say("autotune")
    sim = kgs.simulation_from_problem(p)
    before = sim.read_state()
    best = sim.autotune(steps=2, use_cache=False)
    after = sim.read_state()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert sim.tuning.kernel == best.kernel
    sim.step(3)
    tuned = sim.read_state()
    sim.close()
    (ref, _) = run(p, 3)
    for x, y in zip(tuned, ref):
        assert np.array_equal(x, y)
    # cached winner reused for the same grid
    sim2 = kgs.simulation_from_problem(p)
    again = sim2.autotune(steps=2, use_cache=True)
    assert (again.kernel, again.tile_x, again.tile_y, again.chunk, again.steps_per_launch,
            again.block) == (best.kernel, best.tile_x, best.tile_y, best.chunk,
                             best.steps_per_launch, best.block)
    sim2.close()


def test_autotune_cache_file(tmp_path, monkeypatch):
    import torch

    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KGS_TUNE_CACHE", str(path))
    arch = torch.cuda.get_device_properties(0).gcnArchName.replace(" ", "_")
    # a hand-written line for a grid no other test tunes (sweeps of 128
    # threads): reused as it stands, without timing
    path.write_text(f"not a tuning line\nkgs-tune-v1 {arch} 3 42 0 {kgs.KGS_KERNEL_SWEEP} "
                    "128 0 0 0 0\n")
    p = workloads.random_problem(3, 42, seed=9, tau=0.03, amp=0.5)
    say("autotune cache file")
    sim = kgs.simulation_from_problem(p)
    got = sim.autotune(steps=1, use_cache=True)
    assert (got.kernel, got.block) == (kgs.KGS_KERNEL_SWEEP, 128)
    assert (sim.tuning.kernel, sim.tuning.block) == (kgs.KGS_KERNEL_SWEEP, 128)
    sim.step(2)
    a = sim.read_state()
    sim.close()
    (b, _) = run(p, 2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # a winner found by timing is appended to the file
    q = workloads.random_problem(3, 44, seed=10, tau=0.03, amp=0.5)
    sim = kgs.simulation_from_problem(q)
    best = sim.autotune(steps=1, use_cache=False)
    sim.close()
    last = path.read_text().strip().splitlines()[-1].split()
    assert last[:5] == ["kgs-tune-v1", arch, "3", "44", "0"]
    assert [int(v) for v in last[5:]] == [best.kernel, best.block, best.tile_x, best.tile_y,
                                          best.chunk, best.steps_per_launch]
