"""kgs_step_fields (stepping without device allocation) against kgs_init +
kgs_step + kgs_read_state on the same grids, through the C ABI.

Each pair of calls runs back to back in the fixed scratch area, the second on
a smaller grid than the first, so the second finds the first's contents
there.  The bar is bitwise equality with the handle path (both run the same
kernels), which is stricter than the oracle tolerance; the smaller grids are
also held to the oracle.
"""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _fields(p):
    import torch

    t = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
         for x in (p.psi.real, p.psi.imag, p.u, p.v)]
    return t


def _handle_run(p, steps):
    sim = kgs.simulation_from_problem(p)
    try:
        sim.step(steps)
        psi, u, v = sim.read_state()
        return sim.info().kernel, (psi, u, v)
    finally:
        sim.close()


def _fields_run(p, steps):
    import torch

    P, Q, U, V = _fields(p)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    kgs.kgs_step_fields(kgs.config_of(p), P.data_ptr(), Q.data_ptr(), U.data_ptr(),
                        V.data_ptr(), steps, stream)
    torch.cuda.synchronize()
    P, Q, U, V = [a.cpu().numpy() for a in (P, Q, U, V)]
    return P + 1j * Q, U, V


def _state_bytes(p):
    count = p.n ** p.dim // 2
    stride = (count + 63) // 64 * 64
    return 8 * stride * (4 if p.precision else 8)


# (first, steps), (second, steps): the second grid is smaller
PAIRS = [
    # 2-D 1024^2 float64: two states fill the scratch area exactly (tiled
    # kernel, ping-pong), then a 2-D 192^2 grid
    ((lambda: workloads.config_2d(n=1024, steps=3), 3),
     (lambda: workloads.config_2d(n=192, steps=4), 4)),
    # 3-D 96^3 float64 (z-streaming, ping-pong), then 3-D 64^3 float32 (sweeps)
    ((lambda: workloads.config_3d(n=96, steps=3), 3),
     (lambda: workloads.config_3d(n=64, steps=5, precision=workloads.FP32), 5)),
    # 3-D 128^3 float64: one state fills the scratch area, so the in-place
    # sweeps replace the ping-pong kernel; then the 1-D config (resident)
    ((lambda: workloads.config_3d(n=128, steps=2), 2),
     (lambda: workloads.config_1d(steps=7), 7)),
]


@pytest.mark.parametrize("pair", range(len(PAIRS)))
def test_step_fields_matches_handle_path(pair):
    prev = None
    for make, steps in PAIRS[pair]:
        p = make()
        assert _state_bytes(p) <= kgs.KGS_STEP_FIELDS_SCRATCH_BYTES
        if prev is not None:
            assert p.n ** p.dim < prev
        prev = p.n ** p.dim
        say("step_fields", p.name, p.dim, p.n, steps, "fp32" if p.precision else "fp64")
        kernel, (hpsi, hu, hv) = _handle_run(p, steps)
        fpsi, fu, fv = _fields_run(p, steps)
        assert np.array_equal(fpsi, hpsi), (p.name, "psi")
        assert np.array_equal(fu, hu), (p.name, "u")
        assert np.array_equal(fv, hv), (p.name, "v")
        if p.n ** p.dim <= 192 ** 2 or p.dim == 1 or (p.dim == 3 and p.n <= 64):
            oracle_check.check(p, (fpsi, fu, fv), steps, label="step_fields " + p.name)
        say("ok", p.name, "handle kernel", kernel)


def test_step_fields_zero_steps_is_a_round_trip():
    p = workloads.config_2d(n=256, steps=0)
    say("step_fields zero steps", p.name, p.n)
    psi, u, v = _fields_run(p, 0)
    assert np.array_equal(psi, p.psi)
    assert np.array_equal(u, p.u)
    assert np.array_equal(v, p.v)


def test_step_fields_rejects_grids_beyond_the_scratch_area():
    import torch

    p = workloads.config_2d(n=256, steps=1)
    P, Q, U, V = _fields(p)
    # 3-D 130^3 float64 needs more than the scratch area; the size check comes
    # before any device work, so the small arrays are never touched
    cfg = kgs.make_config(3, 130, -8.0, 8.0, 0.002)
    say("step_fields oversize", 130)
    with pytest.raises(kgs.KgsError) as ei:
        kgs.kgs_step_fields(cfg, P.data_ptr(), Q.data_ptr(), U.data_ptr(), V.data_ptr(), 1,
                            torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == kgs.KGS_ENOMEM
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert np.array_equal(P.cpu().numpy(), p.psi.real)
