"""GPU: the continuous-batching server.  Each request's result equals, bitwise,
the same simulation run alone, however requests join, wait and interleave."""
import sys

import numpy as np
import pytest

from paper_2502_09537_amd import kgs, workloads
from tests import oracle_check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def alone(p, steps):
    s = kgs.simulation_from_problem(p)
    s.step(steps)
    e = s.energy()
    r = s.read_state()
    s.close()
    return r, e


def mix(seed):
    specs = [(1, 512, 0, 30), (2, 64, 1, 17), (3, 64, 0, 11), (3, 20, 1, 23), (2, 130, 0, 9),
             (1, 2050, 1, 40), (3, 16, 0, 0), (2, 34, 0, 25)]
    out = []
    for i, (d, n, prec, steps) in enumerate(specs):
        p = workloads.gaussian_problem(d, n, seed * 10 + i, -6.0, 6.0, 0.01, steps, precision=prec)
        out.append(p)
    return out


def equal(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_results_in_the_mix_equal_results_alone():
    probs = mix(1)
    say("serve mix")
    srv = kgs.Server(budget_bytes=8 << 30, steps_per_round=7)
    ids = [srv.submit_problem(p) for p in probs[:4]]
    srv.run(1)                     # first four start
    ids += [srv.submit_problem(p) for p in probs[4:]]  # the rest join later
    while True:
        nr, nq = srv.run(1)
        if nr == 0 and nq == 0:
            break
    for rid, p in zip(ids, probs):
        info = srv.poll(rid)
        assert info.state == kgs.KGS_REQ_DONE, (rid, info.state, info.status)
        assert info.steps_done == p.steps
        got = srv.result(rid)
        ref, e_ref = alone(p, p.steps)
        assert equal(got, ref), p.name
        assert info.energy_end == e_ref
        if p.precision == workloads.FP64:
            assert abs(info.energy_end - info.energy_start) <= 1e-12 * abs(info.energy_start)
    srv.close()


@pytest.mark.parametrize("sizes", [[130, 514], [2048, 130]], ids=["tiled", "streamed"])
def test_2d_groups_equal_results_alone(sizes):
    # 2-D requests advanced together: tiled launches when every grid is
    # below n = 2048, y-streaming launches otherwise
    probs = [workloads.gaussian_problem(2, n, 40 + i, -6.0, 6.0, 0.01, 5 + i, precision=i % 2)
             for i, n in enumerate(sizes)]
    say("2-D groups", sizes)
    srv = kgs.Server(budget_bytes=8 << 30, steps_per_round=4)
    ids = [srv.submit_problem(p) for p in probs]
    while True:
        nr, nq = srv.run(1)
        if nr == 0 and nq == 0:
            break
    for rid, p in zip(ids, probs):
        info = srv.poll(rid)
        assert info.state == kgs.KGS_REQ_DONE, (rid, info.state, info.status)
        ref, e_ref = alone(p, p.steps)
        assert equal(srv.result(rid), ref), p.n
        assert info.energy_end == e_ref
    srv.close()


def test_3d_streaming_groups_equal_results_alone_and_oracle():
    # 3-D requests of the z-streaming kernel advanced together in member-list
    # launches (rounds of 4 steps; the last round of a request takes 1..3:
    # one step runs the request's own launches), joining at different times
    specs = [(96, 0, 9), (100, 1, 13), (128, 0, 6), (96, 1, 7), (112, 0, 11)]
    probs = [workloads.gaussian_problem(3, n, 60 + i, -6.0, 6.0, 0.01, k, precision=prec)
             for i, (n, prec, k) in enumerate(specs)]
    say("3-D streaming groups", specs)
    srv = kgs.Server(budget_bytes=16 << 30, steps_per_round=4)
    ids = [srv.submit_problem(p) for p in probs[:3]]
    srv.run(1)
    ids += [srv.submit_problem(p) for p in probs[3:]]
    while True:
        nr, nq = srv.run(1)
        if nr == 0 and nq == 0:
            break
    for rid, p in zip(ids, probs):
        info = srv.poll(rid)
        assert info.state == kgs.KGS_REQ_DONE, (rid, info.state, info.status)
        got = srv.result(rid)
        ref, e_ref = alone(p, p.steps)
        assert equal(got, ref), p.n
        assert info.energy_end == e_ref
        oracle_check.check(p, got, p.steps, label=f"served 3-D n={p.n}")
    srv.close()


def test_admission_respects_the_budget():
    probs = [workloads.gaussian_problem(2, 128, i, -6.0, 6.0, 0.01, 12) for i in range(6)]
    say("budget")
    # a request holds its state and its gathered result (32 bytes a point);
    # this budget admits two requests but never a third
    one = kgs.required_bytes(kgs.config_of(probs[0])) + 4 * 128 * 128 * 8
    srv = kgs.Server(budget_bytes=int(2.5 * one), steps_per_round=5)
    ids = [srv.submit_problem(p) for p in probs]
    peak = 0
    while True:
        nr, nq = srv.run(1)
        st = srv.stats()
        peak = max(peak, st.device_bytes_used)
        assert st.device_bytes_used <= 2 * one
        assert nr <= 2
        if nr == 0 and nq == 0:
            break
    assert peak > 0
    for rid, p in zip(ids, probs):
        assert srv.poll(rid).state == kgs.KGS_REQ_DONE
        assert equal(srv.result(rid), alone(p, p.steps)[0])
    srv.close()


def test_oversized_request_fails_and_cancel_works():
    say("oversized + cancel")
    big = workloads.gaussian_problem(3, 64, 1, -6.0, 6.0, 0.01, 5)
    # 2-D n = 130 does not fit one workgroup: it advances in rounds
    small = [workloads.gaussian_problem(2, 130, i, -6.0, 6.0, 0.01, 50) for i in range(3)]
    srv = kgs.Server(budget_bytes=3 << 20, steps_per_round=10, max_active=1)
    rb = srv.submit_problem(big)
    rs = [srv.submit_problem(p) for p in small]
    srv.run(1)
    assert srv.poll(rb).state == kgs.KGS_REQ_FAILED
    assert srv.poll(rb).status == kgs.KGS_ENOMEM
    assert srv.poll(rs[0]).state == kgs.KGS_REQ_RUNNING
    assert srv.poll(rs[0]).steps_done == 10
    srv.cancel(rs[2])  # queued
    assert srv.poll(rs[2]).state == kgs.KGS_REQ_CANCELLED
    srv.cancel(rs[0])  # running
    assert srv.poll(rs[0]).state == kgs.KGS_REQ_CANCELLED
    with pytest.raises(kgs.KgsError):
        srv.cancel(rs[0])
    while srv.run(1) != (0, 0):
        pass
    assert srv.poll(rs[0]).state == kgs.KGS_REQ_CANCELLED
    assert srv.poll(rs[1]).state == kgs.KGS_REQ_DONE
    assert equal(srv.result(rs[1]), alone(small[1], 50)[0])
    srv.release(rs[1])
    with pytest.raises(kgs.KgsError):
        srv.poll(rs[1])
    with pytest.raises(kgs.KgsError):
        srv.submit(kgs.make_config(2, 7, -1.0, 1.0, 0.01), np.zeros((7, 7)), np.zeros((7, 7)),
                   np.zeros((7, 7)), 3)
    srv.close()


def test_small_requests_finish_while_a_big_one_runs():
    say("lanes")
    big = workloads.gaussian_problem(3, 96, 3, -6.0, 6.0, 0.01, 2000)
    small = [workloads.gaussian_problem(1, 512, 20 + i, -6.0, 6.0, 0.01, 300) for i in range(4)]
    srv = kgs.Server(budget_bytes=8 << 30, steps_per_round=20)
    rb = srv.submit_problem(big)
    srv.run(1)
    ids = [srv.submit_problem(p) for p in small]
    rounds = 0
    while any(srv.poll(i).state != kgs.KGS_REQ_DONE for i in ids):
        srv.run(1)
        rounds += 1
        assert rounds < 90
    # the small ones finished on their own lane while the big one still runs
    assert srv.poll(rb).state == kgs.KGS_REQ_RUNNING
    while srv.run(1) != (0, 0):
        pass
    assert srv.poll(rb).state == kgs.KGS_REQ_DONE
    for rid, p in zip(ids + [rb], small + [big]):
        ref, e_ref = alone(p, p.steps)
        assert equal(srv.result(rid), ref)
        assert srv.poll(rid).energy_end == e_ref
    srv.close()


def test_shortest_remaining_work_runs_first():
    say("srpt")
    # three 2-D requests of one size, very different step counts, admitted
    # together; a round holds one request's steps
    probs = [workloads.gaussian_problem(2, 256, 40 + i, -6.0, 6.0, 0.01, k)
             for i, k in enumerate((300, 20, 100))]
    srv = kgs.Server(budget_bytes=8 << 30, steps_per_round=10, round_work=256 * 256 * 10)
    ids = [srv.submit_problem(p) for p in probs]
    while srv.run(1) != (0, 0):
        pass
    t = [srv.poll(i).t_done for i in ids]
    assert t[1] < t[2] < t[0]
    for rid, p in zip(ids, probs):
        assert equal(srv.result(rid), alone(p, p.steps)[0])
    srv.close()


def test_served_results_match_the_oracle():
    """Every request of a mixed 1-D/2-D/3-D, float64/float32 batch, served
    together, against the CPU oracle run from the same initial data (float64
    <= 1e-12; float32 as in tests/oracle_check.py)."""
    probs = mix(2)
    say("serve mix vs oracle")
    srv = kgs.Server(budget_bytes=8 << 30, steps_per_round=5)
    ids = [srv.submit_problem(p) for p in probs]
    while True:
        nr, nq = srv.run(1)
        if nr == 0 and nq == 0:
            break
    for rid, p in zip(ids, probs):
        info = srv.poll(rid)
        assert info.state == kgs.KGS_REQ_DONE, (rid, info.state, info.status)
        oracle_check.check(p, srv.result(rid), p.steps,
                           label=f"served {p.dim}-D n={p.n} {p.steps} steps")
    srv.close()
