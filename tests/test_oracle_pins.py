"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them calls the GPU library.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid, State
from tests.avf_reference import PointProblem, dp_avf_point_solve, energy_matrix_form, laplacian_matrix
from paper_2502_09537_amd import workloads


def rand_state(rng, shape, amp=1.0):
    return State(amp * rng.uniform(-1, 1, shape), amp * rng.uniform(-1, 1, shape),
                 amp * rng.uniform(-1, 1, shape), amp * rng.uniform(-1, 1, shape))


def rel_max(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ---------------------------------------------------------------------------
# Pointwise algebra: the closed-form updates of sec. 4.1 (eq. scheme1 and
# scheme1-adj) against a Newton solve of the DP-AVF definition (eq. dp-avf,
# dp-avf-i) with gradients of E_h by complex step.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", [(1, 6), (2, 4), (3, 4)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_point_updates_match_newton_solve_of_avf_equation(dim, n, adjoint):
    rng = np.random.default_rng(100 * dim + n + adjoint)
    for trial in range(3):
        k1, k2, mu, g = rng.uniform(0.3, 2.0, 4)
        if trial == 1:
            k1 = -k1  # the paper's 3-D example has kappa1 < 0 (sec. 5.2)
        h = rng.uniform(0.2, 1.0)
        tau = rng.uniform(0.01, 0.4)
        grid = Grid(dim, n, 0.0, n * h, k1, k2, mu, g)
        s = rand_state(rng, grid.shape)
        i = int(rng.integers(grid.n ** dim))
        pp = PointProblem(dim, n, h, k1, k2, mu, g, *s.arrays())
        for pair in ("psi", "uv"):
            y = dp_avf_point_solve(pp, tau, i, pair, adjoint)
            t = s.copy()
            if pair == "psi":
                oracle.psi_update(grid, tau, t, i)
                got = np.array([t.P.ravel()[i], t.Q.ravel()[i]])
            else:
                oracle.uv_update(grid, tau, t, i)
                got = np.array([t.U.ravel()[i], t.V.ravel()[i]])
            assert np.all(np.abs(got - y) <= 1e-14 * np.maximum(1.0, np.abs(y))), (pair, got, y)
            # nothing else changes
            for f_new, f_old, name in zip(t.arrays(), s.arrays(), "PQUV"):
                other = np.delete(f_new.ravel(), i)
                assert np.array_equal(other, np.delete(f_old.ravel(), i)), name


# ---------------------------------------------------------------------------
# Energy function: forward-difference form (oracle) == matrix form of sec. 2
# (summation by parts), and closed forms for plane waves.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", [(1, 8), (2, 6), (3, 4)])
def test_energy_equals_matrix_form(dim, n):
    rng = np.random.default_rng(7 + dim)
    k1, k2, mu, g = rng.uniform(-2.0, 2.0, 4)
    grid = Grid(dim, n, -1.0, 2.0, k1, k2, mu, g)
    s = rand_state(rng, grid.shape)
    D = laplacian_matrix(dim, n, grid.h)
    ref = energy_matrix_form(D, grid.h, dim, k1, k2, mu, g, *(a.ravel() for a in s.arrays()))
    assert abs(oracle.energy(grid, s) - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("dim,n", [(1, 64), (2, 24), (3, 12)])
def test_energy_plane_wave_closed_form(dim, n):
    # psi = A e^{i k.x}, u = B cos(k'.x) + C0, v = C: sum |grad_h psi|^2 =
    # N^d A^2 sum_a 4 sin^2(k_a h/2)/h^2, sum |grad_h u|^2 = N^d B^2 sum_a
    # 2 sin^2(k'_a h/2)/h^2, sum u^2 = N^d (B^2/2 + C0^2), sum |psi|^2 u = N^d A^2 C0.
    k1, k2, mu, g = 0.7, 1.3, 0.9, 1.1
    A, B, C0, C = 0.8, 0.6, 0.3, -0.4
    L = 2 * np.pi
    grid = Grid(dim, n, 0.0, L, k1, k2, mu, g)
    X = workloads.axes(dim, n, 0.0, L)
    m = np.array([1, 2, 3][:dim])
    mp = np.array([2, 1, 1][:dim])
    ph = sum(m[a] * X[a] for a in range(dim))
    php = sum(mp[a] * X[a] for a in range(dim))
    s = State(A * np.cos(ph), A * np.sin(ph), B * np.cos(php) + C0, np.full(grid.shape, C))
    h = grid.h
    M = n ** dim
    grad_psi = M * A * A * np.sum(4 * np.sin(m * h / 2) ** 2) / h ** 2
    grad_u = M * B * B * np.sum(2 * np.sin(mp * h / 2) ** 2) / h ** 2
    E = 0.5 * (k1 * grad_psi + k2 * grad_u + M * C * C + mu * mu * M * (B * B / 2 + C0 * C0)) \
        - g * M * A * A * C0
    assert abs(oracle.energy(grid, s) - h ** dim * E) <= 1e-12 * abs(h ** dim * E)


# ---------------------------------------------------------------------------
# Energy conservation (Thm 3.2 / 3.3): every single point update conserves
# E_h, and so does every step in any update order.
# ---------------------------------------------------------------------------
def energy_terms_scale(grid, s):
    # sum of |terms| bounds the rounding of the energy evaluation
    t = State(np.abs(s.P), np.abs(s.Q), np.abs(s.U), np.abs(s.V))
    g = Grid(grid.dim, grid.n, grid.lo, grid.hi, abs(grid.kappa1), abs(grid.kappa2), grid.mu,
             -abs(grid.gamma))
    return abs(oracle.energy(g, t)) + 1.0


@pytest.mark.parametrize("dim,n", [(1, 16), (2, 8), (3, 6)])
def test_each_point_update_conserves_energy(dim, n):
    rng = np.random.default_rng(11 * dim)
    grid = Grid(dim, n, 0.0, 3.0, *rng.uniform(0.5, 2.0, 4))
    s = rand_state(rng, grid.shape)
    scale = energy_terms_scale(grid, s)
    for _ in range(20):
        i = int(rng.integers(n ** dim))
        e0 = oracle.energy(grid, s)
        if rng.uniform() < 0.5:
            oracle.psi_update(grid, 0.3, s, i)
        else:
            oracle.uv_update(grid, 0.3, s, i)
        assert abs(oracle.energy(grid, s) - e0) <= 64 * np.finfo(float).eps * scale


def test_energy_drift_1d_config_10k_steps():
    p = workloads.config_1d()
    grid = Grid(1, p.n, p.lo, p.hi, p.kappa1, p.kappa2, p.mu, p.gamma)
    s = State.from_fields(p.psi, p.u, p.v)
    e0 = oracle.energy(grid, s)
    worst = 0.0
    for _ in range(10):
        oracle.step(grid, p.tau, s, 1000)
        worst = max(worst, abs(oracle.energy(grid, s) - e0) / abs(e0))
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("dim,n,steps", [(2, 32, 2000), (3, 12, 1000)])
def test_energy_drift_2d_3d(dim, n, steps):
    p = workloads.gaussian_problem(dim, n, 5, -6.0, 6.0, 0.02, steps)
    grid = Grid(dim, n, p.lo, p.hi, p.kappa1, p.kappa2, p.mu, p.gamma)
    s = State.from_fields(p.psi, p.u, p.v)
    e0 = oracle.energy(grid, s)
    oracle.step(grid, p.tau, s, steps)
    assert abs(oracle.energy(grid, s) - e0) <= 1e-12 * abs(e0)


def test_random_update_orders_conserve_energy():
    # any update order, even a random one, gives an energy-preserving scheme
    # (sec. 4.2 and the random-order experiment of sec. 5.1)
    rng = np.random.default_rng(3)
    grid = Grid(2, 12, -3.0, 3.0, 1.0, 1.0, 1.0, 1.0)
    p = workloads.gaussian_problem(2, 12, 9, -3.0, 3.0, 0.05, 1, params=(1, 1, 1, 1))
    for trial in range(3):
        s = State.from_fields(p.psi, p.u, p.v)
        e0 = oracle.energy(grid, s)
        oracle.step_order(grid, 0.05, s, rng.permutation(144), 200)
        assert abs(oracle.energy(grid, s) - e0) <= 1e-13 * abs(e0)


def test_block_splitting_orders_conserve_energy_and_blocks_are_independent():
    # Algorithm 2 (the CPU strategy of sec. 4.2): each process count gives
    # its own update order and so its own DP-AVF2 scheme; each conserves the
    # energy (the block-splitting energy experiments of sec. 5), each is
    # reversed by the step with -tau, and the blocks can run in any order
    # (in parallel) without changing a bit of the result.
    n = 16
    grid = Grid(2, n, -4.0, 4.0, 1.0, 1.0, 1.0, 1.0)
    p = workloads.gaussian_problem(2, n, 11, -4.0, 4.0, 0.05, 1, params=(1, 1, 1, 1))
    finals = []
    for n_proc in (1, 2, 3, 4, 7):
        order = oracle.block_splitting_order(n, n_proc)
        assert sorted(order.tolist()) == list(range(n * n))
        s = State.from_fields(p.psi, p.u, p.v)
        e0 = oracle.energy(grid, s)
        oracle.step_order(grid, 0.05, s, order, 40)
        assert abs(oracle.energy(grid, s) - e0) <= 1e-13 * abs(e0)
        finals.append(s.copy())
        if n_proc > 1:
            rev = oracle.block_splitting_order(n, n_proc, block_sequence=range(n_proc - 1, -1, -1))
            assert not np.array_equal(rev, order)
            t = State.from_fields(p.psi, p.u, p.v)
            oracle.step_order(grid, 0.05, t, rev, 40)
            for a, b in zip(s.arrays(), t.arrays()):
                assert np.array_equal(a, b)
        back = s.copy()
        oracle.step_order(grid, -0.05, back, order, 40)
        for a, b in zip(back.arrays(), (p.psi.real, p.psi.imag, p.u, p.v)):
            assert np.max(np.abs(a - b)) <= 1e-12
    # different process counts are different schemes
    assert not np.array_equal(finals[1].P, finals[3].P)


def test_block_splitting_rows_follow_algorithm_2():
    blocks, seps = oracle.block_splitting_rows(16, 3)
    # row 0, blocks of 4, 4 and 4 rows, each followed by a separator row
    assert [list(b) for b in blocks] == [[1, 2, 3, 4], [6, 7, 8, 9], [11, 12, 13, 14]]
    assert seps == [5, 10, 15]
    # a block reads only its own rows, row 0 and the separators: no two
    # blocks are neighbours (periodic in the rows)
    owner = {r: l for l, b in enumerate(blocks) for r in b}
    for r, l in owner.items():
        for nb in ((r - 1) % 16, (r + 1) % 16):
            assert owner.get(nb, l) == l
    with pytest.raises(ValueError):
        oracle.block_splitting_rows(8, 4)


# ---------------------------------------------------------------------------
# Update order structure
# ---------------------------------------------------------------------------
def test_colour_convention_matches_algorithm_3():
    # Algorithm 3: thread (j, k) (1-based) is red when (j + k) mod 2 == 1
    n = 6
    for j in range(1, n + 1):
        for k in range(1, n + 1):
            idx = (j - 1) * n + (k - 1)
            assert oracle.is_red(2, n, idx) == ((j + k) % 2 == 1)
    order = oracle.checkerboard_order(2, n)
    reds = [oracle.is_red(2, n, i) for i in order]
    assert reds == [True] * 18 + [False] * 18


@pytest.mark.parametrize("dim,n", [(1, 10), (2, 8), (3, 6)])
def test_order_within_a_colour_is_irrelevant_bitwise(dim, n):
    # same-colour points never depend on each other (sec. 4.2), so any order
    # inside the red and inside the blue class gives the bitwise same result
    rng = np.random.default_rng(5)
    grid = Grid(dim, n, 0.0, 2.0, *rng.uniform(0.5, 2.0, 4))
    s0 = rand_state(rng, grid.shape)
    order = oracle.checkerboard_order(dim, n)
    half = n ** dim // 2
    shuffled = np.concatenate([rng.permutation(order[:half]), rng.permutation(order[half:])])
    a = oracle.step(grid, 0.1, s0.copy(), 5)
    b = oracle.step_order(grid, 0.1, s0.copy(), shuffled, 5)
    for x, y in zip(a.arrays(), b.arrays()):
        assert np.array_equal(x, y)


def test_worked_example_neighbour_levels():
    """The 4x4 example of sec. 4.1 (figure fig:ex): with the printed update
    order, U_11 uses only level-n neighbours, U_21 uses U_11^{n+1}, U_33 uses
    U_23^{n+1}, U_32^{n+1}, U_34^n, U_43^n, and U_43 uses U_13^{n+1} through
    the periodic wrap.  The order and the levels are read from tests/golden."""
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "fig_ex_4x4_order.txt")
    lines = [l.split("#")[0].strip() for l in open(path)]
    lines = [l for l in lines if l]
    order_jk = [tuple(int(t) for t in l.split(",")) for l in lines[0].split()]
    expect = {}
    for l in lines[1:]:
        pt, nbs = l.split(":")
        expect[tuple(int(t) for t in pt.split(","))] = [
            (tuple(int(t) for t in nb.split("@")[0].split(",")), nb.split("@")[1]) for nb in nbs.split()]
    n = 4
    lin = lambda jk: (jk[0] - 1) * n + (jk[1] - 1)
    order = np.array([lin(jk) for jk in order_jk])
    rng = np.random.default_rng(1)
    grid = Grid(2, n, 0.0, 4.0, 1.2, 0.8, 0.9, 1.1)
    old = rand_state(rng, grid.shape)
    new = oracle.base_half(grid, 0.2, old.copy(), order)
    for pt, nbs in expect.items():
        i = lin(pt)
        # assemble the state the point sees: neighbours at the printed level,
        # Psi_i at n+1 (solved first), U_i and V_i at level n
        t = old.copy()
        for nb, level in nbs:
            src = new if level == "n+1" else old
            for dst, sa in zip(t.arrays(), src.arrays()):
                dst.ravel()[lin(nb)] = sa.ravel()[lin(nb)]
        t.P.ravel()[i] = new.P.ravel()[i]
        t.Q.ravel()[i] = new.Q.ravel()[i]
        oracle.uv_update(grid, 0.2, t, i)
        assert t.U.ravel()[i] == new.U.ravel()[i] and t.V.ravel()[i] == new.V.ravel()[i], pt
        # and the levels matter: flipping one neighbour's level changes U_i
        nb, level = nbs[0]
        t2 = t.copy()
        t2.U.ravel()[i], t2.V.ravel()[i] = old.U.ravel()[i], old.V.ravel()[i]
        flip = old if level == "n+1" else new
        t2.U.ravel()[lin(nb)] = flip.U.ravel()[lin(nb)]
        oracle.uv_update(grid, 0.2, t2, i)
        assert t2.U.ravel()[i] != new.U.ravel()[i], pt


# ---------------------------------------------------------------------------
# Symmetry: the adjoint composition makes the step time-reversible
# (eq. dp-avfm-adj, dp-comp): step(-tau) is the inverse of step(tau).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", [(1, 32), (2, 16), (3, 8)])
def test_time_reversibility(dim, n):
    p = workloads.gaussian_problem(dim, n, 2, -5.0, 5.0, 0.05, 1)
    grid = Grid(dim, n, p.lo, p.hi, p.kappa1, p.kappa2, p.mu, p.gamma)
    s0 = State.from_fields(p.psi, p.u, p.v)
    s = oracle.step(grid, 0.05, s0.copy(), 20)
    moved = rel_max(s.U, s0.U)
    assert moved > 1e-3
    oracle.step(grid, -0.05, s, 20)
    scale = max(np.max(np.abs(a)) for a in s0.arrays())
    for a, b in zip(s.arrays(), s0.arrays()):
        assert np.max(np.abs(a - b)) <= 1e-13 * scale


# ---------------------------------------------------------------------------
# Special case kappa1 = kappa2 = 0: the points decouple.  The Psi update is
# the midpoint rule for i psi_t + g u psi = 0, a rotation by 2 atan(tau g u/2);
# the (U, V) update is the midpoint (Cayley) rule for u'' + mu^2 u = g|psi|^2,
# a rotation of (mu (u - g|psi|^2/mu^2), v) by 2 atan(mu tau/2).
# ---------------------------------------------------------------------------
def test_decoupled_case_closed_form():
    rng = np.random.default_rng(17)
    mu, g = 1.3, 0.7
    grid = Grid(2, 8, 0.0, 1.0, 0.0, 0.0, mu, g)
    s = rand_state(rng, grid.shape)
    tau, steps = 0.15, 7
    psi, U, V = s.psi.copy(), s.U.copy(), s.V.copy()
    th = tau / 2

    def rot_psi(psi, U):
        return psi * np.exp(2j * np.arctan(th * g * U / 2))

    def rot_uv(psi, U, V):
        F = g * np.abs(psi) ** 2 / mu ** 2
        phi = 2 * np.arctan(mu * th / 2)
        w, v = mu * (U - F), V
        w2 = np.cos(phi) * w + np.sin(phi) * v
        v2 = -np.sin(phi) * w + np.cos(phi) * v
        return w2 / mu + F, v2

    for _ in range(steps):
        psi = rot_psi(psi, U)          # base half: Psi, then (U, V)
        U, V = rot_uv(psi, U, V)
        U, V = rot_uv(psi, U, V)       # adjoint half: (U, V), then Psi
        psi = rot_psi(psi, U)
    oracle.step(grid, tau, s, steps)
    assert rel_max(s.psi, psi) <= 1e-14
    assert rel_max(s.U, U) <= 1e-14
    assert rel_max(s.V, V) <= 1e-14


# ---------------------------------------------------------------------------
# Accuracy: second order in time (symmetric composition, sec. 3.1) and in
# space (central differences, sec. 2).
# ---------------------------------------------------------------------------
def test_linear_plane_wave_second_order_in_time():
    # gamma = 0: psi = e^{i k.x} e^{-i w t} with w = (2 k1/h^2) sum sin^2(k_a h/2)
    # and u = cos(k.x) cos(w_u t), w_u^2 = (4 k2/h^2) sum sin^2(k_a h/2) + mu^2,
    # are exact solutions of the semi-discrete system (eq. kgs-semi).
    n, L = 16, 2 * np.pi
    k1, k2, mu = 1.0, 1.0, 1.0
    grid = Grid(2, n, 0.0, L, k1, k2, mu, 0.0)
    X = workloads.axes(2, n, 0.0, L)
    m = np.array([1, 2])
    ph = m[0] * X[0] + m[1] * X[1]
    h = grid.h
    sn = np.sum(np.sin(m * h / 2) ** 2)
    w = 2 * k1 / h ** 2 * sn
    wu = np.sqrt(4 * k2 / h ** 2 * sn + mu ** 2)
    T = 1.0
    errs = []
    for steps in (40, 80, 160):
        s = State(np.cos(ph), np.sin(ph), np.cos(ph), np.zeros_like(ph))
        oracle.step(grid, T / steps, s, steps)
        e_psi = np.max(np.abs(s.psi - np.exp(1j * (ph - w * T))))
        e_u = np.max(np.abs(s.U - np.cos(ph) * np.cos(wu * T)))
        errs.append(max(e_psi, e_u))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.9) & (orders < 2.1)), (errs, orders)


def soliton(x, t, v=0.5):
    """Exact solitary wave of the 1-D KGS equations for k1 = k2 = mu = g = 1."""
    s = np.sqrt(1 - v * v)
    xi = (x - v * t) / (2 * s)
    sech2 = 1 / np.cosh(xi) ** 2
    psi = (3 * np.sqrt(2) / (4 * s)) * sech2 * np.exp(1j * (v * x + (1 - v * v + v ** 4) * t / (2 * (1 - v * v))))
    u = (3 / (4 * (1 - v * v))) * sech2
    ut = u * 2 * np.tanh(xi) * v / (2 * s)
    return psi, u, ut


def _soliton_error(n, steps, T=1.0):
    grid = Grid(1, n, -40.0, 40.0, 1.0, 1.0, 1.0, 1.0)
    (x,) = workloads.axes(1, n, -40.0, 40.0)
    s = State.from_fields(*soliton(x, 0.0))
    oracle.step(grid, T / steps, s, steps)
    psiT, uT, _ = soliton(x, T)
    # discrete L2 errors as in sec. 5.1: max over Re psi, Im psi, and u
    l2 = lambda f: np.sqrt(grid.h * np.sum(np.abs(f) ** 2))
    return max(l2((s.psi - psiT).real), l2((s.psi - psiT).imag), l2(s.U - uT))


@pytest.mark.slow
def test_soliton_second_order_in_space():
    """Exact solitary wave; h halved with tau ~ h^2 (tau*kappa1/h^2 = 0.04).

    The checkerboard scheme's temporal error grows with tau*kappa1/h^2 (it is
    a red/black splitting of the stencil), so the spatial order is measured
    with tau well inside that range."""
    errs = []
    for n in (128, 256, 512):
        h = 80.0 / n
        steps = int(np.ceil(1.0 / (0.04 * h * h)))
        errs.append(_soliton_error(n, steps))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.9) & (orders < 2.1)), (errs, orders)


def test_soliton_accuracy_and_time_order_on_the_paper_grid():
    # n=512 on [-40, 40): h = 5/32, the error against the exact solution is
    # dominated by space once tau is small; halving tau from 1/80 reduces the
    # temporal part (error minus the spatial floor) by ~4 per halving.
    floor = _soliton_error(512, 2560)
    errs = [_soliton_error(512, s) for s in (160, 320, 640)]
    assert floor < 4e-3
    parts = np.array(errs) - floor
    orders = np.log2(parts[:-1] / parts[1:])
    assert np.all(orders > 1.8), (floor, errs, orders)


def test_finite_speed_of_propagation_lets_sub_blocks_stand_in_for_the_grid():
    """K steps are 2K+1 colour sweeps, and a sweep moves information one
    point along each axis, so the oracle on a periodic sub-block that starts
    from the same data agrees bitwise with the full-grid run wherever the
    sub-block's wrong wrap-around cannot reach (the sampled full-size GPU
    check relies on this); one point closer to the block edge it does
    not."""
    p = workloads.random_problem(3, 48, seed=3, tau=0.04, amp=0.5)
    full = oracle.State.from_fields(p.psi, p.u, p.v)
    oracle.step(oracle.Grid(3, 48, p.lo, p.hi, p.kappa1, p.kappa2, p.mu, p.gamma), p.tau,
                full, 4)
    h = (p.hi - p.lo) / p.n
    for st in [(0, 0, 0), (40, 20, 46), (12, 30, 6)]:
        idx = np.ix_(*[(np.arange(24) + s) % 48 for s in st])
        sub = oracle.State.from_fields(p.psi[idx], p.u[idx], p.v[idx])
        oracle.step(oracle.Grid(3, 24, 0.0, 24 * h, p.kappa1, p.kappa2, p.mu, p.gamma), p.tau,
                    sub, 4)
        safe = (slice(9, 15),) * 3  # at least 9 = 2*4+1 points from the block edge
        for a, b in zip(sub.arrays(), full.arrays()):
            assert np.array_equal(a[safe], b[idx][safe])
        wide = (slice(8, 16),) * 3  # one point closer: the wrap has arrived
        assert any(not np.array_equal(a[wide], b[idx][wide])
                   for a, b in zip(sub.arrays(), full.arrays()))


# ---------------------------------------------------------------------------
# The checkerboard step written colour pass by colour pass (sec. 4.2,
# Algorithm 3): the same scheme as the generic-order step, bitwise, on one
# thread and on many (points of one colour are independent), and its
# float32-storage option as the composition of the pinned half passes with
# numpy's float32 rounding at the stated places.
# ---------------------------------------------------------------------------
def _colour_orders(dim, n):
    order = oracle.checkerboard_order(dim, n)
    half = order.size // 2
    assert all(oracle.is_red(dim, n, int(i)) for i in order[:half])
    return order[:half], order[half:]


@pytest.mark.parametrize("dim,n", [(1, 34), (2, 10), (3, 6)])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_colour_passes_equal_the_checkerboard_step_bitwise(dim, n, threads):
    rng = np.random.default_rng(900 + 10 * dim + threads)
    grid = Grid(dim, n, -2.0, 3.0, *rng.uniform(0.5, 2.0, 4))
    s0 = rand_state(rng, grid.shape, 0.7)
    a = oracle.step(grid, 0.05, s0.copy(), 4)
    b = oracle.step_passes(grid, 0.05, s0.copy(), 4, storage_bits=64, threads=threads)
    for x, y in zip(a.arrays(), b.arrays()):
        assert np.array_equal(x, y)


def _f32(s, pts=None):
    for f in s.arrays():
        flat = f.reshape(-1)
        idx = slice(None) if pts is None else pts
        flat[idx] = flat[idx].astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dim,n", [(1, 34), (2, 10), (3, 6)])
def test_float32_storage_rounds_where_the_state_is_stored(dim, n):
    rng = np.random.default_rng(950 + dim)
    grid = Grid(dim, n, -2.0, 3.0, *rng.uniform(0.5, 2.0, 4))
    tau = 0.05
    s0 = rand_state(rng, grid.shape, 0.7)
    red, blue = _colour_orders(dim, n)
    ref = s0.copy()
    _f32(ref)
    for _ in range(3):
        oracle.base_half(grid, tau / 2, ref, red)
        _f32(ref, red)
        oracle.base_half(grid, tau / 2, ref, blue)
        oracle.adjoint_half(grid, tau / 2, ref, blue)
        _f32(ref, blue)
        oracle.adjoint_half(grid, tau / 2, ref, red)
        _f32(ref, red)
    for threads in (1, 4):
        got = oracle.step_passes(grid, tau, s0.copy(), 3, storage_bits=32, threads=threads)
        for x, y in zip(got.arrays(), ref.arrays()):
            assert np.array_equal(x, y)
    # every stored value is a float32 number, and the state differs from the
    # float64 run only by the storage roundings (a few float32 ulps here)
    for f in got.arrays():
        assert np.array_equal(f, f.astype(np.float32).astype(np.float64))
    exact = oracle.step(grid, tau, s0.copy(), 3)
    for x, y in zip(got.arrays(), exact.arrays()):
        err = np.max(np.abs(x - y)) / np.max(np.abs(y))
        assert 1e-9 < err < 1e-5


def test_colour_passes_reject_odd_n():
    grid = Grid(2, 7, 0.0, 1.0)
    s = rand_state(np.random.default_rng(1), grid.shape)
    with pytest.raises(RuntimeError):
        oracle.step_passes(grid, 0.01, s, 1)
