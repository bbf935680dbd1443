"""Discretisation error of the oracle on the 2-D example of sec. 5.1,
measured against an independent pseudo-spectral solution of the PDE.

Tab. conv2d prints the errors of DP-AVF2 at three (h, tau) levels with h and
tau halved together.  The table comes from the serial implementation, whose
update order is lexicographic (sec. 4.1); the oracle's generic-order mode
runs that order and must reproduce the table's magnitudes and second-order
decay.  The checkerboard order of sec. 4.2 (the order of the GPU kernels) is
consistent at fixed h but its temporal error constant grows with the mesh
ratio tau kappa1 / h^2; the last test records that behaviour.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
import spectral_reference as sr
from paper_2502_09537_amd import workloads

LO, HI, T_END = -10.0, 10.0, 1.0
REF_N, REF_STEPS = 128, 500
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tab_conv2d_dp_avf2.txt")


def initial_fields(n):
    p = workloads.accuracy_2d((n // 64).bit_length() - 1)
    assert p.n == n and (p.lo, p.hi) == (LO, HI)
    return p.psi, p.u, p.v


def paper_table():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                lvl, _, _, eu, epsi = line.split()
                rows.append((int(lvl), float(eu), float(epsi)))
    return rows


@pytest.fixture(scope="module")
def reference():
    return sr.solve(*initial_fields(REF_N), LO, HI, T_END, REF_STEPS)


def errors(ref, n, steps, order):
    """(Error_u, Error_psi) of the oracle at t = 1 on an n x n grid."""
    g = oracle.Grid(2, n, LO, HI)
    s = oracle.State.from_fields(*initial_fields(n))
    if order == "checkerboard":
        oracle.step(g, T_END / steps, s, steps)
    else:
        oracle.step_order(g, T_END / steps, s, np.arange(n * n), steps)
    if n >= REF_N:
        rp, ru = sr.resample(ref[0], n), sr.resample(ref[1], n)
    else:
        rp, ru = ref[0][::REF_N // n, ::REF_N // n], ref[1][::REF_N // n, ::REF_N // n]
    h = (HI - LO) / n

    def norm(d):
        return float(np.sqrt(h * h * np.sum(d ** 2)))

    return norm(s.U - ru), max(norm(s.P - rp.real), norm(s.Q - rp.imag))


def test_spectral_reference_is_exact_for_linear_plane_waves():
    # gamma = 0 decouples the system into linear Schroedinger and linear
    # Klein-Gordon equations, whose plane waves are exact solutions:
    # psi = exp(i (k.x - kappa1 |k|^2 t / 2)), u = cos(q.x - w t),
    # w^2 = kappa2 |q|^2 + mu^2.
    n, k1, k2, mu = 32, 1.3, 0.7, 1.1
    x = sr.grid_axis(n, LO, HI)
    X, Y = np.meshgrid(x, x, indexing="ij")
    kv = 2 * np.pi / (HI - LO) * np.array([1.0, 2.0])
    qv = 2 * np.pi / (HI - LO) * np.array([3.0, -1.0])
    w = np.sqrt(k2 * qv @ qv + mu * mu)
    ph = kv[0] * X + kv[1] * Y
    qx = qv[0] * X + qv[1] * Y
    p, u, v = sr.solve(np.exp(1j * ph), np.cos(qx), w * np.sin(qx), LO, HI, 1.0, 200,
                       kappa1=k1, kappa2=k2, mu=mu, gamma=0.0)
    assert np.abs(p - np.exp(1j * (ph - 0.5 * k1 * (kv @ kv)))).max() < 1e-9
    assert np.abs(u - np.cos(qx - w)).max() < 1e-9
    assert np.abs(v - w * np.sin(qx - w)).max() < 1e-9


def test_spectral_reference_conserves_mass_and_energy(reference):
    # Both invariants of the continuous system (sec. 2) hold to the accuracy
    # of the time integrator; a sign or factor slip in either coupling term
    # breaks the energy balance.
    psi0, u0, v0 = initial_fields(REF_N)
    h = (HI - LO) / REF_N
    m0 = h * h * np.sum(np.abs(psi0) ** 2)
    m1 = h * h * np.sum(np.abs(reference[0]) ** 2)
    e0 = sr.energy(psi0, u0, v0, LO, HI)
    e1 = sr.energy(*reference, LO, HI)
    assert abs(m1 - m0) / m0 < 1e-9
    assert abs(e1 - e0) / abs(e0) < 1e-9


def test_tab_conv2d_serial_order_reproduces_the_papers_errors(reference):
    table = paper_table()
    ours = [errors(reference, 64 << lvl, 50 << lvl, "lexicographic") for lvl, _, _ in table]
    for (lvl, eu_paper, epsi_paper), (eu, epsi) in zip(table, ours):
        assert 1 / 1.6 < epsi / epsi_paper < 1.6, (lvl, epsi, epsi_paper)
        # The paper's Error_u is within 2% of its Error_psi at every level and
        # for all four schemes of the table; ours is about a third of it.
        # Only the order of magnitude is held here.
        assert 0.2 < eu / eu_paper < 5.0, (lvl, eu, eu_paper)
    eu = np.array([e[0] for e in ours])
    epsi = np.array([e[1] for e in ours])
    for orders in (np.log2(eu[:-1] / eu[1:]), np.log2(epsi[:-1] / epsi[1:])):
        assert np.all((orders > 1.8) & (orders < 2.7)), (ours, orders)


def test_checkerboard_order_accuracy_depends_on_the_mesh_ratio(reference):
    # tau kappa1 / (2 h^2) = 0.10: both orders are about equally accurate.
    cb0, lex0 = errors(reference, 64, 50, "checkerboard"), errors(reference, 64, 50, "lexicographic")
    assert abs(cb0[1] - lex0[1]) < 0.15 * lex0[1]
    # At fixed h, tau -> 0 takes both orders to the same semi-discrete
    # solution (ratio 0.026 here).
    cb1, lex1 = errors(reference, 128, 800, "checkerboard"), errors(reference, 128, 800, "lexicographic")
    assert abs(cb1[1] - lex1[1]) < 0.05 * lex1[1]
    assert abs(cb1[0] - lex1[0]) < 0.05 * lex1[0]
    # On the paper's refinement path the ratio doubles per level; at the
    # third level (0.41) the checkerboard order has lost the accuracy that
    # the serial order keeps.
    cb2, lex2 = errors(reference, 256, 200, "checkerboard"), errors(reference, 256, 200, "lexicographic")
    assert cb2[1] > 0.1 and cb2[1] > 20 * lex2[1], (cb2, lex2)
