"""Pins of the channel (walls in y) oracle, oracle/walls.py: the PFC step with
no-slip moving walls and no-flux density (Sec. 6, sheared-nanocrystal run).

* FAS reaches the root dense Newton finds for the interior unknowns (8 x 9
  nodes), and that root is a fixed point of the wall smoother;
* plane Couette flow (uniform rho, u linear between the wall speeds, v = 0)
  is an exact steady state of the scheme: zero V-cycles, state unchanged;
* Couette start-up: from rest, one step with wall speeds +-U gives, to first
  order in U, the Crank-Nicolson viscous step rho (u^{k+1} - u^k) =
  (s gamma/2) Delta_yy (u^{k+1} + u^k) with the wall values (a tridiagonal
  solve written here from that equation);
* a step commutes with the mirror y -> L - y (v -> -v, walls swapped) and
  with a translation in x;
* with resting walls the energy does not increase, for s from 1e-3 to 1e3
  (the paper's remark that its stability results hold for zero wall speed),
  on the Newton root;
* the nucleate initial condition (workloads.nucleate): the one-mode
  amplitude for eps = 0.4, rho_s = 0.90073 and the hexagon's size and
  position;
* the transfers reproduce linear fields.
"""
import numpy as np
import pytest

import workloads
from oracle import newton, walls


def make(n, s, ub=0.0, ut=0.0, seed=0, amp=0.05, uamp=0.05, tol=1e-12, h=0.5, **kw):
    rng = np.random.default_rng(seed)
    st = walls.Stepper(n, h, s, alpha=0.6, u_bot=ub, u_top=ut, tol=tol, **kw)
    rho = 0.8 + amp * rng.uniform(-1, 1, (n + 1, n))
    u, v = uamp * rng.standard_normal((2, n + 1, n))
    st.set_state(rho, u, v)
    return st


def newton_root(st, S, lev):
    n = st.n

    def op(gi, lev):
        g = np.zeros((5, n + 1, n), dtype=gi.dtype)
        g[:, 1:-1] = gi
        walls.apply_bc(g, st.u_bot, st.u_top)
        return walls.N(g, lev)[:, 1:-1]

    gi, it, r = newton.solve(st.g[:, 1:-1].copy(), S[:, 1:-1], lev, tol=1e-12, op=op)
    g = np.zeros((5, n + 1, n))
    g[:, 1:-1] = gi
    walls.apply_bc(g, st.u_bot, st.u_top)
    return g, r


@pytest.mark.parametrize("ub,ut", [(0.0, 0.0), (-0.1, 0.3)])
def test_fas_reaches_newton_root(ub, ut):
    st = make(8, 0.05, ub, ut, seed=1)
    S, om = st.build_source()
    sol = st.solver(om)
    lev = sol.levels[0]
    gn, r = newton_root(st, S, lev)
    assert r < 1e-12
    g = st.g.copy()
    sol.solve(g, S, 1e-12, 100)
    assert np.abs(g - gn).max() < 1e-10
    gs = gn.copy()
    walls.sweep(gs, S, lev, 0.5)
    assert np.abs(gs - gn).max() < 1e-11


@pytest.mark.parametrize("U", [0.1, 0.5])
def test_couette_flow_is_a_steady_state(U):
    n, h = 16, 0.5
    st = walls.Stepper(n, h, 0.02, alpha=0.6, u_bot=-U, u_top=U)
    y = np.arange(n + 1) * h
    u = np.repeat((-U + 2 * U * y / (n * h))[:, None], n, axis=1)
    st.set_state(np.full((n + 1, n), 0.85), u, np.zeros((n + 1, n)))
    g0 = st.g.copy()
    cycles, r = st.step()
    assert cycles == 0 and r < 1e-13
    assert np.abs(st.g - g0).max() < 1e-14


def test_couette_start_up_is_crank_nicolson():
    n, h, s, gam, rb, U = 16, 0.5, 0.05, 2.0, 0.85, 1e-4
    out = {}
    for sgn in (1, -1):
        st = walls.Stepper(n, h, s, alpha=0.6, u_bot=-sgn * U, u_top=sgn * U, gamma=gam, tol=1e-13,
                           max_cycles=300)
        st.set_state(np.full((n + 1, n), rb), np.zeros((n + 1, n)), np.zeros((n + 1, n)))
        st.step()
        out[sgn] = st.u.copy()
    u1 = 0.5 * (out[1] - out[-1])
    # from rest: (rho - (s gamma/2) D) u^{k+1} = 2 (s gamma/(2 h^2)) (U_bot e_1 + U_top e_{n-1}),
    # D the second difference on rows 1..n-1, the wall values entering at both time levels
    m = n - 1
    D = (np.diag(-2.0 * np.ones(m)) + np.diag(np.ones(m - 1), 1) + np.diag(np.ones(m - 1), -1)) / h ** 2
    A = rb * np.eye(m) - 0.5 * s * gam * D
    b = np.zeros(m)
    b[0], b[-1] = -U, U
    prof = np.linalg.solve(A, 2.0 * (0.5 * s * gam / h ** 2) * b)
    assert np.allclose(u1[1:-1], prof[:, None], atol=1e-7 * U, rtol=0), np.abs(u1[1:-1] - prof[:, None]).max() / U
    assert np.abs(u1[0] + U).max() == 0.0 and np.abs(u1[-1] - U).max() == 0.0


def test_mirror_and_translation_equivariance():
    n = 16
    base = make(n, 0.05, -0.2, 0.1, seed=7)
    rho, u, v = base.rho.copy(), base.u.copy(), base.v.copy()
    base.step()
    m = make(n, 0.05, 0.1, -0.2, seed=7)
    m.set_state(rho[::-1], u[::-1], -v[::-1])
    m.step()
    assert np.allclose(m.rho, base.rho[::-1], atol=1e-11)
    assert np.allclose(m.u, base.u[::-1], atol=1e-11)
    assert np.allclose(m.v, -base.v[::-1], atol=1e-11)
    t = make(n, 0.05, -0.2, 0.1, seed=7)
    t.set_state(np.roll(rho, 3, axis=1), np.roll(u, 3, axis=1), np.roll(v, 3, axis=1))
    t.step()
    assert np.allclose(t.rho, np.roll(base.rho, 3, axis=1), atol=1e-10)
    assert np.allclose(t.u, np.roll(base.u, 3, axis=1), atol=1e-10)


@pytest.mark.parametrize("s", [1e-3, 1e-1, 1.0, 10.0, 100.0, 1000.0])
def test_energy_non_increase_with_resting_walls(s):
    st = make(8, s, seed=5)
    for _ in range(3):
        E0 = st.energy()[0]
        S, om = st.build_source()
        g, r = newton_root(st, S, st.solver(om).levels[0])
        assert r < 1e-9
        st.g = g
        assert st.energy()[0] <= E0 + 1e-10 * max(1.0, abs(E0))


def test_nucleate_initial_condition():
    n, h = 256, workloads.NANO_H
    rho = workloads.nucleate(n, h, 0.4, workloads.NANO_RHO_S, workloads.NANO_RHO_L)
    assert rho.shape == (n + 1, n)
    a = 4 * np.pi / np.sqrt(3)
    R = 6.5 * a
    L = n * h
    x = np.arange(n) * h
    y = np.arange(n + 1) * h
    X, Y = np.meshgrid(x, y)
    # one-mode amplitude of Sec. 6 at eps = 0.4, rho_s = 0.90073
    dp = workloads.NANO_RHO_S - 1.5
    A = 4 / (5 * np.sqrt(3)) * dp - 4 * np.sqrt(3) / 15 * np.sqrt(6.0 - 12 * dp * dp)
    assert abs(A - (-0.877323)) < 1e-5
    # outside the hexagon's circumscribed circle: liquid; near the centre: the solid formula
    far = np.hypot(X - L / 2, Y - L / 2) > R + h
    assert np.all(rho[far] == workloads.NANO_RHO_L)
    near = np.hypot(X - L / 2, Y - L / 2) < np.sqrt(3) / 2 * R - h
    solid = workloads.NANO_RHO_S + A * (np.cos(np.sqrt(3) / 2 * X + np.pi) * np.cos(Y / 2) - 0.5 * np.cos(Y))
    assert np.allclose(rho[near], solid[near])
    # the hexagon's area (3 sqrt3 / 2) R^2 in nodes, to the boundary's rounding
    inside = np.sum(rho != workloads.NANO_RHO_L)
    assert abs(inside * h * h / (1.5 * np.sqrt(3) * R * R) - 1) < 0.03


def test_transfers_reproduce_linear_fields():
    """Bilinear prolongation and 9-point full weighting (at the interior coarse
    rows) are exact on fields linear in x and y (x linear within the period,
    away from the periodic seam)."""
    m = 8
    I, J = np.meshgrid(np.arange(m), np.arange(m + 1))
    c = 0.3 + 0.7 * J + 0.2 * I
    f = walls.prolong(c)
    i, j = np.meshgrid(np.arange(2 * m), np.arange(2 * m + 1))
    lin = 0.3 + 0.7 * (j / 2) + 0.2 * (i / 2)
    ok = i < 2 * m - 1
    assert np.allclose(f[ok], lin[ok], atol=1e-14)
    F = 0.3 + 0.7 * j + 0.2 * i
    R = walls.restrict(F.astype(float))
    Ic, Jc = np.meshgrid(np.arange(m), np.arange(m + 1))
    ok = (Jc >= 1) & (Jc <= m - 1) & (Ic >= 1) & (Ic <= m - 2)
    assert np.allclose(R[ok], (0.3 + 0.7 * 2 * Jc + 0.2 * 2 * Ic)[ok], atol=1e-13)
