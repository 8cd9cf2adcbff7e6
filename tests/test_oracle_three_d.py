"""Pins of the 3D oracle (oracle/three_d.py), the PFC step in three dimensions.
The FAS tests use s/h^4 <= 0.16: the damped block smoother of App. G, with
six Laplacian neighbours, diverges in 3D from s/h^4 of about 1 (at h = 0.5).

* a state independent of z with w = 0 steps exactly like the 2D scheme of
  the (separately pinned) 2D oracle, and w stays zero;
* a cyclic rotation of the axes (x, y, z) -> (y, z, x), with the velocity
  components rotated alike, commutes with a step (this carries the x and y
  terms the 2D reduction pins over to z, and fixes the orientation of
  omega x u);
* FAS reaches the root dense Newton finds (4^3 nodes);
* one step of a small cosine about a uniform state equals the 2x2 closed form
  of ``linear`` with the 3D Fourier symbols;
* mass is conserved to round-off and the energy does not increase, for s
  from 1e-3 to 1e3 (Newton root); a uniform state is a fixed point.
"""
import numpy as np
import pytest

from oracle import fas, linear, newton
from oracle import three_d as t3


def make(n, s, seed=0, tol=1e-12, amp=0.05, uamp=0.05, h=0.5, **kw):
    rng = np.random.default_rng(seed)
    st = t3.Stepper(n, h, s, alpha=0.975, tol=tol, **kw)
    rho = 1.5 - 0.07 * np.sqrt(3) + amp * rng.uniform(-1, 1, (n, n, n))
    u, v, w = uamp * rng.standard_normal((3, n, n, n))
    st.set_state(rho, u, v, w)
    return st


def test_z_independent_state_steps_like_2d():
    n, h, s = 8, 0.5, 0.01
    rng = np.random.default_rng(3)
    rho2 = 1.38 + 0.05 * rng.uniform(-1, 1, (n, n))
    u2, v2 = 0.05 * rng.standard_normal((2, n, n))
    st2 = fas.Stepper("pfc", n, h, s, alpha=0.975, tol=1e-12)
    st2.set_state(rho2, u2, v2)
    st3 = t3.Stepper(n, h, s, alpha=0.975, tol=1e-12)
    rep = lambda f: np.repeat(f[None], n, axis=0)
    st3.set_state(rep(rho2), rep(u2), rep(v2), np.zeros((n, n, n)))
    for _ in range(2):
        st2.step()
        st3.step()
        g = st3.g
        # w is zero at the root (the red-black colouring by (i + j + l) mod 2
        # makes the iterates z-dependent on the way there)
        assert np.abs(g[3]).max() < 1e-12
        for f3, f2 in [(g[0], st2.rho), (g[1], st2.u), (g[2], st2.v), (g[4], st2.mu), (g[5], st2.kappa)]:
            assert np.abs(f3 - f2[None]).max() < 1e-9 * max(1.0, np.abs(f2).max())


def rotate(g):
    """(x, y, z) -> (y, z, x): the new field at (x', y', z') = (y, z, x) of the
    old point; arrays f[z, y, x]; velocity (u, v, w) -> (v, w, u)."""
    # new[z', y', x'] = old[z, y, x] with x' = y, y' = z, z' = x: new[x, z, y] = old[z, y, x]
    tr = lambda f: np.transpose(f, (2, 0, 1))
    rho, u, v, w, mu, ka = g
    return np.stack([tr(rho), tr(v), tr(w), tr(u), tr(mu), tr(ka)])


def test_axis_rotation_equivariance():
    n = 8
    a = make(n, 0.01, seed=5)
    g0 = a.g.copy()
    a.step()
    b = make(n, 0.01, seed=5)
    r0 = rotate(g0)
    b.set_state(r0[0], r0[1], r0[2], r0[3], r0[4], r0[5])
    b.step()
    assert np.abs(b.g - rotate(a.g)).max() < 1e-11


def test_fas_reaches_newton_root():
    st = make(4, 0.01, seed=2, coarse_sweeps=8)
    S, om = st.build_source()
    sol = st.solver(om)
    lev = sol.levels[0]
    gn, it, r = newton.solve(st.g.copy(), S, lev, tol=1e-12, op=t3.N)
    assert r < 1e-12
    g = st.g.copy()
    sol.solve(g, S, 1e-12, 400)
    assert np.abs(g - gn).max() < 1e-10
    gs = gn.copy()
    t3.sweep(gs, S, lev, 0.5)
    assert np.abs(gs - gn).max() < 1e-11


@pytest.mark.parametrize("p,q,r", [(1, 0, 0), (1, 1, 1), (2, 1, 0)])
def test_linear_growth_closed_form(p, q, r):
    n, h, s, rb, A = 8, 0.5, 0.05, 1.5 - 0.07 * np.sqrt(3), 1e-4
    L = n * h
    x = np.arange(n) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    k = 2 * np.pi * np.array([p, q, r]) / L
    c = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    sn = np.sin(k[0] * X + k[1] * Y + k[2] * Z)
    lam = 4.0 / h ** 2 * float(np.sum(np.sin(0.5 * k * h) ** 2))
    gvec = np.sin(k * h) / h
    G = float(np.sum(gvec ** 2))
    out = {}
    for sgn in (1, -1):
        st = t3.Stepper(n, h, s, alpha=0.975, coarse_sweeps=60)
        z = np.zeros((n, n, n))
        st.set_state(rb + sgn * A * c, z, z, z)
        S, om = st.build_source()
        sol = st.solver(om)
        g = st.g.copy()
        for _ in range(60):
            sol.vcycle(g, S)
        out[sgn] = g
    g1 = 0.5 * (out[1] - out[-1])
    r_num = np.sum(g1[0] * c) / np.sum(c * c)
    z_num = sum(gvec[a] * np.sum(g1[1 + a] * sn) / np.sum(sn * sn) for a in range(3)) / np.sqrt(G)
    cc, ce_ = linear.coefficients_pfc(rb, 0.975, lam)
    r_ex, z_ex = linear.one_step(A, 0.0, rb, s, 2.0, lam, G, cc, ce_)
    assert abs(r_num - r_ex) < 1e-7 * A
    assert abs(z_num - z_ex) < 1e-7 * max(abs(z_ex), A * 1e-3)


@pytest.mark.parametrize("s", [1e-3, 1e-1, 1.0, 10.0, 100.0, 1000.0])
def test_mass_and_energy_any_step(s):
    st = make(4, s, seed=7)
    for _ in range(2):
        E0, m0 = st.energy()[0], st.mass()
        S, om = st.build_source()
        lev = st.solver(om).levels[0]
        g, it, r = newton.solve(st.g.copy(), S, lev, tol=1e-12, op=t3.N)
        assert r < 1e-9
        st.g = g
        assert st.energy()[0] <= E0 + 1e-9 * max(1.0, abs(E0))
        assert abs(st.mass() - m0) < 1e-9 * abs(m0)


def test_uniform_state_is_a_fixed_point():
    n = 8
    st = t3.Stepper(n, 0.5, 0.05, alpha=0.975)
    z = np.zeros((n, n, n))
    st.set_state(np.full((n, n, n), 1.3), z + 0.1, z - 0.2, z + 0.05)
    g0 = st.g.copy()
    c, r = st.step()
    assert c == 0
    assert np.abs(st.g - g0).max() < 1e-14


def test_transfers_reproduce_linear_fields():
    """Trilinear prolongation and 27-point full weighting are exact on fields
    linear in x, y, z (away from the periodic seam)."""
    m = 6
    L_, J_, I_ = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    c = 0.3 + 0.7 * I_ + 0.2 * J_ - 0.4 * L_
    f = t3.prolong(c)
    l2, j2, i2 = np.meshgrid(np.arange(2 * m), np.arange(2 * m), np.arange(2 * m), indexing="ij")
    lin = 0.3 + 0.7 * i2 / 2 + 0.2 * j2 / 2 - 0.4 * l2 / 2
    ok = (i2 < 2 * m - 1) & (j2 < 2 * m - 1) & (l2 < 2 * m - 1)
    assert np.allclose(f[ok], lin[ok], atol=1e-14)
    F = 0.3 + 0.7 * i2 + 0.2 * j2 - 0.4 * l2
    R = t3.restrict(F.astype(float))
    ok = (I_ >= 1) & (I_ <= m - 2) & (J_ >= 1) & (J_ <= m - 2) & (L_ >= 1) & (L_ <= m - 2)
    assert np.allclose(R[ok], (0.3 + 0.7 * 2 * I_ + 0.2 * 2 * J_ - 0.4 * 2 * L_)[ok], atol=1e-13)
