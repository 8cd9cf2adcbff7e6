"""Pins from Thm. thm_energy_stability and its proof (App. F), the convex-splitting
lemmas (Lemmas CDFT_ineq, PFC_ineq) and the linearised closed forms."""
import numpy as np
import pytest

from oracle import grid, kernel, linear, models, newton
from oracle.fas import Stepper


def make(model, n, s, seed=0, tol=1e-12, amp=0.05, uamp=0.05, **kw):
    rng = np.random.default_rng(seed)
    if model == "pfc":
        h = 0.5
        st = Stepper("pfc", n, h, s, alpha=0.975, tol=tol, **kw)
        rho = 1.5 - 0.07 * np.sqrt(3) + amp * rng.uniform(-1, 1, (n, n))
    else:
        h = 17 / 64
        st = Stepper("cdft", n, h, s, nu=2.362, tol=tol, **kw)
        rho = 6 * 0.6 / np.pi + amp * rng.standard_normal((n, n))
    u, v = uamp * rng.standard_normal((2, n, n))
    st.set_state(rho, u, v)
    return st


def energy_terms(st, old, new):
    """KE difference, (rho1 - rho0 || mu1), s gamma (ubar || Delta_h ubar) and F difference."""
    rho0, u0, v0, J0 = old
    rho1, u1, v1, J1 = new
    h, s, gam = st.h, st.s, st.gamma
    mu = st.mu_of(rho1, rho0, J0)
    ke = models.kinetic(rho1, u1, v1, h) - models.kinetic(rho0, u0, v0, h)
    work = grid.ip(rho1 - rho0, mu, h)
    ub, vb = 0.5 * (u0 + u1), 0.5 * (v0 + v1)
    visc = s * gam * (grid.ip(ub, grid.lap(ub, h), h) + grid.ip(vb, grid.lap(vb, h), h))
    if st.model == "pfc":
        dF = models.pfc_F(rho1, h, st.alpha) - models.pfc_F(rho0, h, st.alpha)
    else:
        dF = models.cdft_F(rho1, J1, h) - models.cdft_F(rho0, J0, h)
    return ke, work, visc, dF


def snapshot(st):
    return (st.rho.copy(), st.u.copy(), st.v.copy(),
            None if st.model == "pfc" else st.Jrho.copy())


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_mass_and_energy_identity(model):
    """Mass is conserved to round-off; KE^{k+1} - KE^k + (rho^{k+1} - rho^k || mu^{k+1})
    equals s gamma (u^{k+1/2} || Delta_h u^{k+1/2}) up to the solver tolerance;
    the splitting gap (rho^{k+1} - rho^k || mu^{k+1}) - (F^{k+1} - F^k) is >= 0."""
    st = make(model, 16, 0.02)
    m0 = st.mass()
    for _ in range(4):
        old = snapshot(st)
        E0 = st.energy()[0]
        st.step()
        new = snapshot(st)
        ke, work, visc, dF = energy_terms(st, old, new)
        assert abs(ke + work - visc) < 1e-9
        assert visc < 0
        gap = work - dF
        assert gap > -1e-9
        assert st.energy()[0] <= E0 + 1e-9
        assert abs(st.mass() - m0) < 1e-12 * abs(m0)


@pytest.mark.parametrize("s", [1e-3, 1e-2, 1e-1, 1.0, 10.0, 100.0, 1000.0])
@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_energy_non_increase_any_step(model, s):
    """E^{k+1} <= E^k for any s > 0 (Thm. thm_energy_stability), checked on the
    root found by dense Newton (the FAS smoother of the paper is not meant for
    s/h^4 >> 1; the energy statement is about the scheme's solution)."""
    st = make(model, 8, s, seed=7)
    for _ in range(3):
        E0 = st.energy()[0]
        old = snapshot(st)
        S, om = st.build_source()
        lev = st.solver(om).levels[0]
        g, it, r = newton.solve(st.initial_guess(), S, lev, tol=1e-12)
        assert r < 1e-9, r
        st.rho, st.u, st.v = g[0], g[1], g[2]
        if model == "pfc":
            st.mu, st.kappa = g[3], g[4]
        else:
            st.Jrho = st.conv(st.rho)
        ke, work, visc, dF = energy_terms(st, old, snapshot(st))
        E1 = st.energy()[0]
        assert E1 <= E0 + 1e-9 * max(1.0, abs(E0))
        assert abs(ke + work - visc) < 1e-8 * max(1.0, abs(visc))


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_fas_energy_non_increase(model):
    st = make(model, 32, 0.02 if model == "pfc" else 0.05, seed=3, tol=1e-11)
    E = st.energy()[0]
    for _ in range(5):
        st.step()
        E1 = st.energy()[0]
        assert E1 <= E + 1e-9
        E = E1


def solve_fixed(st, cycles):
    """Run a fixed number of V-cycles on the current step (no stop test)."""
    S, om = st.build_source()
    sol = st.solver(om)
    g = st.initial_guess()
    for _ in range(cycles):
        sol.vcycle(g, S)
    return g[0], g[1], g[2]


def fourier_coeff(f, basis):
    return np.sum(f * basis) / np.sum(basis * basis)


@pytest.mark.parametrize("model,p,q", [("pfc", 4, 1), ("pfc", 3, 3), ("cdft", 1, 0), ("cdft", 2, 1)])
def test_linear_growth_closed_form(model, p, q):
    """One step of a small cosine about the uniform state equals the 2x2
    closed form; the odd part in the amplitude removes O(A^2) terms."""
    n = 16
    if model == "pfc":
        h, s, rb = 0.5, 0.05, 1.5 - 0.07 * np.sqrt(3)
    else:
        h, s, rb = 17 / 16 * 2, 0.02, 6 * 0.6 / np.pi
    A = 1e-4
    L = n * h
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    kx, ky = 2 * np.pi * p / L, 2 * np.pi * q / L
    c, sn = np.cos(kx * X + ky * Y), np.sin(kx * X + ky * Y)
    lam, G = linear.symbols(kx, ky, h)
    gx, gy = np.sin(kx * h) / h, np.sin(ky * h) / h
    out = {}
    for sgn in (1, -1):
        if model == "pfc":
            st = Stepper("pfc", n, h, s, alpha=0.975, coarse_sweeps=60)
        else:
            st = Stepper("cdft", n, h, s, nu=2.362, coarse_sweeps=60)
        st.set_state(rb + sgn * A * c, np.zeros((n, n)), np.zeros((n, n)))
        out[sgn] = solve_fixed(st, 60)
        stp = st
    # odd part
    rho1 = 0.5 * (out[1][0] - out[-1][0])
    u1 = 0.5 * (out[1][1] - out[-1][1])
    v1 = 0.5 * (out[1][2] - out[-1][2])
    r_num = fourier_coeff(rho1, c)
    z_num = (gx * fourier_coeff(u1, sn) + gy * fourier_coeff(v1, sn)) / np.sqrt(G)
    if model == "pfc":
        cc, ce_ = linear.coefficients_pfc(rb, 0.975, lam)
    else:
        Jh = h * h * np.sum(stp.J * np.cos(kx * (np.where(np.arange(n) <= n // 2, np.arange(n), np.arange(n) - n) * h)[None, :]
                                           + ky * (np.where(np.arange(n) <= n // 2, np.arange(n), np.arange(n) - n) * h)[:, None]))
        cc, ce_ = linear.coefficients_cdft(rb, stp.ce, Jh)
    r_ex, z_ex = linear.one_step(A, 0.0, rb, s, stp.gamma, lam, G, cc, ce_)
    assert abs(r_num - r_ex) < 1e-7 * A
    assert abs(z_num - z_ex) < 1e-7 * max(abs(z_ex), A * 1e-3)


def test_shear_decay_crank_nicolson():
    n, h, s, rb, q = 16, 0.5, 0.05, 1.2, 2
    L = n * h
    A = 1e-4
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    prof = np.sin(2 * np.pi * q * Y / L)
    lam_y = 4 / h ** 2 * np.sin(np.pi * q * h / L) ** 2
    res = {}
    for sgn in (1, -1):
        st = Stepper("pfc", n, h, s, alpha=0.975)
        st.set_state(np.full((n, n), rb), sgn * A * prof, np.zeros((n, n)))
        res[sgn] = solve_fixed(st, 60)[1]
    u1 = 0.5 * (res[1] - res[-1])
    fac = linear.shear_factor(rb, s, 2.0, lam_y)
    assert np.allclose(u1, fac * A * prof, atol=1e-9 * A)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_symmetry_equivariance(model):
    """A step commutes with a one-cell translation and with a quarter turn
    (x, y) -> (-y, x), (u, v) -> (-v, u)."""
    base = make(model, 16, 0.02, seed=11, tol=1e-12)
    rho, u, v = base.rho.copy(), base.u.copy(), base.v.copy()
    ref = make(model, 16, 0.02, seed=11, tol=1e-12)
    ref.step()

    def rot(f):   # f'(x, y) = f(y, -x): new[j, i] = f[-i, j]
        n = f.shape[0]
        idx = np.arange(n)
        return f[(-idx[None, :]) % n, idx[:, None]]

    t = make(model, 16, 0.02, seed=11, tol=1e-12)
    t.set_state(np.roll(rho, 1, axis=1), np.roll(u, 1, axis=1), np.roll(v, 1, axis=1))
    t.step()
    assert np.allclose(t.rho, np.roll(ref.rho, 1, axis=1), atol=1e-10)
    assert np.allclose(t.u, np.roll(ref.u, 1, axis=1), atol=1e-10)
    r = make(model, 16, 0.02, seed=11, tol=1e-12)
    r.set_state(rot(rho), -rot(v), rot(u))
    r.step()
    assert np.allclose(r.rho, rot(ref.rho), atol=1e-10)
    assert np.allclose(r.u, -rot(ref.v), atol=1e-10)
    assert np.allclose(r.v, rot(ref.u), atol=1e-10)
