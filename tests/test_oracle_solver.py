"""Pins of the oracle's FAS solve: it reaches the root that dense Newton finds
(the plain definition of the implicit step), the smoother leaves that root
fixed, and the uniform states the scheme must keep are kept."""
import numpy as np
import pytest

from oracle import newton, smoother, system
from oracle.fas import Solver, Stepper, resnorm


def small_stepper(model, n=8, s=0.05, seed=0, tol=1e-13, **kw):
    rng = np.random.default_rng(seed)
    if model == "pfc":
        h = 0.8
        st = Stepper("pfc", n, h, s, alpha=0.6, tol=tol, coarse_sweeps=40, **kw)
        rho = 0.85 + 0.05 * rng.uniform(-1, 1, (n, n))
    else:
        h = 0.7
        st = Stepper("cdft", n, h, s, nu=2.362, tol=tol, coarse_sweeps=40, **kw)
        rho = 1.146 + 0.03 * rng.standard_normal((n, n))
    u, v = 0.05 * rng.standard_normal((2, n, n))
    st.set_state(rho, u, v)
    return st


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_fas_reaches_newton_root(model):
    st = small_stepper(model, continuity_fix=False)
    S, om = st.build_source()
    g0 = st.initial_guess()
    lev = st.solver(om).levels[0]
    gN, it, r = newton.solve(g0, S, lev)
    assert r < 1e-12 and it >= 2
    st.step()
    gF = np.stack([st.rho, st.u, st.v] + ([st.mu, st.kappa] if model == "pfc" else []))
    scale = np.abs(gN).max(axis=(1, 2))
    err = np.abs(gF - gN).max(axis=(1, 2)) / np.maximum(scale, 1e-3)
    assert err.max() < 1e-11, err


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_root_is_a_fixed_point_of_the_smoother(model):
    st = small_stepper(model, continuity_fix=False)
    S, om = st.build_source()
    lev = st.solver(om).levels[0]
    gN, _, _ = newton.solve(st.initial_guess(), S, lev)
    g = gN.copy()
    smoother.sweep(g, S, lev, 0.5)
    assert np.abs(g - gN).max() < 1e-11


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_smoother_block_solve_zeroes_its_rows(model):
    """Undamped, the block solve at a node zeroes that node's residual rows
    except the linearised cubic, which it zeroes to first order."""
    st = small_stepper(model, continuity_fix=False)
    S, om = st.build_source()
    lev = st.solver(om).levels[0]
    g = st.initial_guess()
    mask = smoother.colour_mask(g.shape[-1]) == 0
    gs = smoother.block_solve(g, S, lev)
    g1 = g.copy()
    g1[:, mask] = gs[:, mask]
    d = S - system.N(g1, lev)
    rows = [0, 1, 2, 4] if model == "pfc" else [1, 2]
    for r in rows:
        assert np.abs(d[r][mask]).max() < 1e-11, r
    if model == "cdft":   # the projection with delta = 1e-10 is a no-op here
        assert np.abs(d[0][mask]).max() < 1e-11
    else:                 # cubic linearisation error (rho^ - rho_l)^2 (rho^ + 2 rho_l - 9/2)/3
        dr = gs[0] - g[0]
        lin = dr ** 2 * (gs[0] + 2 * g[0] - 4.5) / 3.0
        assert np.allclose(d[3][mask], lin[mask], atol=1e-11)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_uniform_states_are_fixed_points(model):
    n = 16
    if model == "pfc":
        st = Stepper("pfc", n, 0.25, 0.01, alpha=0.975, tol=1e-12)
        rb = 1.3
    else:
        st = Stepper("cdft", n, 17 / 128, 0.02, nu=2.362, tol=1e-12)
        rb = 1.1
    for U, V in [(0.0, 0.0), (0.3, -0.2)]:
        rho = np.full((n, n), rb)
        st.set_state(rho, np.full((n, n), U), np.full((n, n), V))
        cycles, r = st.step()
        assert cycles == 0
        assert np.allclose(st.rho, rb, rtol=1e-15, atol=1e-15)
        assert np.allclose(st.u, U, atol=1e-15) and np.allclose(st.v, V, atol=1e-15)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_vcycle_contracts(model):
    st = small_stepper(model, n=32, s=0.01)
    S, om = st.build_source()
    sol = st.solver(om)
    g = st.initial_guess()
    hist = []
    sol.solve(g, S, 1e-11, 200, hist)
    rates = np.array(hist[2:]) / np.array(hist[1:-1])
    assert len(hist) < 60 and np.median(rates) < 0.7
