"""Pins of the gradient-flow oracle (Thm. thm_grad, Eq. gradient_scheme).

Each check is fixed by the paper or by the mathematics, not by the oracle's
own rows:

* the converged step satisfies Eq. gradient_scheme written directly with the
  discrete gradients dF_c, dF_e of Sec. 5 (``models``: Delta_h^2 rho for PFC,
  a separate transcription from the kappa-row system);
* FAS reaches the root dense Newton finds on 8x8, and that root is a fixed
  point of the block smoother, whose block zeroes the linearised rows;
* one step of a small cosine about a uniform state equals the closed-form
  factor (1 + s lam c_e)/(1 + s lam c_c) (Fourier symbols of App. E, the
  linearised splittings of Lemmas PFC_ineq / CDFT_ineq), above one for the
  CDFT mode the uniform state is unstable to;
* mass is conserved to round-off; (mu || rho^{k+1} - rho^k) equals
  -s h^2 sum |D^+ mu|^2 (summation by parts); F never increases, for s from
  1e-3 to 1e3 (Thm. thm_grad);
* a uniform state is a fixed point (no V-cycles); a step commutes with a
  translation and a quarter turn.
"""
import numpy as np
import pytest

from oracle import gradflow as gf
from oracle import grid, linear, models, newton


def make(model, n, s, seed=0, tol=1e-12, amp=0.05, **kw):
    rng = np.random.default_rng(seed)
    if model == "pfc":
        st = gf.Stepper("pfc", n, 0.5, s, alpha=0.975, tol=tol, **kw)
        rho = 1.5 - 0.07 * np.sqrt(3) + amp * rng.uniform(-1, 1, (n, n))
    else:
        st = gf.Stepper("cdft", n, 17 / 64, s, nu=2.362, tol=tol, **kw)
        rho = 6 * 0.6 / np.pi + amp * rng.standard_normal((n, n))
    st.set_state(rho)
    return st


def dF(st, rho, Jrho=None):
    if st.model == "pfc":
        return models.pfc_dFc(rho, st.h, st.alpha), models.pfc_dFe(rho, st.h)
    return models.cdft_dFc(rho, st.ce), models.cdft_dFe(rho, Jrho, st.ce)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_step_satisfies_the_scheme_directly(model):
    st = make(model, 16, 0.05, tol=1e-12)
    rho0, J0 = st.rho.copy(), None if model == "pfc" else st.Jrho.copy()
    st.step()
    c1 = dF(st, st.rho, st.Jrho)[0]
    e0 = dF(st, rho0, J0)[1]
    r = st.rho - rho0 - st.s * grid.lap(c1 - e0, st.h)
    # the step's rows hold to 1e-13 in the oracle's norm; the direct form
    # multiplies the mu-row residual by s Delta_h (|.| <= 8 s / h^2)
    assert np.abs(r).max() < 1e-10, np.abs(r).max()
    # and mu^{k+1} is dF_c[rho^{k+1}] - dF_e[rho^k]
    assert np.abs(st.mu - (c1 - e0)).max() < 1e-10


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_fas_reaches_newton_root(model):
    st = make(model, 8, 0.1, tol=1e-13)
    S = st.build_source()
    g0 = st.initial_guess()
    lev = st.solver().levels[0]
    gn, it, r = newton.solve(g0, S, lev, op=gf.N)
    assert r < 1e-12
    g = g0.copy()
    st.solver().solve(g, S, 1e-12, 100)
    assert np.abs(g - gn).max() < 1e-11
    # the root is a fixed point of the damped smoother
    gs = gn.copy()
    gf.sweep(gs, S, lev, 0.5)
    assert np.abs(gs - gn).max() < 1e-11


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_block_solve_zeroes_linearised_rows(model):
    """At every node, the block value with the neighbours held satisfies the
    node's rows with the nonlinearity linearised about the current iterate:
    exact for the linear rows, and for the nonlinear row exact once the
    linearisation point is the block value itself (one more solve from it)."""
    st = make(model, 8, 0.1, seed=3)
    S = st.build_source()
    lev = st.solver().levels[0]
    g = st.initial_guess() + 0.01 * np.random.default_rng(4).standard_normal((lev.ncomp, 8, 8))
    if model == "cdft":
        g[0] = np.abs(g[0])
    gh = gf.block_solve(g, S, lev)
    # replace one node of each colour by its block value and check rows 1 (and 3)
    for (j, i) in [(2, 3), (5, 5)]:
        t = g.copy()
        t[:, j, i] = gh[:, j, i]
        R = gf.N(t, lev) - S
        assert abs(R[0, j, i]) < 1e-11 * max(1.0, np.abs(S[0]).max())
        if model == "pfc":
            assert abs(R[2, j, i]) < 1e-11 * max(1.0, np.abs(S[2]).max(), 1 / lev.h ** 2)
    # iterate the node's block solve from its own value: the nonlinear row
    # converges to zero (Newton on the node's rows)
    j, i = 4, 1
    t = g.copy()
    for _ in range(30):
        t[:, j, i] = gf.block_solve(t, S, lev)[:, j, i]
    R = gf.N(t, lev) - S
    assert np.abs(R[:, j, i]).max() < 1e-10


def solve_fixed(st, cycles=60):
    """rho^{k+1} after a fixed number of V-cycles (no stop test), with the
    continuity row applied as in the stepper."""
    S = st.build_source()
    sol = st.solver()
    g = st.initial_guess()
    for _ in range(cycles):
        sol.vcycle(g, S)
    return st.rho + st.s * grid.lap(g[1], st.h)


@pytest.mark.parametrize("model,p,q", [("pfc", 4, 1), ("pfc", 3, 3), ("pfc", 1, 0), ("cdft", 1, 0), ("cdft", 2, 1), ("cdft", 5, 2)])
def test_linear_amplification_closed_form(model, p, q):
    n = 16
    if model == "pfc":
        h, s, rb = 0.5, 0.05, 1.5 - 0.07 * np.sqrt(3)
    else:
        h, s, rb = 17 / 8, 0.02, 6 * 0.6 / np.pi
    A = 1e-4
    L = n * h
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    kx, ky = 2 * np.pi * p / L, 2 * np.pi * q / L
    c = np.cos(kx * X + ky * Y)
    lam, _ = linear.symbols(kx, ky, h)
    out = {}
    for sgn in (1, -1):
        if model == "pfc":
            st = gf.Stepper("pfc", n, h, s, alpha=0.975)
        else:
            st = gf.Stepper("cdft", n, h, s, nu=2.362)
        st.set_state(rb + sgn * A * c)
        out[sgn] = solve_fixed(st)
        stp = st
    rho1 = 0.5 * (out[1] - out[-1])
    r_num = np.sum(rho1 * c) / np.sum(c * c)
    if model == "pfc":
        cc, ce_ = linear.coefficients_pfc(rb, 0.975, lam)
    else:
        off = np.where(np.arange(n) <= n // 2, np.arange(n), np.arange(n) - n) * h
        Jh = h * h * np.sum(stp.J * np.cos(kx * off[None, :] + ky * off[:, None]))
        cc, ce_ = linear.coefficients_cdft(rb, stp.ce, Jh)
    fac = linear.gf_factor(s, lam, cc, ce_)
    assert abs(r_num - fac * A) < 1e-7 * A, (r_num / A, fac)
    # the mode keeps its shape
    assert np.abs(rho1 - r_num * c).max() < 1e-7 * A
    if model == "cdft":
        # 1 - rho_bar Jhat(k) < 0 exactly on the unstable band of the liquid
        assert (fac > 1.0) == (1.0 - rb * Jh < 0.0)
        assert (p, q) != (5, 2) or fac > 1.0


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_mass_and_dissipation_identity(model):
    st = make(model, 16, 0.1)
    m0 = st.mass()
    rho0 = st.rho.copy()
    F0 = st.free_energy()
    st.step()
    assert abs(st.mass() - m0) <= 1e-14 * abs(m0) * 16
    mu, h = st.mu, st.h
    work = grid.ip(mu, st.rho - rho0, h)
    diss = -st.s * h * h * float(np.sum(grid.Dx(mu, h) ** 2 + grid.Dy(mu, h) ** 2))
    assert abs(work - diss) <= 1e-10 * abs(diss)
    # the convex-splitting inequality: F^{k+1} - F^k <= (mu || rho^{k+1} - rho^k)
    assert st.free_energy() - F0 <= work + 1e-10 * abs(work)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
@pytest.mark.parametrize("s", [1e-3, 1e-1, 1.0, 1e1, 1e2, 1e3])
def test_energy_non_increase_any_step(model, s):
    """F^{k+1} <= F^k for any s > 0 (Thm. thm_grad), on the root dense Newton
    finds on 8x8 (the damped smoother is not meant for s/h^4 >> 1; the
    statement is about the scheme's solution), with the dissipation identity."""
    st = make(model, 8, s, seed=5)
    lev = st.solver().levels[0]
    for _ in range(3):
        F0, rho0 = st.free_energy(), st.rho.copy()
        g, it, r = newton.solve(st.initial_guess(), st.build_source(), lev, tol=1e-12, op=gf.N)
        assert r < 1e-9, r
        st.set_state(rho0 + s * grid.lap(g[1], st.h))
        work = grid.ip(g[1], st.rho - rho0, st.h)
        diss = -s * st.h ** 2 * float(np.sum(grid.Dx(g[1], st.h) ** 2 + grid.Dy(g[1], st.h) ** 2))
        assert abs(work - diss) <= 1e-9 * max(1.0, abs(diss))
        assert st.free_energy() <= F0 + 1e-9 * max(1.0, abs(F0))


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_uniform_state_is_a_fixed_point(model):
    st = make(model, 16, 0.1, amp=0.0)
    rho0 = st.rho.copy()
    cycles, r = st.step()
    assert cycles == 0 and r <= 1e-12
    assert np.abs(st.rho - rho0).max() < 1e-14


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_symmetry_equivariance(model):
    base = make(model, 16, 0.05, seed=7)
    rho = base.rho.copy()
    base.step()

    def rot(f):
        n = f.shape[0]
        idx = np.arange(n)
        return f[(-idx[None, :]) % n, idx[:, None]]

    t = make(model, 16, 0.05, seed=7)
    t.set_state(np.roll(rho, 1, axis=1))
    t.step()
    assert np.allclose(t.rho, np.roll(base.rho, 1, axis=1), atol=1e-11)
    r = make(model, 16, 0.05, seed=7)
    r.set_state(rot(rho))
    r.step()
    assert np.allclose(r.rho, rot(base.rho), atol=1e-11)
