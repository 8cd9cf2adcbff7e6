"""Two independent transcriptions of the implicit step agree: the vector form of
Eqs. discrete_a-d (oracle.scheme, built from the App. E operators) and the
App. G system N(g) = S (oracle.system, neighbour-by-neighbour rows)."""
import numpy as np
import pytest

from oracle import grid, kernel, scheme, system


def random_problem(model, n=12, seed=0):
    rng = np.random.default_rng(seed)
    h, s, gamma = 0.4, 0.07, 2.0
    rho0 = 1.2 + 0.1 * rng.uniform(-1, 1, (n, n))
    u0, v0 = 0.2 * rng.standard_normal((2, n, n))
    rho1 = rho0 + 0.05 * rng.standard_normal((n, n))
    u1, v1 = u0 + 0.1 * rng.standard_normal((2, n, n))
    return h, s, gamma, (rho0, u0, v0), (rho1, u1, v1)


@pytest.mark.parametrize("sigma", [1.0, -1.0])
@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_system_equals_scheme(model, sigma):
    h, s, gamma, st0, st1 = random_problem(model, seed=3 if model == "pfc" else 4)
    rho0, u0, v0 = st0
    rho1, u1, v1 = st1
    if model == "pfc":
        alpha = 0.975
        kw = dict(alpha=alpha)
        kap = grid.lap(rho1, h)
        mu = scheme.mu_implicit("pfc", rho1, rho0, h, alpha=alpha)
        g = np.stack([rho1, u1, v1, mu, kap])
        S, om = system.source("pfc", rho0, u0, v0, h, s, gamma, sigma, alpha=alpha)
        lev = system.Level("pfc", h, s, gamma, sigma, rho0, om, alpha=alpha)
        ref = scheme.residual("pfc", st0, st1, h, s, gamma, sigma, alpha=alpha)
    else:
        J = kernel.tabulate(rho0.shape[0], h, 1.3)
        ce = kernel.ce(J, h)
        Jrho0 = kernel.conv_direct(J, rho0, h)
        g = np.stack([rho1, u1, v1])
        S, om = system.source("cdft", rho0, u0, v0, h, s, gamma, sigma, ce=ce, Jrho0=Jrho0)
        lev = system.Level("cdft", h, s, gamma, sigma, rho0, om, ce=ce)
        ref = scheme.residual("cdft", st0, st1, h, s, gamma, sigma, ce=ce, Jrho0=Jrho0)
    d = system.N(g, lev) - S
    scale = np.abs(ref).max()
    assert scale > 1e-3
    assert np.allclose(d[:3], ref, atol=1e-12 * max(1.0, scale))
    if model == "pfc":
        assert np.allclose(d[3:], 0.0, atol=1e-10)


def test_pfc_aux_rows_hold_for_initial_guess():
    """mu, kappa built for rho^{k+1} = rho^k satisfy rows N4, N5 exactly."""
    rng = np.random.default_rng(5)
    n, h, s, gamma, alpha = 8, 0.5, 0.01, 2.0, 0.6
    rho0 = 0.9 + 0.05 * rng.uniform(-1, 1, (n, n))
    z = np.zeros((n, n))
    mu, kap = system.initial_guess_pfc_aux(rho0, h, alpha)
    S, om = system.source("pfc", rho0, z, z, h, s, gamma, 1.0, alpha=alpha)
    lev = system.Level("pfc", h, s, gamma, 1.0, rho0, om, alpha=alpha)
    d = system.N(np.stack([rho0, z, z, mu, kap]), lev) - S
    assert np.allclose(d[3:], 0.0, atol=1e-10)
    assert np.allclose(d[0], 0.0, atol=1e-14)    # no flow: rho row holds too
