"""Exact pins of the discrete free energies (``oracle.models``) against their
variational derivatives.

Sec. 5.2 / 5.3 (Eqs. CS_DFT_discrete1-2, CS_PFC_discrete1-2 and Lemmas
CDFT_ineq / PFC_ineq) give the discrete energies F = F_c - F_e and the
discrete gradients dF_c, dF_e whose difference is the chemical potential of
Eq. discrete_c.  The directional derivative of each energy along a direction
eta, d/dt F[rho + t eta] at t = 0, must equal (dF[rho] || eta).  The complex
step F[rho + i eps eta] gives that derivative as Im F / eps with no
cancellation, so the identity holds to rounding: a wrong factor or sign in F,
F_c or F_e (or in the gradients) fails it.  These tie the energies the GPU's
diagnostics are compared with to the gradients that define the scheme.
"""
import numpy as np
import pytest

from oracle import grid, kernel, models

EPS = 1e-30


def pfc_state(n, seed):
    rng = np.random.default_rng(seed)
    rho = 1.5 - 0.07 * np.sqrt(3) + 0.3 * rng.uniform(-1, 1, (n, n))
    eta = rng.standard_normal((n, n))
    return rho, eta


def cdft_state(n, seed):
    rng = np.random.default_rng(seed)
    rho = 6 * 0.6 / np.pi + 0.2 * rng.standard_normal((n, n))
    eta = rng.standard_normal((n, n))
    return rho, eta


@pytest.mark.parametrize("n,h,seed", [(8, 0.5, 0), (16, 0.25, 1), (32, 0.7, 2)])
def test_pfc_energy_derivatives(n, h, seed):
    """d/dt F_c = (phi^3/3 + alpha phi + Delta_h^2 rho || eta),
    d/dt F_e = (-2 Delta_h rho || eta), d/dt F = (dF_c - dF_e || eta)."""
    alpha = 0.975
    rho, eta = pfc_state(n, seed)
    z = rho + 1j * EPS * eta
    for F, dF in [(lambda r: models.pfc_Fc(r, h, alpha), models.pfc_dFc(rho, h, alpha)),
                  (lambda r: models.pfc_Fe(r, h), models.pfc_dFe(rho, h)),
                  (lambda r: models.pfc_F(r, h, alpha),
                   models.pfc_dFc(rho, h, alpha) - models.pfc_dFe(rho, h))]:
        got = np.imag(F(z)) / EPS
        want = grid.ip(dF, eta, h)
        scale = h * h * float(np.sum(np.abs(dF * eta)))
        assert abs(got - want) <= 1e-13 * scale, (got, want)
    assert abs(models.pfc_F(rho, h, alpha) - (models.pfc_Fc(rho, h, alpha) - models.pfc_Fe(rho, h))) \
        <= 1e-13 * abs(models.pfc_Fc(rho, h, alpha))


@pytest.mark.parametrize("n,h,seed", [(8, 17 / 32, 0), (16, 17 / 64, 1), (32, 17 / 128, 2)])
def test_cdft_energy_derivatives(n, h, seed):
    """With J*rho linear in rho (J*(rho + i eps eta) = J*rho + i eps J*eta):
    d/dt F_id = (ln rho || eta), d/dt F_ex = (-J*rho || eta) (J even),
    d/dt F_c = (ln rho + 2 c_e rho || eta), d/dt F_e = (2 c_e rho + J*rho || eta),
    and d/dt F = (dF_c - dF_e || eta)."""
    J = kernel.tabulate(n, h, 2.362)
    ce = kernel.ce(J, h)
    rho, eta = cdft_state(n, seed)
    z = rho + 1j * EPS * eta
    Jz = kernel.conv_fft(J, rho, h) + 1j * EPS * kernel.conv_fft(J, eta, h)
    Jr = kernel.conv_fft(J, rho, h)
    dFc = models.cdft_dFc(rho, ce)
    dFe = models.cdft_dFe(rho, Jr, ce)
    for got_c, dF in [(models.cdft_Fid(z, h), np.log(rho)),
                      (models.cdft_Fex(z, Jz, h), -Jr),
                      (models.cdft_Fc(z, h, ce), dFc),
                      (models.cdft_Fe(z, Jz, h, ce), dFe),
                      (models.cdft_F(z, Jz, h), dFc - dFe)]:
        got = np.imag(got_c) / EPS
        want = grid.ip(dF, eta, h)
        scale = h * h * float(np.sum(np.abs(dF * eta)))
        assert abs(got - want) <= 1e-12 * scale, (got, want)
    F = models.cdft_F(rho, Jr, h)
    assert abs(F - (models.cdft_Fc(rho, h, ce) - models.cdft_Fe(rho, Jr, h, ce))) <= 1e-13 * abs(
        models.cdft_Fc(rho, h, ce))


def test_kinetic_and_mass_derivatives():
    """KE = (rho u || u)/2: d/dt along (eta_rho, eta_u, eta_v) equals
    ((u^2 + v^2)/2 || eta_rho) + (rho u || eta_u) + (rho v || eta_v);
    the mass (rho || 1) is linear with derivative (1 || eta_rho)."""
    rng = np.random.default_rng(4)
    n, h = 16, 0.3
    rho = 1 + 0.1 * rng.standard_normal((n, n))
    u, v = rng.standard_normal((2, n, n))
    er, eu, ev = rng.standard_normal((3, n, n))
    got = np.imag(models.kinetic(rho + 1j * EPS * er, u + 1j * EPS * eu, v + 1j * EPS * ev, h)) / EPS
    want = grid.ip(0.5 * (u * u + v * v), er, h) + grid.ip(rho * u, eu, h) + grid.ip(rho * v, ev, h)
    assert abs(got - want) <= 1e-13 * h * h * float(np.sum(np.abs(rho * u * eu) + np.abs(u * u * er)))
    assert abs(np.imag(models.mass(rho + 1j * EPS * er, h)) / EPS - h * h * er.sum()) < 1e-12


def test_three_d_energy_of_a_z_independent_state():
    """The 3D energy (weight h^3, 7-point Delta_h) of a state independent of z
    with w = 0 equals n h times the 2D energy of its x-y slice: Delta_h has no
    z part there, so E_3D = L_z E_2D with the exactly pinned 2D energy."""
    from oracle import three_d
    n, h, alpha = 8, 0.5, 0.975
    rng = np.random.default_rng(11)
    rho = 1.38 + 0.2 * rng.uniform(-1, 1, (n, n))
    u, v = 0.3 * rng.standard_normal((2, n, n))
    st = three_d.Stepper(n, h, 0.01, alpha)
    rep = lambda f: np.repeat(f[None], n, axis=0)
    st.set_state(rep(rho), rep(u), rep(v), np.zeros((n, n, n)))
    E, ke, F = st.energy()
    F2 = models.pfc_F(rho, h, alpha)
    ke2 = models.kinetic(rho, u, v, h)
    assert abs(F - n * h * F2) <= 1e-13 * abs(n * h * F2) + 1e-13
    assert abs(ke - n * h * ke2) <= 1e-13 * abs(n * h * ke2)
    assert abs(st.mass() - n * h * models.mass(rho, h)) <= 1e-13 * abs(st.mass())


def test_channel_energy_is_half_the_mirrored_periodic_energy():
    """The channel's energy sums the interior rows 1..n-1, and its no-flux wall
    rows copy their neighbours (rho_0 = rho_1, rho_n = rho_{n-1}).  So the
    Laplacian on the interior rows is that of the periodic grid of 2(n - 1)
    rows holding rows 1..n-1 and then the same rows mirrored, and the channel's
    F, KE and mass are half those of that periodic state (2D models, pinned
    above)."""
    from oracle import walls
    n, h, alpha = 16, 0.4, 0.6
    rng = np.random.default_rng(12)
    rho = 0.8 + 0.2 * rng.uniform(-1, 1, (n + 1, n))
    u, v = 0.3 * rng.standard_normal((2, n + 1, n))
    st = walls.Stepper(n, h, 0.02, alpha, u_bot=-0.1, u_top=0.1)
    st.set_state(rho, u, v)
    E, ke, F = st.energy()
    inner = lambda f: f[1:n]
    mirror = lambda f: np.concatenate([inner(f), inner(f)[::-1]], axis=0)
    g = st.g
    F2 = models.pfc_F(mirror(g[0]), h, alpha)
    ke2 = models.kinetic(mirror(g[0]), mirror(g[1]), mirror(g[2]), h)
    assert abs(F - 0.5 * F2) <= 1e-13 * abs(F2)
    assert abs(ke - 0.5 * ke2) <= 1e-13 * abs(ke2)
    assert abs(st.mass() - 0.5 * models.mass(mirror(g[0]), h)) <= 1e-13 * abs(st.mass())
