"""Pins of the oracle's discrete operators (App. E) against closed forms:
Fourier symbols, summation by parts, Green's identities, and the vorticity
identity behind the sign reading of Eq. discrete_b."""
import numpy as np
import pytest

from oracle import grid


def mode(n, h, p, q, phase=0.3):
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    L = n * h
    kx, ky = 2 * np.pi * p / L, 2 * np.pi * q / L
    return kx, ky, X, Y, np.cos(kx * X + ky * Y + phase), np.sin(kx * X + ky * Y + phase)


@pytest.mark.parametrize("n,h,p,q", [(16, 0.3, 1, 2), (32, 0.25, 5, -3), (24, 1.7, 11, 7), (16, 0.5, 8, 0)])
def test_laplacian_symbol(n, h, p, q):
    kx, ky, X, Y, c, s_ = mode(n, h, p, q)
    lam = 4 / h ** 2 * (np.sin(kx * h / 2) ** 2 + np.sin(ky * h / 2) ** 2)
    assert np.allclose(grid.lap(c, h), -lam * c, atol=1e-12 * max(1, lam))


@pytest.mark.parametrize("n,h,p,q", [(16, 0.3, 1, 2), (32, 0.25, 5, -3), (24, 1.7, 11, 7), (16, 0.5, 8, 8)])
def test_gradient_symbol(n, h, p, q):
    kx, ky, X, Y, c, s_ = mode(n, h, p, q)
    gx, gy = np.sin(kx * h) / h, np.sin(ky * h) / h
    assert np.allclose(grid.grad_x(c, h), -gx * s_, atol=1e-13)
    assert np.allclose(grid.grad_y(c, h), -gy * s_, atol=1e-13)
    # the Nyquist mode is invisible to the centred gradient
    if p == n // 2 and q == n // 2:
        assert np.allclose(grid.grad_x(c, h), 0, atol=1e-12)


def test_operators_by_hand():
    """Stencils written out for one node of a small array."""
    rng = np.random.default_rng(1)
    f = rng.standard_normal((6, 6))
    h = 0.7
    j, i = 2, 4
    assert np.isclose(grid.grad_x(f, h)[j, i], (f[j, 5] - f[j, 3]) / (2 * h))
    assert np.isclose(grid.grad_y(f, h)[j, i], (f[3, i] - f[1, i]) / (2 * h))
    assert np.isclose(grid.lap(f, h)[j, i],
                      (f[j, 5] + f[j, 3] + f[3, i] + f[1, i] - 4 * f[j, i]) / h ** 2)
    # periodic wrap at the corner
    assert np.isclose(grid.grad_x(f, h)[0, 0], (f[0, 1] - f[0, 5]) / (2 * h))
    assert np.isclose(grid.lap(f, h)[5, 5],
                      (f[5, 0] + f[5, 4] + f[0, 5] + f[4, 5] - 4 * f[5, 5]) / h ** 2)


def test_summation_by_parts():
    """(grad_h phi || u) = -(phi || div_h u) and Green's identities with periodic
    boundary terms vanishing (App. E, Props. sbp / divergence_thm / green)."""
    rng = np.random.default_rng(2)
    n, h = 20, 0.37
    phi, psi, u, v = rng.standard_normal((4, n, n))
    lhs = grid.ip(grid.grad_x(phi, h), u, h) + grid.ip(grid.grad_y(phi, h), v, h)
    rhs = -grid.ip(phi, grid.div(u, v, h), h)
    assert np.isclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    assert np.isclose(grid.ip(phi, grid.lap(psi, h), h), grid.ip(grid.lap(phi, h), psi, h), rtol=1e-12)
    # Green's first identity: -(phi || Delta_h psi) = h^2 sum over edges D phi D psi
    g1 = h * h * np.sum(grid.Dx(phi, h) * grid.Dx(psi, h) + grid.Dy(phi, h) * grid.Dy(psi, h))
    assert np.isclose(-grid.ip(phi, grid.lap(psi, h), h), g1, rtol=1e-12)
    # discrete divergence theorem: sum of a divergence is zero
    assert abs(grid.ip(grid.div(u, v, h), 1.0, h)) < 1e-12
    # curl of a gradient vanishes
    assert np.allclose(grid.curl(grid.grad_x(phi, h), grid.grad_y(phi, h), h), 0, atol=1e-12)


def vorticity_defect(n, sigma):
    """max | sigma-form (omega x u) + grad|u|^2/2 - (u.grad) u | for a smooth field."""
    L = 2 * np.pi
    h = L / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    u = np.sin(X) * np.cos(2 * Y) + 0.3 * np.cos(Y)
    v = -0.5 * np.cos(X) * np.sin(2 * Y) + 0.2 * np.sin(X + Y)
    om = grid.curl(u, v, h)
    q = u * u + v * v
    cx, cy = -sigma * om * v, sigma * om * u
    ax = cx + 0.5 * grid.grad_x(q, h) - (u * grid.grad_x(u, h) + v * grid.grad_y(u, h))
    ay = cy + 0.5 * grid.grad_y(q, h) - (u * grid.grad_x(v, h) + v * grid.grad_y(v, h))
    return max(np.abs(ax).max(), np.abs(ay).max())


def test_vorticity_sign_reading():
    """Only sigma = +1 makes omega x u + grad|u|^2/2 a consistent (O(h^2))
    approximation of u.grad u; the App. G sign (sigma = -1) leaves an O(1) defect."""
    e1, e2 = vorticity_defect(32, 1.0), vorticity_defect(64, 1.0)
    assert 3.5 < e1 / e2 < 4.5
    assert vorticity_defect(64, -1.0) > 0.1
