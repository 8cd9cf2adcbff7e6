"""The hydrodynamic PFC step in three dimensions (Sec. 3 states that the
methods, theorems and proofs carry over to 3D; the paper works in 2D).

TEST INFRASTRUCTURE ONLY (part of the oracle; see the package docstring).

Readings, each the 2D scheme with one more direction:

* Grid n x n x n, periodic, spacing h; arrays f[l, j, i] (x = i fastest,
  then y = j, then z = l).  Unknowns per node g = (rho, u, v, w, mu, kappa).
* Operators: the wide central difference delta_d per direction, the 7-point
  Laplacian Delta_h, grad_h = (delta_x, delta_y, delta_z), and the frozen
  vorticity omega^k = grad_h x u^k, a vector.
* Rows (Eqs. discrete_a-d with the vector form of the advection term,
  -rho^k omega^k x u^{k+1/2}, and u.grad u = omega x u + grad|u|^2 / 2):

    N1 = rho + (s/2) div_h(rho^k u)
    N_u = rho^k u + (s/2) sigma rho^k omega^k x u + (s/2) rho^k grad_h |u|^2
          + s rho^k grad_h mu - (s gamma/2) Delta_h u        (three rows)
    N5 = mu - phi^3/3 - alpha phi - Delta_h kappa,   N6 = kappa - Delta_h rho
    S1 = rho^k - (s/2) div_h(rho^k u^k)
    S_u = rho^k u^k - (s/2) sigma rho^k omega^k x u^k + (s gamma/2) Delta_h u^k
    S5 = 2 Delta_h rho^k,   S6 = 0

  For fields independent of z with w = 0 these are the 2D rows (``system``).
* Smoother: the App. G block solve with the same triangular structure:
  rho^ from row 1, then the 3x3 velocity block (a I + [b x]) u^ = r with
  a = rho^k + 3 s gamma / h^2, b = (s/2) sigma rho^k omega^k, solved by
      u^ = (a^2 r - a (b x r) + (b . r) b) / (a (a^2 + |b|^2)),
  then kappa^ and mu^ (cubic linearised about the current iterate), damping
  w; red-black by (i + j + l) mod 2.
* FAS: 27-point full weighting (the tensor product of (1/4)[1 2 1]),
  trilinear prolongation, coarse levels as in 2D; norm, energy and mass with
  the weight h^3.
"""
from dataclasses import dataclass

import numpy as np

from . import fas


def sh(f, axis, k):
    """f at index + k along axis (periodic)."""
    return np.roll(f, -k, axis=axis)


# axes of a field f[l, j, i]: x -> -1, y -> -2, z -> -3
AX = (-1, -2, -3)


def d(f, a, h):
    """Wide central difference along direction a (0 x, 1 y, 2 z)."""
    return (sh(f, AX[a], 1) - sh(f, AX[a], -1)) / (2.0 * h)


def nsum(f):
    return sum(sh(f, ax, 1) + sh(f, ax, -1) for ax in AX)


def lap(f, h):
    return (nsum(f) - 6.0 * f) / (h * h)


def curl(U, h):
    u, v, w = U
    return np.stack([d(w, 1, h) - d(v, 2, h), d(u, 2, h) - d(w, 0, h), d(v, 0, h) - d(u, 1, h)])


def cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


@dataclass
class Level3:
    h: float
    s: float
    gamma: float
    sigma: float
    alpha: float
    rho_k: np.ndarray
    omega_k: np.ndarray   # (3, n, n, n)
    model: str = "pfc3"

    @property
    def ncomp(self):
        return 6


def N(g, lev):
    h, s, gam, sig = lev.h, lev.s, lev.gamma, lev.sigma
    rk, om = lev.rho_k, lev.omega_k
    rho, U, mu, kap = g[0], g[1:4], g[4], g[5]
    n1 = rho + 0.5 * s * sum(d(rk * U[a], a, h) for a in range(3))
    q = U[0] ** 2 + U[1] ** 2 + U[2] ** 2
    oxu = cross(om, U)
    nu = [rk * U[a] + 0.5 * s * sig * rk * oxu[a] + 0.5 * s * rk * d(q, a, h) + s * rk * d(mu, a, h)
          - 0.5 * s * gam * lap(U[a], h) for a in range(3)]
    phi = rho - 1.5
    n5 = mu - phi ** 3 / 3.0 - lev.alpha * phi - lap(kap, h)
    n6 = kap - lap(rho, h)
    return np.stack([n1] + nu + [n5, n6])


def source(rho0, U0, h, s, gamma, sigma):
    """S and omega^k from the old state."""
    om = curl(U0, h)
    s1 = rho0 - 0.5 * s * sum(d(rho0 * U0[a], a, h) for a in range(3))
    oxu = cross(om, U0)
    su = [rho0 * U0[a] - 0.5 * s * sigma * rho0 * oxu[a] + 0.5 * s * gamma * lap(U0[a], h) for a in range(3)]
    s5 = 2.0 * lap(rho0, h)
    return np.stack([s1] + su + [s5, np.zeros_like(rho0)]), om


def block_solve(g, f, lev):
    """Undamped block solution at every node from the current iterate."""
    h, s, gam, sig = lev.h, lev.s, lev.gamma, lev.sigma
    rk, om = lev.rho_k, lev.omega_k
    rho, U, mu, kap = g[0], g[1:4], g[4], g[5]
    c4 = s / (4.0 * h)
    rho_h = f[0] - c4 * sum(sh(rk * U[a], AX[a], 1) - sh(rk * U[a], AX[a], -1) for a in range(3))
    q = U[0] ** 2 + U[1] ** 2 + U[2] ** 2
    a = rk + 3.0 * s * gam / (h * h)
    b = 0.5 * s * sig * rk * om
    r = np.stack([f[1 + c] - c4 * rk * (sh(q, AX[c], 1) - sh(q, AX[c], -1))
                  - s / (2.0 * h) * rk * (sh(mu, AX[c], 1) - sh(mu, AX[c], -1))
                  + 0.5 * s * gam / (h * h) * nsum(U[c]) for c in range(3)])
    bb = b[0] ** 2 + b[1] ** 2 + b[2] ** 2
    br = b[0] * r[0] + b[1] * r[1] + b[2] * r[2]
    bxr = cross(b, r)
    Uh = (a * a * r - a * bxr + br * b) / (a * (a * a + bb))
    ih2 = 1.0 / (h * h)
    kap_h = f[5] + nsum(rho) * ih2 - 6.0 * rho_h * ih2
    phl = rho - 1.5
    mu_h = (f[4] + (lev.alpha + phl * phl) * (rho_h - 1.5) - (2.0 / 3.0) * phl ** 3
            + nsum(kap) * ih2 - 6.0 * kap_h * ih2)
    return np.stack([rho_h, Uh[0], Uh[1], Uh[2], mu_h, kap_h])


def sweep(g, f, lev, w):
    n = g.shape[-1]
    assert n % 2 == 0
    l, j, i = np.indices(g.shape[-3:])
    par = (i + j + l) % 2
    for colour in (0, 1):
        gs = block_solve(g, f, lev)
        m = par == colour
        g[:, m] = (1.0 - w) * gs[:, m] + w * g[:, m]
    return g


def fw(f, ax):
    return 0.25 * (sh(f, ax, -1) + 2.0 * f + sh(f, ax, 1))


def restrict(f):
    """27-point full weighting onto the coarse nodes (coarse I = fine 2I)."""
    r = fw(fw(fw(f, -1), -2), -3)
    return np.ascontiguousarray(r[..., ::2, ::2, ::2])


def prolong(c):
    """Trilinear interpolation to the fine grid."""
    out = c
    for ax in (-1, -2, -3):
        shp = list(out.shape)
        shp[ax] *= 2
        o = np.empty(shp, dtype=out.dtype)
        sl_even = [slice(None)] * o.ndim
        sl_odd = [slice(None)] * o.ndim
        sl_even[ax] = slice(0, None, 2)
        sl_odd[ax] = slice(1, None, 2)
        o[tuple(sl_even)] = out
        o[tuple(sl_odd)] = 0.5 * (out + sh(out, ax, 1))
        out = o
    return out


class Solver(fas.Solver):
    N = staticmethod(N)
    sweep = staticmethod(sweep)

    def resnorm(self, g, f, lev):
        dd = f - self.N(g, lev)
        return np.sqrt(lev.h ** 3 * float(np.sum(dd * dd)))

    @staticmethod
    def build(h, s, gamma, sigma, alpha, rho_k, omega_k, coarsest_n=4):
        levels = [Level3(h, s, gamma, sigma, alpha, rho_k, omega_k)]
        while levels[-1].rho_k.shape[-1] > coarsest_n:
            f = levels[-1]
            levels.append(Level3(2.0 * f.h, s, gamma, sigma, alpha, restrict(f.rho_k), restrict(f.omega_k)))
        return levels

    def vcycle(self, g, f, l=0):
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            for _ in range(self.coarse_sweeps):
                self.sweep(g, f, lev, self.w)
            return g
        for _ in range(self.nu1):
            self.sweep(g, f, lev, self.w)
        dd = f - self.N(g, lev)
        coarse = self.levels[l + 1]
        g0 = restrict(g)
        fc = self.N(g0, coarse) + restrict(dd)
        gc = self.vcycle(g0.copy(), fc, l + 1)
        g += prolong(gc - g0)
        for _ in range(self.nu2):
            self.sweep(g, f, lev, self.w)
        return g


class Stepper:
    """Time stepper of the 3D PFC step."""

    def __init__(self, n, h, s, alpha, gamma=2.0, w=0.5, tol=1e-10, nu1=2, nu2=2, max_cycles=100,
                 coarsest_n=4, coarse_sweeps=64, sigma=1.0, continuity_fix=True):
        self.n, self.h, self.s, self.alpha = n, h, s, alpha
        self.gamma, self.w, self.tol, self.sigma = gamma, w, tol, sigma
        self.nu1, self.nu2, self.max_cycles = nu1, nu2, max_cycles
        self.coarsest_n, self.coarse_sweeps = coarsest_n, coarse_sweeps
        self.continuity_fix = continuity_fix

    def set_state(self, rho, u, v, w, mu=None, kappa=None):
        rho = np.array(rho, dtype=np.float64)
        if mu is None:
            kappa = lap(rho, self.h)
            phi = rho - 1.5
            mu = phi ** 3 / 3.0 + self.alpha * phi + lap(kappa, self.h) + 2.0 * kappa
        self.g = np.stack([rho, np.asarray(u, float), np.asarray(v, float), np.asarray(w, float), mu, kappa])

    @property
    def rho(self):
        return self.g[0]

    def build_source(self):
        return source(self.g[0], self.g[1:4], self.h, self.s, self.gamma, self.sigma)

    def solver(self, omega_k):
        levels = Solver.build(self.h, self.s, self.gamma, self.sigma, self.alpha, self.g[0], omega_k,
                              self.coarsest_n)
        return Solver(levels, self.w, self.nu1, self.nu2, self.coarse_sweeps)

    def step(self, history=None):
        S, om = self.build_source()
        sol = self.solver(om)
        g = self.g.copy()
        cycles, r = sol.solve(g, S, self.tol, self.max_cycles, history)
        if self.continuity_fix:
            rk = self.g[0]
            g[0] = S[0] - self.s / (4.0 * self.h) * sum(
                sh(rk * g[1 + a], AX[a], 1) - sh(rk * g[1 + a], AX[a], -1) for a in range(3))
        self.g = g
        return cycles, r

    def energy(self):
        """(E, KE, F) with the weight h^3."""
        rho, U = self.g[0], self.g[1:4]
        h3 = self.h ** 3
        phi = rho - 1.5
        L = lap(rho, self.h)
        ke = 0.5 * h3 * float(np.sum(rho * (U[0] ** 2 + U[1] ** 2 + U[2] ** 2)))
        F = h3 * float(np.sum(phi ** 4 / 12.0 + 0.5 * self.alpha * phi ** 2 + 0.5 * L * L + rho * L))
        return ke + F, ke, F

    def mass(self):
        return self.h ** 3 * float(np.sum(self.g[0]))
