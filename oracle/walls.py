"""The hydrodynamic PFC step in a channel: periodic in x, walls in y (Sec. 6,
the sheared-nanocrystal run; App. E, boundary conditions).

TEST INFRASTRUCTURE ONLY (part of the oracle; see the package docstring).

Readings (the paper states the wall conditions of its flow run and the
ghost-point forms of App. E, not a discretisation around them):

* Grid.  x is periodic with n nodes (i = 0..n-1); y has the node rows
  j = 0..n, the walls at j = 0 (y = 0) and j = n (y = L = n h).  The unknowns
  live on the interior rows 1..n-1; fields are stored with all n + 1 rows,
  shape (n + 1, n), the wall rows holding the boundary values.
* Wall rows.  No-slip moving walls: u = u_wall,0 at j = 0 and u_wall,n at j = n,
  v = 0 (Sec. 6).  No flux for the density: rho_{i,0} = rho_{i,1},
  rho_{i,n} = rho_{i,n-1} (Sec. 6); the same copy for the PFC auxiliaries mu
  and kappa (the paper is silent; homogeneous Neumann, the App. E condition
  for which its results carry over) and for the frozen rho^k.  omega^k is
  needed only at interior nodes (it reads the wall velocity).
* Rows.  N(g) and S at interior rows are those of the periodic system
  (``system``) evaluated on the (n + 1)-row arrays: every interior row's
  neighbours are rows of the array (the wall rows at j = 1 and j = n - 1),
  so a periodic shift in y changes only the results on the wall rows, which
  are discarded (set to zero here).
* Smoother.  The App. G damped point-block Gauss-Seidel on interior nodes,
  red-black; after every half sweep the wall rows are refreshed from the
  current iterate, so the next colour reads the boundary values of the
  current iterate.
* FAS.  Nested vertex grids: coarse row J is fine row 2J, the wall rows are
  wall rows on every level (coarse sizes n/2 x (n/2 + 1)).  R g, R d, R rho^k,
  R omega^k by 9-point full weighting at the interior coarse rows (their
  footprints lie on fine rows 1..n-1); the coarse wall rows follow the same
  boundary rules (for R g as for the iterate), so the coarse correction
  g_c - R g is zero on the walls for u, v and equals its first interior
  row's for rho, mu, kappa; bilinear prolongation of it to the interior fine
  rows, then the wall rows refreshed.
* Norm, energy, mass: sums over the interior rows.
* After convergence rho^{k+1} is recomputed from the continuity row at the
  interior rows (as the periodic step does), then the wall rows refreshed.

Only the PFC model: the CDFT convolution is periodic by construction.
"""
from dataclasses import dataclass

import numpy as np

from . import fas
from . import smoother
from . import system
from .grid import east, lap, north, south, west


@dataclass
class WallLevel(system.Level):
    """A periodic-system level plus the wall velocities; arrays have n + 1 rows."""
    u_bot: float = 0.0
    u_top: float = 0.0


def apply_bc(g, u_bot, u_top):
    """Wall rows of an iterate (rho, u, v, mu, kappa), in place."""
    for c in (0, 3, 4):
        g[c, 0] = g[c, 1]
        g[c, -1] = g[c, -2]
    g[1, 0], g[1, -1] = u_bot, u_top
    g[2, 0], g[2, -1] = 0.0, 0.0
    return g


def neumann_rows(f):
    """Wall rows of a no-flux field (rho^k): copies of the adjacent rows."""
    f = f.copy()
    f[0], f[-1] = f[1], f[-2]
    return f


def interior(a):
    """Zeroes the wall rows (the rows are not equations there)."""
    a = a.copy()
    a[..., 0, :] = 0.0
    a[..., -1, :] = 0.0
    return a


def N(g, lev):
    """Rows of N(g) at the interior rows (periodic rows on the padded arrays)."""
    return interior(system.N(g, lev))


def source(rho0, u0, v0, h, s, gamma, sigma, alpha, u_bot, u_top):
    """S and omega^k of App. G at the interior rows, from a state whose wall rows
    hold the boundary values (omega^k is returned with zero wall rows)."""
    g = apply_bc(np.stack([rho0, u0, v0, np.zeros_like(rho0), np.zeros_like(rho0)]), u_bot, u_top)
    S, om = system.source("pfc", g[0], g[1], g[2], h, s, gamma, sigma, alpha=alpha)
    return interior(S), interior(om)


def sweep(g, f, lev, w):
    """One damped red-black sweep over the interior nodes, in place; the wall
    rows are refreshed after each half sweep."""
    n = g.shape[-1]
    assert n % 2 == 0
    j, i = np.indices(g.shape[-2:])
    par = (i + j) % 2
    inner = (j > 0) & (j < g.shape[-2] - 1)
    for colour in (0, 1):
        gs = smoother.block_solve(g, f, lev)
        m = (par == colour) & inner
        g[:, m] = (1.0 - w) * gs[:, m] + w * g[:, m]
        apply_bc(g, lev.u_bot, lev.u_top)
    return g


def restrict(f):
    """9-point full weighting onto the coarse nodes (coarse row J = fine row 2J);
    the coarse wall rows come out meaningless and are set by the caller."""
    fw = (4.0 * f + 2.0 * (east(f) + west(f) + north(f) + south(f))
          + east(north(f)) + west(north(f)) + east(south(f)) + west(south(f))) / 16.0
    return np.ascontiguousarray(fw[..., ::2, ::2])


def prolong(c):
    """Bilinear interpolation from coarse (m + 1 rows) to fine (2m + 1 rows)."""
    rows, m = c.shape[-2], c.shape[-1]
    out = np.empty(c.shape[:-2] + (2 * rows - 1, 2 * m), dtype=c.dtype)
    ce_ = east(c)
    out[..., ::2, ::2] = c
    out[..., ::2, 1::2] = 0.5 * (c + ce_)
    out[..., 1::2, ::2] = 0.5 * (c[..., :-1, :] + c[..., 1:, :])
    out[..., 1::2, 1::2] = 0.25 * (c[..., :-1, :] + ce_[..., :-1, :] + c[..., 1:, :] + ce_[..., 1:, :])
    return out


class Solver(fas.Solver):
    """FAS V(nu1, nu2) for the channel (module docstring)."""

    N = staticmethod(N)
    sweep = staticmethod(sweep)

    @staticmethod
    def build(h, s, gamma, sigma, rho_k, omega_k, alpha, u_bot, u_top, coarsest_n=4):
        mk = lambda hh, r, o: WallLevel("pfc", hh, s, gamma, sigma, neumann_rows(r), o,
                                        alpha=alpha, u_bot=u_bot, u_top=u_top)
        levels = [mk(h, rho_k, omega_k)]
        while levels[-1].rho_k.shape[-1] > coarsest_n:
            f = levels[-1]
            levels.append(mk(2.0 * f.h, restrict(f.rho_k), interior(restrict(f.omega_k))))
        return levels

    def vcycle(self, g, f, l=0):
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            for _ in range(self.coarse_sweeps):
                self.sweep(g, f, lev, self.w)
            return g
        for _ in range(self.nu1):
            self.sweep(g, f, lev, self.w)
        d = f - self.N(g, lev)
        coarse = self.levels[l + 1]
        g0 = apply_bc(restrict(g), lev.u_bot, lev.u_top)
        fc = self.N(g0, coarse) + interior(restrict(d))
        gc = self.vcycle(g0.copy(), fc, l + 1)
        e = prolong(gc - g0)
        g[:, 1:-1] += e[:, 1:-1]
        apply_bc(g, lev.u_bot, lev.u_top)
        for _ in range(self.nu2):
            self.sweep(g, f, lev, self.w)
        return g


class Stepper:
    """Time stepper of Eqs. discrete_a-d (PFC) in the channel."""

    def __init__(self, n, h, s, alpha, u_bot=0.0, u_top=0.0, gamma=2.0, w=0.5, tol=1e-10,
                 nu1=2, nu2=2, max_cycles=100, coarsest_n=4, coarse_sweeps=64, sigma=1.0,
                 continuity_fix=True):
        self.n, self.h, self.s, self.alpha = n, h, s, alpha
        self.u_bot, self.u_top = u_bot, u_top
        self.gamma, self.w, self.tol, self.sigma = gamma, w, tol, sigma
        self.nu1, self.nu2, self.max_cycles = nu1, nu2, max_cycles
        self.coarsest_n, self.coarse_sweeps = coarsest_n, coarse_sweeps
        self.continuity_fix = continuity_fix
        self.steps_done = 0

    def set_state(self, rho, u, v, mu=None, kappa=None):
        """Fields of shape (n + 1, n); their wall rows are replaced by the
        boundary values.  mu, kappa default to the values consistent with
        rho^{k+1} = rho^k (``system.initial_guess_pfc_aux``), wall rows copied."""
        g = np.zeros((5,) + np.shape(rho))
        g[0], g[1], g[2] = rho, u, v
        apply_bc(g, self.u_bot, self.u_top)
        if mu is None:
            # kappa = Delta_h rho (wall rows copied before mu reads them), then
            # mu = phi^3/3 + alpha phi + Delta_h kappa + 2 Delta_h rho
            g[4] = lap(g[0], self.h)
            apply_bc(g, self.u_bot, self.u_top)
            phi = g[0] - 1.5
            g[3] = phi ** 3 / 3.0 + self.alpha * phi + lap(g[4], self.h) + 2.0 * g[4]
        else:
            g[3], g[4] = mu, kappa
        apply_bc(g, self.u_bot, self.u_top)
        self.g = g

    @property
    def rho(self):
        return self.g[0]

    @property
    def u(self):
        return self.g[1]

    @property
    def v(self):
        return self.g[2]

    def build_source(self):
        return source(self.g[0], self.g[1], self.g[2], self.h, self.s, self.gamma, self.sigma,
                      self.alpha, self.u_bot, self.u_top)

    def solver(self, omega_k):
        levels = Solver.build(self.h, self.s, self.gamma, self.sigma, self.g[0], omega_k,
                              self.alpha, self.u_bot, self.u_top, self.coarsest_n)
        return Solver(levels, self.w, self.nu1, self.nu2, self.coarse_sweeps)

    def step(self, history=None):
        S, om = self.build_source()
        sol = self.solver(om)
        g = self.g.copy()
        cycles, r = sol.solve(g, S, self.tol, self.max_cycles, history)
        if self.continuity_fix:
            rk = self.g[0]
            ru, rv = rk * g[1], rk * g[2]
            rho1 = S[0] - self.s / (4 * self.h) * (east(ru) - west(ru) + north(rv) - south(rv))
            g[0, 1:-1] = rho1[1:-1]
            apply_bc(g, self.u_bot, self.u_top)
        self.g = g
        self.steps_done += 1
        return cycles, r

    def energy(self):
        """(E, KE, F) summed over the interior rows (the wall rows are boundary
        values, not unknowns)."""
        rho, u, v = self.g[0], self.g[1], self.g[2]
        h = self.h
        phi = rho - 1.5
        L = lap(rho, h)
        ke = 0.5 * h * h * float(np.sum((rho * (u * u + v * v))[1:-1]))
        F = h * h * float(np.sum((phi ** 4 / 12.0 + 0.5 * self.alpha * phi ** 2 + 0.5 * L * L + rho * L)[1:-1]))
        return ke + F, ke, F

    def mass(self):
        return self.h * self.h * float(np.sum(self.g[0][1:-1]))

