"""FAS multigrid for the implicit step and the time stepper (Sec. 6; App. G).

The paper uses "a standard non-linear Full Approximation Scheme" with the
App. G smoother and defers its transfer operators to an earlier paper.  The
choices made here, each the plain reading of what the paper states:

* Nested nodal grids: coarse node I sits on fine node 2I (the same nesting the
  paper's Cauchy error e_ij = rho^h_ij - rho^{h/2}_{2i,2j} uses).  Grid sizes
  halve down to ``coarsest_n`` (4: the centred differences of a 2x2 periodic
  grid vanish identically).
* Restriction R: 9-point full weighting (1/16)[1 2 1; 2 4 2; 1 2 1].
  Prolongation P: bilinear interpolation.
* Coarse operators: the same rows N with h_{l+1} = 2 h_l and frozen
  coefficients rho^k_{l+1} = R rho^k_l, omega^k_{l+1} = R omega^k_l; the
  scalar (J_e * 1) is the same on every level.
* V(nu1, nu2) cycle, FAS coarse problem N_c(g_c) = N_c(R g) + R(f - N(g)),
  correction g <- g + P(g_c - R g).  The coarsest level takes a fixed number of
  sweeps.  CDFT re-applies the positivity projection to rho after the
  coarse-grid correction, the only other place rho is updated.
* Stop when ||S - N(g)||_2 <= tol, with ||d||_2 = (h^2 sum_components sum d^2)^(1/2)
  (the paper's norm, App. E).  The residual is tested before the first cycle.
* After convergence rho^{k+1} is recomputed from the continuity row,
  rho^{k+1} = S1 - s/(4h)[...](u^{k+1}), so that the discrete mass is conserved
  to round-off (App. F) rather than to the solver tolerance.
"""
import numpy as np

from . import kernel as jker
from . import models
from .grid import east, north, south, west
from .smoother import sweep
from .system import Level, N, initial_guess_pfc_aux, source


class NoConvergence(RuntimeError):
    pass


def restrict(f):
    """Full weighting onto the coarse nodes (I = fine 2I)."""
    fw = (4.0 * f + 2.0 * (east(f) + west(f) + north(f) + south(f))
          + east(north(f)) + west(north(f)) + east(south(f)) + west(south(f))) / 16.0
    return np.ascontiguousarray(fw[..., ::2, ::2])


def prolong(c):
    """Bilinear interpolation from the coarse nodes to the fine grid."""
    shp = c.shape[:-2] + (2 * c.shape[-2], 2 * c.shape[-1])
    out = np.empty(shp, dtype=c.dtype)
    ce_, cn = east(c), north(c)
    out[..., ::2, ::2] = c
    out[..., ::2, 1::2] = 0.5 * (c + ce_)
    out[..., 1::2, ::2] = 0.5 * (c + cn)
    out[..., 1::2, 1::2] = 0.25 * (c + ce_ + cn + east(cn))
    return out


def resnorm(g, f, lev):
    d = f - N(g, lev)
    return np.sqrt(lev.h * lev.h * float(np.sum(d * d)))


class Solver:
    """FAS V(nu1, nu2) over a hierarchy of frozen-coefficient levels.

    The level operator and the smoother are the class attributes ``N`` and
    ``sweep`` (the hydrodynamic system and its App. G smoother here; the
    gradient-flow variant substitutes its own)."""

    N = staticmethod(N)
    sweep = staticmethod(sweep)

    def __init__(self, levels, w=0.5, nu1=2, nu2=2, coarse_sweeps=64):
        self.levels = levels
        self.w, self.nu1, self.nu2 = w, nu1, nu2
        self.coarse_sweeps = coarse_sweeps

    @staticmethod
    def build(model, h, s, gamma, sigma, rho_k, omega_k, coarsest_n=4, **kw):
        levels = [Level(model, h, s, gamma, sigma, rho_k, omega_k, **kw)]
        while levels[-1].rho_k.shape[-1] > coarsest_n:
            f = levels[-1]
            levels.append(Level(model, 2.0 * f.h, s, gamma, sigma,
                                restrict(f.rho_k), restrict(f.omega_k), **kw))
        return levels

    def _project(self, g, lev):
        if lev.model == "cdft":
            g[0] = np.sqrt(g[0] * g[0] + lev.delta * lev.delta)

    def resnorm(self, g, f, lev):
        d = f - self.N(g, lev)
        return np.sqrt(lev.h * lev.h * float(np.sum(d * d)))

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
        g0 = restrict(g)
        fc = self.N(g0, coarse) + restrict(d)
        gc = self.vcycle(g0.copy(), fc, l + 1)
        g += prolong(gc - g0)
        self._project(g, lev)
        for _ in range(self.nu2):
            self.sweep(g, f, lev, self.w)
        return g

    def solve(self, g, f, tol, max_cycles, history=None):
        lev = self.levels[0]
        r = self.resnorm(g, f, lev)
        if history is not None:
            history.append(r)
        cycles = 0
        while not (r <= tol):
            if cycles >= max_cycles or not np.isfinite(r):
                raise NoConvergence(f"residual {r:.3e} after {cycles} V-cycles")
            self.vcycle(g, f)
            cycles += 1
            r = self.resnorm(g, f, lev)
            if history is not None:
                history.append(r)
        return cycles, r


class Stepper:
    """Time stepper for Eqs. discrete_a-d with the FAS solve of each step."""

    def __init__(self, model, n, h, s, gamma=2.0, alpha=None, nu=None,
                 delta=1e-10, w=0.5, tol=1e-10, nu1=2, nu2=2, max_cycles=100,
                 coarsest_n=4, coarse_sweeps=64, sigma=1.0, continuity_fix=True):
        assert model in ("pfc", "cdft")
        self.model, self.n, self.h, self.s, self.gamma = model, n, h, s, gamma
        self.alpha, self.nu, self.delta, self.sigma = alpha, nu, delta, sigma
        self.w, self.tol, self.nu1, self.nu2 = w, tol, nu1, nu2
        self.max_cycles, self.coarsest_n = max_cycles, coarsest_n
        self.coarse_sweeps, self.continuity_fix = coarse_sweeps, continuity_fix
        if model == "cdft":
            self.J = jker.tabulate(n, h, nu)
            self.ce = jker.ce(self.J, h)
        else:
            self.J, self.ce = None, 0.0
        self.steps_done = 0

    def conv(self, rho):
        return jker.conv_fft(self.J, rho, self.h)

    def set_state(self, rho, u, v, mu=None, kappa=None):
        self.rho = np.array(rho, dtype=np.float64)
        self.u = np.array(u, dtype=np.float64)
        self.v = np.array(v, dtype=np.float64)
        if self.model == "pfc":
            if mu is None:
                mu, kappa = initial_guess_pfc_aux(self.rho, self.h, self.alpha)
            self.mu = np.array(mu, dtype=np.float64)
            self.kappa = np.array(kappa, dtype=np.float64)
        else:
            self.Jrho = self.conv(self.rho)

    def level_kwargs(self):
        if self.model == "pfc":
            return dict(alpha=self.alpha)
        return dict(ce=self.ce, delta=self.delta)

    def build_source(self):
        """S and omega^k of the current state (App. G)."""
        return source(self.model, self.rho, self.u, self.v, self.h, self.s,
                      self.gamma, self.sigma, alpha=self.alpha, ce=self.ce,
                      Jrho0=None if self.model == "pfc" else self.Jrho)

    def solver(self, omega_k):
        levels = Solver.build(self.model, self.h, self.s, self.gamma, self.sigma,
                              self.rho, omega_k, self.coarsest_n,
                              **self.level_kwargs())
        return Solver(levels, self.w, self.nu1, self.nu2, self.coarse_sweeps)

    def initial_guess(self):
        comps = [self.rho, self.u, self.v]
        if self.model == "pfc":
            comps += [self.mu, self.kappa]
        return np.stack(comps).copy()

    def step(self, history=None):
        S, om = self.build_source()
        sol = self.solver(om)
        g = self.initial_guess()
        cycles, r = sol.solve(g, S, self.tol, self.max_cycles, history)
        if self.continuity_fix:
            g[0] = self.continuity_rho(S, g)
        self.rho, self.u, self.v = g[0].copy(), g[1].copy(), g[2].copy()
        if self.model == "pfc":
            self.mu, self.kappa = g[3].copy(), g[4].copy()
        else:
            self.Jrho = self.conv(self.rho)
        self.steps_done += 1
        return cycles, r

    def continuity_rho(self, S, g):
        """rho^{k+1} from Eq. discrete_a with the converged velocity."""
        h, s = self.h, self.s
        ru, rv = self.rho * g[1], self.rho * g[2]
        return S[0] - s / (4 * h) * (east(ru) - west(ru) + north(rv) - south(rv))

    def energy(self):
        """(E, KE, F) of the current state; for CDFT also (F_id, F_ex)."""
        ke = models.kinetic(self.rho, self.u, self.v, self.h)
        if self.model == "pfc":
            F = models.pfc_F(self.rho, self.h, self.alpha)
            return ke + F, ke, F
        Fid = models.cdft_Fid(self.rho, self.h)
        Fex = models.cdft_Fex(self.rho, self.Jrho, self.h)
        return ke + Fid + Fex, ke, Fid + Fex, Fid, Fex

    def mass(self):
        return models.mass(self.rho, self.h)

    def mu_of(self, rho1, rho0, Jrho0=None):
        """mu^{k+1} = dF_c[rho^{k+1}] - dF_e[rho^k] from the model (Eq. discrete_c)."""
        if self.model == "pfc":
            return models.pfc_dFc(rho1, self.h, self.alpha) - models.pfc_dFe(rho0, self.h)
        return models.cdft_dFc(rho1, self.ce) - models.cdft_dFe(rho0, Jrho0, self.ce)
