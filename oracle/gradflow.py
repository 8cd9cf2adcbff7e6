"""Gradient-flow variant of the convex-splitting scheme (Sec. 5, Thm.
thm_grad, Eq. gradient_scheme), on the grid and with the operators of the
hydrodynamic step.

TEST INFRASTRUCTURE ONLY (part of the oracle; see the package docstring).

The scheme is

  rho^{k+1} - rho^k = s Delta_h ( dF_c[rho^{k+1}] - dF_e[rho^k] ),

with the discrete gradients of the proper convex splittings of Sec. 5.2
(CDFT) and Sec. 5.3 (PFC), ``models``, and the 5-point Delta_h of App. E.
The paper proves mass conservation and unconditional energy decay for it
and gives no discretisation or solver of its own; the readings here reuse
the hydrodynamic step's choices:

* Unknowns per node.  PFC: g = (rho, mu, kappa), kappa = Delta_h rho (the
  auxiliary of App. G that keeps the rows 5-point); CDFT: g = (rho, mu).
* Rows N(g) = S:

    N1 = rho - s Delta_h mu                        S1 = rho^k
    PFC:  N2 = mu - phi^3/3 - alpha phi - Delta_h kappa,  S2 = 2 Delta_h rho^k
          N3 = kappa - Delta_h rho,                       S3 = 0
    CDFT: N2 = mu - ln rho - 2 c_e rho,   S2 = -(J*rho^k + 2 c_e rho^k)

  with phi = rho - 3/2: N2 - S2 = mu - (dF_c[rho] - dF_e[rho^k]) and
  N1 - S1 is the scheme itself.  The PFC rows 2-3 are App. G's rows 4-5.
* Smoother: damped red-black point-block Gauss-Seidel as in App. G, the
  block solved exactly with the local nonlinearity linearised about the
  current iterate (the App. G treatment of the cubic), then damping
  x <- (1 - w) x^ + w x_l; CDFT projects rho^ <- sqrt(rho^2 + delta^2)
  before mu^ is formed from it (Sec. 6).
* FAS, transfers, coarse levels, norm and stop test: those of ``fas``; no
  frozen coefficients (the rows have constant coefficients).
* Initial guess: rho^k, mu^0 = dF_c[rho^k] - dF_e[rho^k], kappa^0 =
  Delta_h rho^k (the auxiliaries consistent with rho^{k+1} = rho^k; a
  uniform state is then an exact fixed point, zero V-cycles).
* After convergence rho^{k+1} = rho^k + s Delta_h mu^{k+1} (row 1 exactly),
  so that the mass is conserved to round-off (the reading the hydrodynamic
  step takes for its continuity row).

With the exact root, (mu^{k+1} || rho^{k+1} - rho^k) = s (mu || Delta_h mu)
= -s h^2 sum |D^+ mu|^2 (summation by parts, App. E), and the convex-splitting
inequality (Lemmas CDFT_ineq, PFC_ineq) bounds F[rho^{k+1}] - F[rho^k] by
that, so F is non-increasing for every s > 0 (the proof of Thm. thm_grad).
"""
from dataclasses import dataclass

import numpy as np

from . import fas
from . import kernel as jker
from . import models
from .grid import lap
from .smoother import colour_mask, nb_sum


@dataclass
class GFLevel:
    """Operator of one grid level of the gradient-flow system."""
    model: str            # "pfc" or "cdft"
    h: float
    s: float
    alpha: float = 0.0    # PFC
    ce: float = 0.0       # CDFT (J_e * 1)
    delta: float = 0.0    # CDFT positivity projection parameter

    @property
    def ncomp(self):
        return 3 if self.model == "pfc" else 2


def N(g, lev):
    """Rows N(g) of the gradient-flow system (module docstring)."""
    h, s = lev.h, lev.s
    rho, mu = g[0], g[1]
    n1 = rho - s * lap(mu, h)
    if lev.model == "pfc":
        kap = g[2]
        phi = rho - 1.5
        n2 = mu - phi ** 3 / 3.0 - lev.alpha * phi - lap(kap, h)
        n3 = kap - lap(rho, h)
        return np.stack([n1, n2, n3])
    n2 = mu - np.log(rho) - 2.0 * lev.ce * rho
    return np.stack([n1, n2])


def source(model, rho0, h, ce=None, Jrho0=None):
    """S of the gradient-flow system from the old density."""
    if model == "pfc":
        return np.stack([rho0, 2.0 * lap(rho0, h), np.zeros_like(rho0)])
    return np.stack([rho0, -(Jrho0 + 2.0 * ce * rho0)])


def initial_guess(model, rho0, h, alpha=None, ce=None, Jrho0=None):
    """(rho^k, dF[rho^k] (, Delta_h rho^k)) with dF = dF_c - dF_e (Sec. 5)."""
    if model == "pfc":
        mu0 = models.pfc_dFc(rho0, h, alpha) - models.pfc_dFe(rho0, h)
        return np.stack([rho0, mu0, lap(rho0, h)])
    mu0 = models.cdft_dFc(rho0, ce) - models.cdft_dFe(rho0, Jrho0, ce)
    return np.stack([rho0, mu0])


def block_solve(g, f, lev):
    """Undamped point-block solution at every node from the current iterate.

    With c = 1/h^2 and sums over the four neighbours, the rows at node P with
    the neighbours held are

      PFC   rho + 4 s c mu          = f1 + s c sum(mu)                 =: b1
            mu - A rho + 4 c kappa  = f2 - 3A/2 - (2/3) phi_l^3 + c sum(kappa) =: b2
            kappa + 4 c rho         = f3 + c sum(rho)                  =: b3
            A = alpha + phi_l^2  (phi^3/3 ~ phi_l^2 phi - (2/3) phi_l^3)
      CDFT  rho + 4 s c mu          = b1
            mu - B rho              = f2 + ln rho_l - 1                 =: b2
            B = 1/rho_l + 2 c_e      (ln rho ~ ln rho_l + (rho - rho_l)/rho_l)

    solved by substitution: PFC rho^ = (b1 - 4sc(b2 - 4c b3)) / (1 + 4sc(A +
    16c^2)), kappa^ = b3 - 4c rho^, mu^ = b2 + A rho^ - 4c kappa^; CDFT
    rho^ = (b1 - 4sc b2)/(1 + 4sc B), projected, mu^ = b2 + B rho^."""
    h, s = lev.h, lev.s
    c = 1.0 / (h * h)
    rho, mu = g[0], g[1]
    b1 = f[0] + s * c * nb_sum(mu)
    if lev.model == "pfc":
        kap = g[2]
        phl = rho - 1.5
        A = lev.alpha + phl * phl
        b2 = f[1] - 1.5 * A - (2.0 / 3.0) * phl ** 3 + c * nb_sum(kap)
        b3 = f[2] + c * nb_sum(rho)
        rho_h = (b1 - 4.0 * s * c * (b2 - 4.0 * c * b3)) / (1.0 + 4.0 * s * c * (A + 16.0 * c * c))
        kap_h = b3 - 4.0 * c * rho_h
        mu_h = b2 + A * rho_h - 4.0 * c * kap_h
        return np.stack([rho_h, mu_h, kap_h])
    B = 1.0 / rho + 2.0 * lev.ce
    b2 = f[1] + np.log(rho) - 1.0
    rho_h = (b1 - 4.0 * s * c * b2) / (1.0 + 4.0 * s * c * B)
    rho_h = np.sqrt(rho_h * rho_h + lev.delta * lev.delta)
    mu_h = b2 + B * rho_h
    return np.stack([rho_h, mu_h])


def sweep(g, f, lev, w):
    """One damped red-black sweep, in place (even nodes, then odd)."""
    n = g.shape[-1]
    assert n % 2 == 0, "red-black ordering needs an even grid"
    par = colour_mask(n)
    for colour in (0, 1):
        gs = block_solve(g, f, lev)
        m = par == colour
        g[:, m] = (1.0 - w) * gs[:, m] + w * g[:, m]
    return g


class Solver(fas.Solver):
    """FAS V(nu1, nu2) on the gradient-flow system."""

    N = staticmethod(N)
    sweep = staticmethod(sweep)

    @staticmethod
    def build(model, h, s, n, coarsest_n=4, **kw):
        levels = [GFLevel(model, h, s, **kw)]
        m = n
        while m > coarsest_n:
            m //= 2
            levels.append(GFLevel(model, levels[-1].h * 2.0, s, **kw))
        return levels


class Stepper:
    """Time stepper of Eq. gradient_scheme with the FAS solve of each step."""

    def __init__(self, model, n, h, s, alpha=None, nu=None, delta=1e-10, w=0.5,
                 tol=1e-10, nu1=2, nu2=2, max_cycles=100, coarsest_n=4,
                 coarse_sweeps=64, continuity_fix=True):
        assert model in ("pfc", "cdft")
        self.model, self.n, self.h, self.s = model, n, h, s
        self.alpha, self.nu, self.delta = alpha, nu, delta
        self.w, self.tol, self.nu1, self.nu2 = w, tol, nu1, nu2
        self.max_cycles, self.coarsest_n = max_cycles, coarsest_n
        self.coarse_sweeps, self.continuity_fix = coarse_sweeps, continuity_fix
        if model == "cdft":
            self.J = jker.tabulate(n, h, nu)
            self.ce = jker.ce(self.J, h)
        else:
            self.J, self.ce = None, 0.0
        self.steps_done = 0
        self.mu = None

    def set_state(self, rho):
        self.rho = np.array(rho, dtype=np.float64)
        self.Jrho = jker.conv_fft(self.J, self.rho, self.h) if self.model == "cdft" else None

    def level_kwargs(self):
        if self.model == "pfc":
            return dict(alpha=self.alpha)
        return dict(ce=self.ce, delta=self.delta)

    def build_source(self):
        return source(self.model, self.rho, self.h, self.ce, self.Jrho)

    def initial_guess(self):
        return initial_guess(self.model, self.rho, self.h, self.alpha, self.ce, self.Jrho)

    def solver(self):
        levels = Solver.build(self.model, self.h, self.s, self.n, self.coarsest_n,
                              **self.level_kwargs())
        return Solver(levels, self.w, self.nu1, self.nu2, self.coarse_sweeps)

    def step(self, history=None):
        S = self.build_source()
        sol = self.solver()
        g = self.initial_guess()
        cycles, r = sol.solve(g, S, self.tol, self.max_cycles, history)
        if self.continuity_fix:
            g[0] = self.rho + self.s * lap(g[1], self.h)
        self.mu = g[1].copy()
        self.rho = g[0].copy()
        if self.model == "cdft":
            self.Jrho = jker.conv_fft(self.J, self.rho, self.h)
        self.steps_done += 1
        return cycles, r

    def free_energy(self):
        """F of the current density (``models``): PFC F; CDFT F_id + F_ex."""
        if self.model == "pfc":
            return models.pfc_F(self.rho, self.h, self.alpha)
        return models.cdft_F(self.rho, self.Jrho, self.h)

    def mass(self):
        return models.mass(self.rho, self.h)
