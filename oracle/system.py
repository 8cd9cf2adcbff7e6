"""The implicit step as the nonlinear system N(g) = S of App. G.

Unknowns per node (App. G):
  CDFT  g = (rho, u, v)                    (Eqs. MGN_DFT_a-c, MGS_DFT_a-c)
  PFC   g = (rho, u, v, mu, kappa)         (Eqs. MGN_PFC_a-e, MGS_PFC_a-e)

With neighbour shorthand X_E = X_{i+1,j}, X_W = X_{i-1,j}, X_N = X_{i,j+1},
X_S = X_{i,j-1}, frozen coefficients rho^k, omega^k and q = u^2 + v^2:

  N1 = rho + s/(4h) [ (rho^k u)_E - (rho^k u)_W + (rho^k v)_N - (rho^k v)_S ]
  N2 = rho^k u - (s/2) sigma rho^k omega^k v + s/(4h) rho^k (q_E - q_W)
       + s/(2h) rho^k (M_E - M_W) - (s gamma / 2) Delta_h u
  N3 = rho^k v + (s/2) sigma rho^k omega^k u + s/(4h) rho^k (q_N - q_S)
       + s/(2h) rho^k (M_N - M_S) - (s gamma / 2) Delta_h v
  PFC:  M = mu,  N4 = mu - phi^3/3 - alpha phi - Delta_h kappa,
        N5 = kappa - Delta_h rho,  phi = rho - 3/2
  CDFT: M = ln rho + 2 c_e rho   (the implicit part of mu, Lemma CDFT_ineq)

and the source built from the old state (rho^k, u^k, v^k):

  S1 = rho^k - s/(4h) [ (rho^k u^k)_E - (rho^k u^k)_W + (rho^k v^k)_N - (rho^k v^k)_S ]
  S2 = rho^k u^k + (s/2) sigma rho^k omega^k v^k + (s gamma/2) Delta_h u^k
       + s/(2h) rho^k (E_E - E_W)
  S3 = rho^k v^k - (s/2) sigma rho^k omega^k u^k + (s gamma/2) Delta_h v^k
       + s/(2h) rho^k (E_N - E_S)
  PFC:  E = 0,  S4 = 2 Delta_h rho^k,  S5 = 0
  CDFT: E = J*rho^k + 2 c_e rho^k   (the explicit part dF_e[rho^k])

The printed App. G rows carry typos that are corrected here from
Eqs. discrete_a-d: the repeated index in the y-difference of N3
((rho_{i,j-1} - rho_{i,j-1}), (mu_{i,j-1} - mu_{i,j-1})); the sign of the mu
term of MGN_PFC_b, which must match MG_PFC_b; and the vorticity sign, which
App. G prints as sigma = -1 (see ``scheme``).  With sigma = -1 these rows are
the printed ones after those fixes.
"""
from dataclasses import dataclass

import numpy as np

from .grid import curl, east, lap, north, south, west


@dataclass
class Level:
    """Frozen-coefficient operator of one grid level."""
    model: str            # "pfc" or "cdft"
    h: float
    s: float
    gamma: float
    sigma: float
    rho_k: np.ndarray     # rho^k on this level
    omega_k: np.ndarray   # omega^k on this level
    alpha: float = 0.0    # PFC
    ce: float = 0.0       # CDFT (J_e * 1)
    delta: float = 0.0    # CDFT positivity projection parameter

    @property
    def ncomp(self):
        return 5 if self.model == "pfc" else 3


def potential(g, lev):
    """M: the part of mu^{k+1} that depends on the unknowns."""
    if lev.model == "pfc":
        return g[3]
    return np.log(g[0]) + 2.0 * lev.ce * g[0]


def N(g, lev):
    h, s, gam, sig = lev.h, lev.s, lev.gamma, lev.sigma
    rk, om = lev.rho_k, lev.omega_k
    rho, u, v = g[0], g[1], g[2]
    ru, rv = rk * u, rk * v
    q = u * u + v * v
    M = potential(g, lev)
    n1 = rho + s / (4 * h) * (east(ru) - west(ru) + north(rv) - south(rv))
    n2 = (rk * u - 0.5 * s * sig * rk * om * v
          + s / (4 * h) * rk * (east(q) - west(q))
          + s / (2 * h) * rk * (east(M) - west(M))
          - 0.5 * s * gam * lap(u, h))
    n3 = (rk * v + 0.5 * s * sig * rk * om * u
          + s / (4 * h) * rk * (north(q) - south(q))
          + s / (2 * h) * rk * (north(M) - south(M))
          - 0.5 * s * gam * lap(v, h))
    if lev.model == "pfc":
        mu, kap = g[3], g[4]
        phi = rho - 1.5
        n4 = mu - phi ** 3 / 3.0 - lev.alpha * phi - lap(kap, h)
        n5 = kap - lap(rho, h)
        return np.stack([n1, n2, n3, n4, n5])
    return np.stack([n1, n2, n3])


def source(model, rho0, u0, v0, h, s, gamma, sigma, alpha=None, ce=None,
           Jrho0=None):
    """S of App. G and the frozen coefficient omega^k (Eq. MG_DFT_d)."""
    om = curl(u0, v0, h)
    ru, rv = rho0 * u0, rho0 * v0
    s1 = rho0 - s / (4 * h) * (east(ru) - west(ru) + north(rv) - south(rv))
    if model == "pfc":
        E = np.zeros_like(rho0)
    else:
        E = Jrho0 + 2.0 * ce * rho0
    s2 = (rho0 * u0 + 0.5 * s * sigma * rho0 * om * v0 + 0.5 * s * gamma * lap(u0, h)
          + s / (2 * h) * rho0 * (east(E) - west(E)))
    s3 = (rho0 * v0 - 0.5 * s * sigma * rho0 * om * u0 + 0.5 * s * gamma * lap(v0, h)
          + s / (2 * h) * rho0 * (north(E) - south(E)))
    if model == "pfc":
        s4 = 2.0 * lap(rho0, h)
        s5 = np.zeros_like(rho0)
        return np.stack([s1, s2, s3, s4, s5]), om
    return np.stack([s1, s2, s3]), om


def initial_guess_pfc_aux(rho0, h, alpha):
    """mu and kappa consistent with rho^{k+1} = rho^k: kappa = Delta_h rho^k,
    mu = phi^3/3 + alpha phi + Delta_h kappa + 2 Delta_h rho^k (Eqs. MG_PFC_d-e
    evaluated at rho^{k+1} = rho^k).  The paper does not state the starting
    guess of the auxiliary unknowns."""
    phi = rho0 - 1.5
    kap = lap(rho0, h)
    mu = phi ** 3 / 3.0 + alpha * phi + lap(kap, h) + 2.0 * kap
    return mu, kap
