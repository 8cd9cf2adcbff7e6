"""Damped point-block nonlinear Gauss-Seidel smoother (App. G, Eqs.
MGSM_DFT_a-c, MGSM_PFC_a-e, and "Damped Gauss-Seidel Iteration").

At a node P the rows N1..Nc couple the unknowns of P as follows: N1 holds
rho_P alone (the centred differences skip P); N2, N3 hold (u_P, v_P) through
the diagonal rho^k + 2 s gamma / h^2 and the vorticity term; N5 holds
(kappa_P, rho_P); N4 holds (mu_P, rho_P, kappa_P) with the cubic linearised
about the current iterate, phi^3 ~ 3 phi_l^2 phi - 2 phi_l^3 (App. G).  The
paper's 3x3 and 5x5 block systems solved by Cramer's rule are therefore
block triangular, and the exact block solve is

  rho^   = S1 - s/(4h) [ (rho^k u)_E - (rho^k u)_W + (rho^k v)_N - (rho^k v)_S ]
           (CDFT: rho^ <- sqrt(rho^2 + delta^2), the positivity projection of Sec. 6)
  [a -b; b a] [u^; v^] = [r_u; r_v],   a = rho^k + 2 s gamma/h^2,
           b = (s/2) sigma rho^k omega^k,
           r_u = S2 - s/(4h) rho^k (q_E - q_W) - s/(2h) rho^k (M_E - M_W)
                 + s gamma/(2h^2) (u_E + u_W + u_N + u_S),  r_v likewise in y
  kappa^ = S5 + (rho_E + rho_W + rho_N + rho_S)/h^2 - 4 rho^/h^2
  mu^    = S4 + (alpha + phi_l^2)(rho^ - 3/2) - (2/3) phi_l^3
           + (kappa_E + kappa_W + kappa_N + kappa_S)/h^2 - 4 kappa^/h^2

followed by damping of every component, x <- (1 - w) x^ + w x_l, w = 0.5.
The printed smoother rows differ from this in signs and factors that the
system they smooth fixes (the sign of the rho row's bracket, the missing
factor s in the diagonal, the u-for-v slip in MGSM_PFC_a, the sign of the
3/2 constant in MGSM_PFC_d).

Ordering: red-black.  Nodes with (i + j) even are updated first, from the
current values of their (odd) neighbours, then the odd nodes.  This is the
lexicographic sweep of App. G reordered so that each half-sweep is a
simultaneous update; it needs an even grid size.
"""
import numpy as np

from .grid import east, north, south, west


def nb_sum(f):
    return east(f) + west(f) + north(f) + south(f)


def block_solve(g, f, lev):
    """Undamped block solution at every node from the current iterate g."""
    h, s, gam, sig = lev.h, lev.s, lev.gamma, lev.sigma
    rk, om = lev.rho_k, lev.omega_k
    rho, u, v = g[0], g[1], g[2]
    ru, rv = rk * u, rk * v
    rho_h = f[0] - s / (4 * h) * (east(ru) - west(ru) + north(rv) - south(rv))
    if lev.model == "cdft":
        rho_h = np.sqrt(rho_h * rho_h + lev.delta * lev.delta)
        M = np.log(rho) + 2.0 * lev.ce * rho
    else:
        M = g[3]
    q = u * u + v * v
    a = rk + 2.0 * s * gam / (h * h)
    b = 0.5 * s * sig * rk * om
    r_u = (f[1] - s / (4 * h) * rk * (east(q) - west(q))
           - s / (2 * h) * rk * (east(M) - west(M))
           + s * gam / (2 * h * h) * nb_sum(u))
    r_v = (f[2] - s / (4 * h) * rk * (north(q) - south(q))
           - s / (2 * h) * rk * (north(M) - south(M))
           + s * gam / (2 * h * h) * nb_sum(v))
    det = a * a + b * b
    u_h = (a * r_u + b * r_v) / det
    v_h = (a * r_v - b * r_u) / det
    if lev.model == "cdft":
        return np.stack([rho_h, u_h, v_h])
    kap = g[4]
    kap_h = f[4] + nb_sum(rho) / (h * h) - 4.0 * rho_h / (h * h)
    phl = rho - 1.5
    mu_h = (f[3] + (lev.alpha + phl * phl) * (rho_h - 1.5) - (2.0 / 3.0) * phl ** 3
            + nb_sum(kap) / (h * h) - 4.0 * kap_h / (h * h))
    return np.stack([rho_h, u_h, v_h, mu_h, kap_h])


def colour_mask(n):
    j, i = np.indices((n, n))
    return (i + j) % 2


def sweep(g, f, lev, w):
    """One damped red-black sweep, in place."""
    n = g.shape[-1]
    assert n % 2 == 0, "red-black ordering needs an even grid"
    par = colour_mask(n)
    for colour in (0, 1):
        gs = block_solve(g, f, lev)
        m = par == colour
        g[:, m] = (1.0 - w) * gs[:, m] + w * g[:, m]
    return g
