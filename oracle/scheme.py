"""The fully discrete scheme, Eqs. discrete_a-d (Sec. 5), in vector form.

Given (rho^k, u^k) and a candidate (rho^{k+1}, u^{k+1}) the residuals are

  r_a = rho^{k+1} - rho^k + s div_h(rho^k u^{k+1/2})
  r_b = rho^k (u^{k+1} - u^k)
        - s[ -rho^k omega^k x u^{k+1/2} - (rho^k/2) grad_h |u^{k+1}|^2
             - rho^k grad_h mu^{k+1} + gamma Delta_h u^{k+1/2} ]
  mu^{k+1} = dF_c[rho^{k+1}] - dF_e[rho^k],   omega^k = curl_h u^k,
  u^{k+1/2} = (u^k + u^{k+1}) / 2   (Eq. u_half).

In two dimensions omega is the z-component of the curl and
omega x u = (-omega v, omega u); this is the form under which the identity
u.grad u = omega x u + grad|u|^2/2 quoted with the semi-discrete scheme
holds.  ``sigma`` multiplies the vorticity term: +1 is that vector form, -1
the component form printed in App. G (Eqs. MG_DFT_b/c, MG_PFC_b/c), which has
the opposite sign.  The scheme is energy stable for either sign because
(omega x u).u = 0.
"""
import numpy as np

from .grid import curl, div, grad_x, grad_y, lap
from . import models


def mu_implicit(model, rho1, rho0, h, alpha=None, ce=None, Jrho0=None):
    """mu^{k+1} = dF_c[rho^{k+1}] - dF_e[rho^k] (Eq. discrete_c)."""
    if model == "pfc":
        return models.pfc_dFc(rho1, h, alpha) - models.pfc_dFe(rho0, h)
    return models.cdft_dFc(rho1, ce) - models.cdft_dFe(rho0, Jrho0, ce)


def residual(model, state0, state1, h, s, gamma, sigma=1.0, alpha=None,
             ce=None, Jrho0=None):
    """Residuals (r_a, r_b, r_c) of Eqs. discrete_a-b for the candidate
    state1 = (rho^{k+1}, u^{k+1}, v^{k+1}) given state0 = (rho^k, u^k, v^k)."""
    rho0, u0, v0 = state0
    rho1, u1, v1 = state1
    ub = 0.5 * (u0 + u1)
    vb = 0.5 * (v0 + v1)
    om = curl(u0, v0, h)
    cross_x = -sigma * om * vb          # (omega x u^{k+1/2})_x
    cross_y = sigma * om * ub           # (omega x u^{k+1/2})_y
    mu = mu_implicit(model, rho1, rho0, h, alpha, ce, Jrho0)
    q = u1 * u1 + v1 * v1
    ra = rho1 - rho0 + s * div(rho0 * ub, rho0 * vb, h)
    rb = rho0 * (u1 - u0) - s * (-rho0 * cross_x - 0.5 * rho0 * grad_x(q, h)
                                 - rho0 * grad_x(mu, h) + gamma * lap(ub, h))
    rc = rho0 * (v1 - v0) - s * (-rho0 * cross_y - 0.5 * rho0 * grad_y(q, h)
                                 - rho0 * grad_y(mu, h) + gamma * lap(vb, h))
    return np.stack([ra, rb, rc])
