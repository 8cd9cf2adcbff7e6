"""Discrete free energies and their proper convex splittings.

PFC (Sec. 5.3, Eqs. CS_PFC_discrete, CS_PFC_discrete1-2, Lemma PFC_ineq):
  F   = h^2 sum[ phi^4/12 + (alpha/2) phi^2 + (Delta_h rho)^2 / 2 + rho Delta_h rho ],
        phi = rho - 3/2.  The printed norms lack their powers; the powers are
        the ones that make the stated gradients the gradients of F.
  F_c = h^2 sum[ phi^4/12 + (alpha/2) phi^2 + (Delta_h rho)^2 / 2 ]
  F_e = -(rho || Delta_h rho)
  dF_c = phi^3/3 + alpha phi + Delta_h^2 rho,   dF_e = -2 Delta_h rho

CDFT (Sec. 5.2, Eqs. CS_DFT_discrete, CS_DFT_discrete1-2, Lemma CDFT_ineq):
  F   = (rho || ln rho - 1) - (rho || J*rho) / 2
  F_c = (rho || ln rho - 1) + c_e ||rho||^2,     c_e = (J_e * 1)
  F_e = c_e ||rho||^2 + (rho || J*rho) / 2
  dF_c = ln rho + 2 c_e rho,   dF_e = 2 c_e rho + J*rho

Kinetic energy and total energy (Thm. thm_energy_stability):
  KE = (rho u || u)/2 = h^2 sum rho (u^2 + v^2) / 2,   E = KE + F.
Mass (same theorem): (rho || 1).
"""
import numpy as np

from .grid import ip, lap


# ---------------------------------------------------------------- PFC ------

def pfc_F(rho, h, alpha):
    phi = rho - 1.5
    L = lap(rho, h)
    return ip(phi ** 4 / 12.0 + 0.5 * alpha * phi ** 2 + 0.5 * L * L + rho * L,
              1.0, h)


def pfc_Fc(rho, h, alpha):
    phi = rho - 1.5
    L = lap(rho, h)
    return ip(phi ** 4 / 12.0 + 0.5 * alpha * phi ** 2 + 0.5 * L * L, 1.0, h)


def pfc_Fe(rho, h):
    return -ip(rho, lap(rho, h), h)


def pfc_dFc(rho, h, alpha):
    phi = rho - 1.5
    return phi ** 3 / 3.0 + alpha * phi + lap(lap(rho, h), h)


def pfc_dFe(rho, h):
    return -2.0 * lap(rho, h)


# --------------------------------------------------------------- CDFT ------

def cdft_Fid(rho, h):
    return ip(rho * (np.log(rho) - 1.0), 1.0, h)


def cdft_Fex(rho, Jrho, h):
    return -0.5 * ip(rho, Jrho, h)


def cdft_F(rho, Jrho, h):
    return cdft_Fid(rho, h) + cdft_Fex(rho, Jrho, h)


def cdft_Fc(rho, h, ce):
    return cdft_Fid(rho, h) + ce * ip(rho, rho, h)


def cdft_Fe(rho, Jrho, h, ce):
    return ce * ip(rho, rho, h) + 0.5 * ip(rho, Jrho, h)


def cdft_dFc(rho, ce):
    return np.log(rho) + 2.0 * ce * rho


def cdft_dFe(rho, Jrho, ce):
    return 2.0 * ce * rho + Jrho


# ------------------------------------------------------------- common ------

def kinetic(rho, u, v, h):
    return 0.5 * ip(rho, u * u + v * v, h)


def mass(rho, h):
    return ip(rho, 1.0, h)
