"""Closed forms of the scheme linearised about a uniform state.

About rho = rho_bar, u = 0 the vorticity and |u|^2 terms of Eqs.
discrete_a-b are quadratic and drop out.  For a Fourier mode
rho' = r cos(k.x), u' = (g/|g|) z sin(k.x), with the App. E operators acting as

  Delta_h cos(k.x) = -lam cos(k.x),   lam = (4/h^2)[sin^2(k_x h/2) + sin^2(k_y h/2)]
  grad_h cos(k.x)  = -g sin(k.x),     g   = (sin k_x h, sin k_y h)/h,  G = |g|^2,

and the linearised potential mu' = c_c r^{k+1} - c_e r^k (Eq. discrete_c with
dF_c, dF_e linearised), one step is exactly the 2x2 system

  [ 1,                 s rho_bar sqrt(G)/2    ] [r]^{k+1}
  [ -s rho_bar sqrt(G) c_c, rho_bar + s gamma lam/2 ] [z]
      = [ 1,                  -s rho_bar sqrt(G)/2   ] [r]^k
        [ -s rho_bar sqrt(G) c_e, rho_bar - s gamma lam/2 ] [z]

with
  PFC  (Lemma PFC_ineq):  c_c = (rho_bar - 3/2)^2 + alpha + lam^2,  c_e = 2 lam
  CDFT (Lemma CDFT_ineq): c_c = 1/rho_bar + 2 (J_e*1),  c_e = 2 (J_e*1) + Jhat_h(k).

The continuum limit of the growth rate, (eig - 1)/s -> sigma with
sigma^2 + (gamma k^2/rho_bar) sigma + rho_bar k^2 (c_c - c_e) = 0, is unstable
exactly when c_c < c_e; for CDFT that is 1 - rho_bar Jhat(k) < 0 (Sec. 6.2).

The gradient-flow scheme (Thm. thm_grad) about rho_bar has no velocity: with
the same c_c, c_e the mode evolves as
  r^{k+1} (1 + s lam c_c) = r^k (1 + s lam c_e),
a factor above one exactly when c_c < c_e (the same instability criterion).

A pure shear u = A sin(2 pi q y / L), v = 0 about rho_bar decays as
Crank-Nicolson viscous diffusion: u^{k+1} = A (1 - s gamma lam_y/(2 rho_bar))
/ (1 + s gamma lam_y/(2 rho_bar)) sin(...) + O(A^2).
"""
import numpy as np


def symbols(kx, ky, h):
    lam = 4.0 / (h * h) * (np.sin(0.5 * kx * h) ** 2 + np.sin(0.5 * ky * h) ** 2)
    G = (np.sin(kx * h) ** 2 + np.sin(ky * h) ** 2) / (h * h)
    return lam, G


def coefficients_pfc(rho_bar, alpha, lam):
    return (rho_bar - 1.5) ** 2 + alpha + lam * lam, 2.0 * lam


def coefficients_cdft(rho_bar, ce, Jhat):
    return 1.0 / rho_bar + 2.0 * ce, 2.0 * ce + Jhat


def one_step(r0, z0, rho_bar, s, gamma, lam, G, cc, ce_):
    sg = np.sqrt(G)
    A = np.array([[1.0, 0.5 * s * rho_bar * sg],
                  [-s * rho_bar * sg * cc, rho_bar + 0.5 * s * gamma * lam]])
    B = np.array([[1.0, -0.5 * s * rho_bar * sg],
                  [-s * rho_bar * sg * ce_, rho_bar - 0.5 * s * gamma * lam]])
    return np.linalg.solve(A, B @ np.array([r0, z0]))


def shear_factor(rho_bar, s, gamma, lam_y):
    c = 0.5 * s * gamma * lam_y / rho_bar
    return (1.0 - c) / (1.0 + c)


def gf_factor(s, lam, cc, ce_):
    """Amplification of a Fourier mode by one linearised gradient-flow step."""
    return (1.0 + s * lam * ce_) / (1.0 + s * lam * cc)
