"""The CDFT convolution kernel and the discrete periodic convolution.

* J(x) = sqrt(2) exp(-pi^2 |x|^2 / (2 nu^2)) - exp(-pi^2 |x|^2 / (4 nu^2))
  (Sec. 6, model convolution kernel).
* J_e = -J where J <= 0, else 0; J_c = J + J_e (Sec. 6).
* Restriction to the periodic grid, J_{k,l} = J(x_k, y_l) (Sec. 5.2).  The
  displacement of grid offset (k, l) is taken as its minimum image in
  [-L/2, L/2], which makes the tabulated kernel even and Omega-periodic, as
  Sec. 2.1 requires of J.
* (J * rho)_{ij} = h^2 sum_{k,l} J_{k,l} rho_{i-k, j-l}
  (Eq. discrete_convolution).
* (J_e * 1) = h^2 sum_{k,l} (J_e)_{k,l}, the scalar of Lemma CDFT_ineq.
"""
import numpy as np


def J_of_r2(r2, nu):
    """Sec. 6 model kernel as a function of |x|^2."""
    c = np.pi ** 2 / (nu * nu)
    return np.sqrt(2.0) * np.exp(-0.5 * c * r2) - np.exp(-0.25 * c * r2)


def min_image_offsets(n, h):
    """Displacements k h of grid offsets k = 0..n-1, wrapped into [-L/2, L/2]."""
    k = np.arange(n)
    k = np.where(k <= n // 2, k, k - n)
    return k * h


def tabulate(n, h, nu):
    """J_{k,l} on the periodic n x n grid, array indexed [l, k]."""
    x = min_image_offsets(n, h)
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    return J_of_r2(r2, nu)


def split_e(J):
    """J_e of Sec. 6: -J where J <= 0, 0 elsewhere."""
    return np.where(J <= 0.0, -J, 0.0)


def ce(J, h):
    """(J_e * 1) = h^2 sum J_e (the constant convolution of J_e with 1)."""
    return h * h * float(np.sum(split_e(J)))


def conv_direct(J, rho, h):
    """Eq. discrete_convolution by its definition (O(n^4)); for small grids.
    np.roll(rho, (l, k))[j, i] = rho[j - l, i - k]."""
    n = rho.shape[-1]
    out = np.zeros_like(rho, dtype=np.result_type(rho, J))
    for l in range(n):
        for k in range(n):
            out += J[l, k] * np.roll(rho, (l, k), axis=(-2, -1))
    return h * h * out


def symbol(J, h):
    """Multiplier of the discrete convolution on Fourier modes:
    Jhat_h(k) = h^2 sum_{k,l} J_{k,l} exp(-i k.x_{kl}); real because J is even."""
    return h * h * np.real(np.fft.fft2(J))


def conv_fft(J, rho, h):
    """Eq. discrete_convolution through the DFT (the route the paper's
    abstract names for the non-local term)."""
    return np.real(np.fft.ifft2(symbol(J, h) * np.fft.fft2(rho)))
