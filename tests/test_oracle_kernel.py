"""Pins of the CDFT kernel and convolution (Sec. 2.1 assumptions, Eq.
discrete_convolution, Sec. 6 kernel and Fourier image)."""
import numpy as np

from oracle import kernel


def test_fft_convolution_equals_direct_sum():
    rng = np.random.default_rng(0)
    for n, h, nu in [(16, 0.6, 1.0), (12, 17 / 128 * 8, 2.362)]:
        J = kernel.tabulate(n, h, nu)
        rho = 1.0 + 0.1 * rng.standard_normal((n, n))
        a = kernel.conv_direct(J, rho, h)
        b = kernel.conv_fft(J, rho, h)
        assert np.allclose(a, b, atol=1e-12 * np.abs(a).max())


def test_direct_sum_by_hand():
    """One entry of the definition, written out with explicit indices."""
    rng = np.random.default_rng(1)
    n, h = 6, 0.9
    J = kernel.tabulate(n, h, 1.7)
    rho = rng.standard_normal((n, n))
    i, j = 1, 4
    ref = h * h * sum(J[l, k] * rho[(j - l) % n, (i - k) % n] for k in range(n) for l in range(n))
    assert np.isclose(kernel.conv_direct(J, rho, h)[j, i], ref)


def test_kernel_assumptions():
    """J even and periodic; J = J_c - J_e with J_c, J_e >= 0; sum J < 0 (Sec. 2.1)."""
    n, h, nu = 128, 17 / 128, 2.362
    J = kernel.tabulate(n, h, nu)
    assert np.array_equal(J, np.roll(J[::-1, ::-1], (1, 1), axis=(0, 1)))
    Je = kernel.split_e(J)
    Jc = J + Je
    assert (Je >= 0).all() and (Jc >= 0).all()
    assert h * h * J.sum() < 0
    # continuum integral nu^2 (2 sqrt 2 - 4) / pi of the Sec. 6 kernel
    assert np.isclose(h * h * J.sum(), nu ** 2 * (2 * np.sqrt(2) - 4) / np.pi, rtol=1e-6)
    assert kernel.ce(J, h) > 0


def test_symbol_real_and_continuum_limit():
    """Jhat_h is real (J even) and tends to the continuous Fourier transform
    (2 nu^2/pi)[sqrt2 exp(-k^2 nu^2/(2 pi^2)) - 2 exp(-k^2 nu^2/pi^2)]."""
    n, h, nu = 128, 17 / 128, 2.362
    J = kernel.tabulate(n, h, nu)
    full = h * h * np.fft.fft2(J)
    assert np.abs(full.imag).max() < 1e-12 * np.abs(full.real).max()
    k = 2 * np.pi * np.fft.fftfreq(n, d=h)
    K2 = k[None, :] ** 2 + k[:, None] ** 2
    cont = (2 * nu ** 2 / np.pi) * (np.sqrt(2) * np.exp(-K2 * nu ** 2 / (2 * np.pi ** 2))
                                    - 2 * np.exp(-K2 * nu ** 2 / np.pi ** 2))
    Jh = kernel.symbol(J, h)
    assert np.abs(Jh - cont).max() < 2e-3
    # the uniform state at the packing-fraction-0.6 density is unstable
    rho_bar = 6 * 0.6 / np.pi
    assert (1 - rho_bar * Jh).min() < 0
    # and the literal pi/6 * 0.6 would be stable
    assert (1 - np.pi / 6 * 0.6 * Jh).min() > 0
