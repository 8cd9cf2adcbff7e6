"""Dense Newton solve of N(g) = S on tiny grids.

The implicit step's result is, by definition, a root of the App. G system
N(g) = S (equivalently of Eqs. discrete_a-d).  The paper does not prove the
root unique; the root meant is the one reached from the old state.  This
module finds it with plain Newton iterations on the whole system, the
Jacobian taken column by column with the complex-step derivative
dN/dg_j = Im N(g + i eps e_j) / eps (exact to round-off, since every row of
N is analytic near the real iterate), and a dense LU solve.  For grids up to
about 8x8 (320 unknowns for PFC, 192 for CDFT).  ``op`` selects the system
(default the App. G one; the gradient-flow variant passes its own rows).
"""
import numpy as np

from .system import N


def jacobian(g, lev, op=N):
    shape = g.shape
    x = g.ravel().astype(np.complex128)
    n = x.size
    Jm = np.empty((n, n))
    eps = 1e-30
    for j in range(n):
        xp = x.copy()
        xp[j] += 1j * eps
        Jm[:, j] = np.imag(op(xp.reshape(shape), lev).ravel()) / eps
    return Jm


def solve(g0, S, lev, tol=1e-14, max_iter=50, op=N):
    """Newton iterations from g0 until the max-norm of N(g) - S is <= tol
    (or stops decreasing); returns (g, iterations, final max-norm)."""
    g = np.array(g0, dtype=np.float64)
    best = np.inf
    for it in range(max_iter):
        F = op(g, lev) - S
        r = float(np.max(np.abs(F)))
        if r <= tol or (it > 3 and r >= best):
            return g, it, r
        best = min(best, r)
        step = np.linalg.solve(jacobian(g, lev, op), -F.ravel())
        g = g + step.reshape(g.shape)
    F = op(g, lev) - S
    return g, max_iter, float(np.max(np.abs(F)))
