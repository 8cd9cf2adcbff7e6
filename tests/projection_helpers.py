"""Test helpers for the CDFT positivity projection (Sec. 6): counting how
often the smoother's continuity update goes negative.  Counting only: the
values compared are the oracle's own."""
import contextlib

import numpy as np

from oracle import smoother
from oracle.fas import Solver
from oracle.grid import east, north, south, west


def rho_hat_unprojected(g, f, lev):
    """The rho row's block update before the projection (the quantity the
    projection acts on)."""
    ru, rv = lev.rho_k * g[1], lev.rho_k * g[2]
    return f[0] - lev.s / (4 * lev.h) * (east(ru) - west(ru) + north(rv) - south(rv))


def count_negative_sweep(g, f, lev, w=0.5):
    """Number of nodes whose rho update goes negative in one damped red-black
    sweep of (a copy of) g, without changing g."""
    g = g.copy()
    par = smoother.colour_mask(g.shape[-1])
    neg = 0
    for colour in (0, 1):
        m = par == colour
        neg += int((rho_hat_unprojected(g, f, lev)[m] <= 0).sum())
        gs = smoother.block_solve(g, f, lev)
        g[:, m] = (1.0 - w) * gs[:, m] + w * g[:, m]
    return neg


@contextlib.contextmanager
def counting_sweeps(counts):
    """Within the block, every Solver sweep also adds its number of negative
    rho updates to counts[n] (n the level's grid size)."""
    orig = Solver.sweep

    def sweep(g, f, lev, w):
        n = g.shape[-1]
        counts[n] = counts.get(n, 0) + count_negative_sweep(g, f, lev, w)
        return orig(g, f, lev, w)

    Solver.sweep = staticmethod(sweep)
    try:
        yield counts
    finally:
        Solver.sweep = staticmethod(orig)
