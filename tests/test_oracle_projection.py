"""Pins of the CDFT positivity projection in the oracle (Sec. 6, first
modification of the scheme): after every update of rho in the smoother,
rho <- sqrt(rho^2 + delta^2), before rho enters the potential ln rho.

* By hand: on an 8 x 8 level with rho^k = 1, omega^k = 0 and the iterate at
  rho = 0.7, u = v = 0, a red node whose rho row has right-hand side -0.3 gets
  rho^ = -0.3 in the red half sweep (its black neighbours still carry u = v = 0),
  projected to sqrt(0.09 + delta^2): 0.5 for delta = 0.4 and 0.3 for
  delta = 1e-10, then damped with w = 0.5 against 0.7.  Without the
  projection it would be 0.2.
* In the near-vacuum regime of the projection workload (peaks of density 2 on
  troughs of 1e-3, flow out of the troughs, s = 0.03) the first V-cycle of the
  first step projects some finest-level updates, and the step still converges
  to a positive density.
"""
import numpy as np
import pytest

import workloads
from oracle import smoother, system
from tests.helpers import oracle_stepper
from tests.projection_helpers import count_negative_sweep, counting_sweeps


@pytest.mark.parametrize("delta,want", [(0.4, 0.5 * 0.5 + 0.35), (1e-10, 0.5 * 0.3 + 0.35)])
def test_projection_by_hand(delta, want):
    n, h, s = 8, 0.5, 0.01
    lev = system.Level("cdft", h, s, 2.0, 1.0, np.ones((n, n)), np.zeros((n, n)), ce=0.3, delta=delta)
    g = np.zeros((3, n, n))
    g[0] = 0.7
    f = np.zeros((3, n, n))
    f[0] = 0.4
    f[0, 2, 4] = -0.3     # node (i, j) = (4, 2): red, (i + j) even
    smoother.sweep(g, f, lev, 0.5)
    assert abs(g[0, 2, 4] - want) < 1e-15
    # the other red nodes: rho^ = 0.4 (no projection effect beyond rounding)
    red = (smoother.colour_mask(n) == 0)
    red[2, 4] = False
    assert np.abs(g[0][red] - (0.5 * np.sqrt(0.16 + delta * delta) + 0.35)).max() < 1e-15


def test_near_vacuum_workload_projects_and_converges():
    cfg, rho, u, v = workloads.cdft_vacuum_lattice(64, coarse_sweeps=4)
    assert rho.min() > 0 and rho.min() < 1.1e-3
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    S, om = ora.build_source()
    sol = ora.solver(om)
    g = ora.initial_guess()
    counts = {}
    with counting_sweeps(counts):
        sol.vcycle(g, S)
    assert counts[64] > 20, counts
    assert np.all(g[0] > 0)
    for _ in range(2):
        cycles, r = ora.step()
        assert r <= cfg.tol and cycles < 40
        assert ora.rho.min() > 0
