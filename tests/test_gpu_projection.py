"""GPU parity in the regime of the CDFT positivity projection (Sec. 6, first
modification: rho <- sqrt(rho^2 + delta^2) after every rho update), through
the C ABI against the CPU FP64 oracle.

The near-vacuum projection workload (``workloads.cdft_vacuum_lattice``:
density peaks on troughs of 1e-3, flow out of the troughs) makes the first
V-cycle's continuity updates negative at some finest-level nodes; a right-hand
side forced negative at chosen nodes makes every kernel that updates rho (the
tiled smoother at 64^2 and 128^2, the one-workgroup tail at 32^2) project.
The oracle counts the projected updates, so each test shows the branch ran.
"""
import numpy as np
import pytest

import workloads
from tests.helpers import oracle_stepper, rel_err, state_errors
from tests.projection_helpers import count_negative_sweep, counting_sweeps

pytestmark = pytest.mark.gpu


def np_(t):
    return t.cpu().numpy()


def sim_for(cfg, rho, u, v):
    import paper_1503_07416_amd as pkg
    s = pkg.Simulation(cfg)
    s.set_state(rho, u, v)
    return s


def forced_rhs(S, frac=0.1, seed=0):
    """S with the rho row's right-hand side made negative at a random tenth of
    the nodes (the continuity update there starts below zero)."""
    rng = np.random.default_rng(seed)
    f0 = S[0].copy()
    m = rng.uniform(size=f0.shape) < frac
    f0[m] = -np.abs(f0[m]) - 0.05
    return f0


@pytest.mark.parametrize("n", [64, 128])
def test_sweeps_with_forced_negative_updates(n):
    """One and two sweeps of the tiled smoother on level 0 with a forced
    negative right-hand side, node for node against the oracle (1e-12)."""
    cfg, rho, u, v = workloads.cdft_vacuum_lattice(n)
    print(f"projection sweeps {n}^2", flush=True)
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    sim.begin_step()
    S, om = ora.build_source()
    lev = ora.solver(om).levels[0]
    S[0] = forced_rhs(S)
    sim.write(1, 0, 0, S[0])
    g = ora.initial_guess()
    from oracle import smoother
    for sweeps in (1, 2):
        neg = 0
        for _ in range(sweeps):
            neg += count_negative_sweep(g, S, lev)
            smoother.sweep(g, S, lev, cfg.w)
        sim.smooth(0, sweeps)
        assert neg > 0.05 * n * n, neg
        for c in range(3):
            assert rel_err(np_(sim.read(0, 0, c)), g[c]) < 1e-12, (sweeps, c)
        assert np_(sim.read(0, 0, 0)).min() > 0


def test_tail_vcycle_with_forced_negative_updates():
    """A 32^2 grid runs its whole V-cycle in the one-workgroup tail kernel; with
    a forced negative right-hand side two V-cycles agree with the oracle's."""
    cfg, rho, u, v = workloads.cdft_vacuum_lattice(32)
    print("projection tail 32^2", flush=True)
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    S[0] = forced_rhs(S, seed=1)
    sim.write(1, 0, 0, S[0])
    g = ora.initial_guess()
    counts = {}
    for k in range(2):
        with counting_sweeps(counts):
            sol.vcycle(g, S)
        sim.vcycle(1)
        errs = [rel_err(np_(sim.read(0, 0, c)), g[c]) for c in range(3)]
        assert max(errs) < 1e-11, (k, errs)
    assert counts[32] > 50, counts


@pytest.mark.parametrize("n", [64, 128])
def test_vcycles_in_the_projection_regime(n):
    """Three V-cycles of the first step of the near-vacuum workload (the first
    projects finest-level updates), against the oracle's."""
    cfg, rho, u, v = workloads.cdft_vacuum_lattice(n)
    print(f"projection vcycles {n}^2", flush=True)
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    g = ora.initial_guess()
    counts = {}
    for k in range(3):
        with counting_sweeps(counts):
            sol.vcycle(g, S)
        sim.vcycle(1)
        errs = [rel_err(np_(sim.read(0, 0, c)), g[c]) for c in range(3)]
        assert max(errs) < 1e-11, (k, errs)
    assert counts[n] > 20, counts


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_steps_in_the_projection_regime(precision, tol):
    """Three whole steps of the near-vacuum workload at 64^2 (FP64 and mixed
    precision) against the oracle: fields, V-cycle counts (FP64), energy and
    mass."""
    cfg, rho, u, v = workloads.cdft_vacuum_lattice(64, precision=precision)
    print(f"projection steps {precision}", flush=True)
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    counts = {}
    for k in range(3):
        st = sim.step(1)
        with counting_sweeps(counts):
            c, r = ora.step()
        if precision == "fp64":
            assert abs(st.cycles_last - c) <= 1, (k, st.cycles_last, c)
        assert st.residual_last <= cfg.tol
        errs = state_errors([np_(x) for x in sim.get_state()], (ora.rho, ora.u, ora.v))
        assert max(errs) < tol, (k, errs)
        E, Eo = sim.energy(), ora.energy()
        assert abs(E[0] - Eo[0]) < tol * max(1.0, abs(Eo[0]))
    assert counts[64] > 20, counts
    assert abs(sim.mass() - ora.mass()) < 1e-12 * ora.mass()
