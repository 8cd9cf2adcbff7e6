"""GPU parity of other cycle shapes than V(2,2) with a 4^2 coarsest grid, and
the non-finite failure path, through the C ABI against the CPU FP64 oracle.

* FP64: V(1,0), V(0,3), V(1,1), V(3,1) at 64^2 and 128^2 (PFC and CDFT):
  three V-cycles stage by stage (the tiled levels, the per-level residual
  and prolongation kernels that nu1 = 0 / nu2 = 0 need, the tail) and two
  steps; a coarsest grid of 64^2 at 128^2 (the per-colour smoother on the
  coarsest level) and of 8^2, 16^2, 32^2 (the tail's bottom).
* Mixed precision (FP32 correction form inside FP64 defect correction), which
  takes nu1 >= 1, nu2 >= 1 and coarsest_n <= 32: V(1,1), V(1,3), V(3,1) and
  coarsest 8^2 to 32^2, two steps within 1e-6 of the FP64 oracle.
* HFZ_ENAN: a non-finite value in the initial state makes the first residual
  non-finite; the step fails with HFZ_ENAN and leaves the state as it was
  (device stop test and host-tested loop, FP64 and mixed).
"""
import numpy as np
import pytest

import workloads
from tests.helpers import oracle_stepper, rel_err, state_errors

pytestmark = pytest.mark.gpu


def np_(t):
    return t.cpu().numpy()


def case(model, n, seed=0, **kw):
    if model == "pfc":
        cfg, rho, u, v = workloads.pfc_uniform_noise(n, 0.25, 0.01, seed, **kw)
        u, v = workloads.random_velocity(n, seed + 100, 0.02)
    else:
        cfg, rho, u, v = workloads.cdft_gauss_noise(n, 17.0 / 128.0 * 2, 0.02, seed, **kw)
        u, v = workloads.random_velocity(n, seed + 100, 0.02)
    return cfg, rho, u, v


def sim_for(cfg, rho, u, v):
    import paper_1503_07416_amd as pkg
    s = pkg.Simulation(cfg)
    s.set_state(rho, u, v)
    return s


SHAPES = [(1, 0), (0, 3), (1, 1), (3, 1)]


@pytest.mark.parametrize("model", ["pfc", "cdft"])
@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("nu1,nu2", SHAPES, ids=[f"V{a}{b}" for a, b in SHAPES])
def test_fp64_cycle_shapes(model, n, nu1, nu2):
    cfg, rho, u, v = case(model, n, nu1=nu1, nu2=nu2)
    print(f"fp64 {model} {n}^2 V({nu1},{nu2})", flush=True)
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    g = ora.initial_guess()
    for k in range(3):
        sim.vcycle(1)
        sol.vcycle(g, S)
        errs = [rel_err(np_(sim.read(0, 0, c)), g[c]) for c in range(g.shape[0])]
        assert max(errs) < 1e-11, (k, errs)
    # two whole steps (a fresh handle: the staged cycles above left its iterate mid-solve)
    cfg.max_cycles = 400
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    for k in range(2):
        st = sim.step(1)
        c, r = ora.step()
        assert abs(st.cycles_last - c) <= 1, (k, st.cycles_last, c)
        errs = state_errors([np_(x) for x in sim.get_state()], (ora.rho, ora.u, ora.v))
        assert max(errs) < 1e-10, (k, errs)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
@pytest.mark.parametrize("n,cn", [(128, 64), (128, 32), (64, 16), (64, 8)])
def test_fp64_coarsest_grids(model, n, cn):
    cfg, rho, u, v = case(model, n, seed=1, coarsest_n=cn)
    print(f"fp64 {model} {n}^2 coarsest {cn}^2", flush=True)
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    assert sim.levels() == len(ora.solver(ora.build_source()[1]).levels)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    g = ora.initial_guess()
    for k in range(2):
        sim.vcycle(1)
        sol.vcycle(g, S)
        errs = [rel_err(np_(sim.read(0, 0, c)), g[c]) for c in range(g.shape[0])]
        assert max(errs) < 1e-11, (k, errs)


MIXED = [(1, 1, 4), (1, 3, 4), (3, 1, 4), (2, 2, 8), (2, 2, 16), (2, 2, 32)]


@pytest.mark.parametrize("model", ["pfc", "cdft"])
@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("nu1,nu2,cn", MIXED, ids=[f"V{a}{b}-c{c}" for a, b, c in MIXED])
def test_mixed_cycle_shapes(model, n, nu1, nu2, cn):
    cfg, rho, u, v = case(model, n, seed=2, nu1=nu1, nu2=nu2, coarsest_n=cn, precision="mixed")
    print(f"mixed {model} {n}^2 V({nu1},{nu2}) coarsest {cn}^2", flush=True)
    cfg.max_cycles = 400
    sim = sim_for(cfg, rho, u, v)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    for k in range(2):
        st = sim.step(1)
        ora.step()
        assert st.residual_last <= cfg.tol
        errs = state_errors([np_(x) for x in sim.get_state()], (ora.rho, ora.u, ora.v))
        assert max(errs) < 1e-6, (k, errs)


@pytest.mark.parametrize("model,precision,graph", [("pfc", "fp64", "1"), ("pfc", "fp64", "0"),
                                                   ("pfc", "mixed", "1"), ("cdft", "fp64", "1"),
                                                   ("cdft", "mixed", "0")])
def test_nonfinite_state_is_enan_and_rolled_back(model, precision, graph, monkeypatch):
    monkeypatch.setenv("HFZ_GRAPH", graph)
    cfg, rho, u, v = case(model, 64, seed=3, precision=precision)
    print(f"ENAN {model} {precision} graph={graph}", flush=True)
    if model == "pfc":
        rho[5, 7] = np.nan
    else:
        u[5, 7] = np.inf  # CDFT set_state refuses rho <= 0; a velocity carries the non-finite value
    sim = sim_for(cfg, rho, u, v)
    before = [np_(x) for x in sim.get_state()]
    rc, st = sim.step(2, raise_on_error=False)
    assert rc == -5 and st.steps_done == 0, (rc, st.steps_done)
    after = [np_(x) for x in sim.get_state()]
    for a, b in zip(before, after):
        assert np.array_equal(a, b, equal_nan=True)
