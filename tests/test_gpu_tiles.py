"""GPU: every tile shape of the tiled sweep kernel, and every variant of the
FAS restriction kernel, gives the same iterates.

The red-black sweeps update each node from the same neighbour values whatever
tile owns it (the halo is recomputed, not exchanged), so the shape changes
only the grouping of work.  For each shape forced through HFZ_TILE, three
V-cycles (FP64) or two mixed-precision steps must match shape 0 to 1e-13
relative; the kernels are separate instantiations, so floating-point
contraction may differ in the last bit.  The same holds for the restriction
variants forced through HFZ_RESTRICT.  The tuned shapes are reported."""
import numpy as np
import pytest

import workloads
from oracle import fas
from tests.helpers import oracle_stepper, rel_err

pytestmark = pytest.mark.gpu

SHAPES = list(range(10))


def case(model, n, precision):
    if model == "pfc":
        cfg, rho, u, v = workloads.pfc_uniform_noise(n, 0.25, 0.01, 4, precision=precision)
        u, v = workloads.random_velocity(n, 104, 0.02)
    else:
        cfg, rho, u, v = workloads.cdft_gauss_noise(n, 17.0 / 64.0, 0.02, 4, precision=precision)
    return cfg, rho, u, v


def run_vcycles(monkeypatch, shape, model, n, env="HFZ_TILE"):
    import paper_1503_07416_amd as pkg
    monkeypatch.setenv(env, str(shape))
    cfg, rho, u, v = case(model, n, "fp64")
    sim = pkg.Simulation(cfg)
    sim.set_state(rho, u, v)
    sim.begin_step()
    sim.vcycle(3)
    out = [sim.read(0, 0, c).cpu().numpy() for c in range(5 if model == "pfc" else 3)]
    shape0 = sim.tile_shape(0)
    sim.close()
    return out, shape0


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_vcycles_same_for_every_shape(monkeypatch, model):
    n = 256
    ref, s0 = run_vcycles(monkeypatch, 0, model, n)
    assert s0 == (32, 16, 256)
    for shape in SHAPES[1:]:
        got, sh = run_vcycles(monkeypatch, shape, model, n)
        assert sh is not None
        for c, (x, y) in enumerate(zip(got, ref)):
            assert rel_err(x, y) <= 1e-13, (shape, c, rel_err(x, y))


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_mixed_steps_same_for_every_shape(monkeypatch, model):
    import paper_1503_07416_amd as pkg
    res = {}
    for shape in SHAPES:
        monkeypatch.setenv("HFZ_TILE", str(shape))
        cfg, rho, u, v = case(model, 128, "mixed")
        sim = pkg.Simulation(cfg)
        sim.set_state(rho, u, v)
        st = sim.step(2)
        res[shape] = ([x.cpu().numpy() for x in sim.get_state()], st.cycles_total)
        sim.close()
    for shape in SHAPES[1:]:
        assert res[shape][1] == res[0][1]
        for x, y in zip(res[shape][0], res[0][0]):
            assert rel_err(x, y) <= 1e-13


def test_tuned_shapes_match_oracle(monkeypatch):
    """The tuned configuration (whatever shapes it picked) against the oracle."""
    import paper_1503_07416_amd as pkg
    monkeypatch.delenv("HFZ_TILE", raising=False)
    cfg, rho, u, v = case("pfc", 256, "fp64")
    sim = pkg.Simulation(cfg)
    sim.set_state(rho, u, v)
    shapes = [sim.tile_shape(l) for l in range(sim.levels())]
    print("tuned tile shapes per level:", shapes)
    assert shapes[0] is not None and shapes[-1] is None
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    g = ora.initial_guess()
    for k in range(2):
        sim.vcycle(1)
        sol.vcycle(g, S)
    errs = [rel_err(sim.read(0, 0, c).cpu().numpy(), g[c]) for c in range(5)]
    assert max(errs) < 1e-11, errs
    r = fas.resnorm(g, S, sol.levels[0])
    assert abs(sim.residual() - r) < 1e-9 * r


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_vcycles_same_for_every_restriction(monkeypatch, model):
    monkeypatch.setenv("HFZ_TILE", "0")
    ref, _ = run_vcycles(monkeypatch, 0, model, 256, env="HFZ_RESTRICT")
    for rs in (1, 2, 3):
        got, _ = run_vcycles(monkeypatch, rs, model, 256, env="HFZ_RESTRICT")
        for c, (x, y) in enumerate(zip(got, ref)):
            assert rel_err(x, y) <= 1e-13, (rs, c, rel_err(x, y))


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_mixed_steps_same_for_every_restriction(monkeypatch, model):
    import paper_1503_07416_amd as pkg
    monkeypatch.setenv("HFZ_TILE", "0")
    res = {}
    for rs in (0, 1, 2, 3):
        monkeypatch.setenv("HFZ_RESTRICT", str(rs))
        cfg, rho, u, v = case(model, 128, "mixed")
        sim = pkg.Simulation(cfg)
        sim.set_state(rho, u, v)
        st = sim.step(2)
        res[rs] = ([x.cpu().numpy() for x in sim.get_state()], st.cycles_total)
        sim.close()
    for rs in (1, 2, 3):
        assert res[rs][1] == res[0][1]
        for x, y in zip(res[rs][0], res[0][0]):
            assert rel_err(x, y) <= 1e-13


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_vcycles_same_for_either_sweep_schedule(monkeypatch, model):
    """One sweep per launch (HFZ_SWEEPS=1) against two fused sweeps."""
    monkeypatch.setenv("HFZ_TILE", "0")
    monkeypatch.setenv("HFZ_RESTRICT", "0")
    ref, _ = run_vcycles(monkeypatch, 2, model, 256, env="HFZ_SWEEPS")
    got, _ = run_vcycles(monkeypatch, 1, model, 256, env="HFZ_SWEEPS")
    for c, (x, y) in enumerate(zip(got, ref)):
        assert rel_err(x, y) <= 1e-13, (c, rel_err(x, y))
