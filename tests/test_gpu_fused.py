"""GPU: the V-cycle with the FAS restriction folded into the sweep launches
(HFZ_FUSE=1: the last pre-smoothing launch of every level forms R g and R d;
f_c = R d + N_c(R g) is completed on the coarse grid by k_fas_rhs, or by the
tail kernel as it loads) against the same V-cycle with separate restriction
launches (HFZ_FUSE=0) and against the oracle, for every model, cycle shapes,
coarsest grids, sweep schedules and tile shapes; each separate restriction
variant against the oracle; and a coarse level's right-hand side completed by
its own pre-sweep launch (RES = 4) against k_fas_rhs (HFZ_FOLD_RHS=0)."""
import numpy as np
import pytest

import workloads
from tests.helpers import oracle_stepper, rel_err

pytestmark = pytest.mark.gpu


def np_(t):
    return t.cpu().numpy()


def case(model, n, seed=0, **kw):
    if model in ("pfc", "cdft"):
        if model == "pfc":
            cfg, rho, u, v = workloads.pfc_uniform_noise(n, 0.25, 0.01, seed, **kw)
        else:
            cfg, rho, u, v = workloads.cdft_gauss_noise(n, 17.0 / 128.0 * 2, 0.02, seed, **kw)
        u, v = workloads.random_velocity(n, seed + 100, 0.02)
        return cfg, rho, u, v
    return workloads.gradflow(model, n, seed, **kw)


def cycles(cfg, rho, u, v, count, env, monkeypatch):
    import paper_1503_07416_amd as pkg
    for k, val in env.items():
        monkeypatch.setenv(k, val)
    sim = pkg.Simulation(cfg)
    if cfg.gradflow:
        sim.set_state(rho)
    else:
        sim.set_state(rho, u, v)
    sim.begin_step()
    out = []
    for _ in range(count):
        sim.vcycle(1)
        out.append([np_(sim.read(0, 0, c)) for c in range(nc(cfg))])
    for k in env:
        monkeypatch.delenv(k)
    return out


def nc(cfg):
    return {"pfc": 5, "cdft": 3, "pfc_gf": 3, "cdft_gf": 2}[cfg.model]


def oracle_cycles(cfg, rho, u, v, count):
    ora = oracle_stepper(cfg)
    if cfg.gradflow:
        ora.set_state(rho)
    else:
        ora.set_state(rho, u, v)
    if cfg.gradflow:
        S = ora.build_source()
        sol = ora.solver()
    else:
        S, om = ora.build_source()
        sol = ora.solver(om)
    g = ora.initial_guess()
    out = []
    for _ in range(count):
        sol.vcycle(g, S)
        out.append([g[c].copy() for c in range(g.shape[0])])
    return out


CASES = [("pfc", 128, {}), ("pfc", 256, dict(coarsest_n=32)), ("cdft", 128, {}), ("cdft", 64, dict(nu1=1, nu2=1)),
         ("pfc", 128, dict(nu1=3, nu2=1)), ("pfc", 64, dict(nu1=1, nu2=0)), ("pfc_gf", 128, {}),
         ("cdft_gf", 128, dict(coarsest_n=16))]
ENVS = [{}, {"HFZ_SWEEPS": "1"}, {"HFZ_TILE": "2"}, {"HFZ_TILE": "3"}, {"HFZ_TILE": "6"}, {"HFZ_TILE": "9"}]


@pytest.mark.parametrize("model,n,kw", CASES, ids=[f"{m}-{n}-{'-'.join(f'{k}{v}' for k, v in kw.items())}"
                                                   for m, n, kw in CASES])
@pytest.mark.parametrize("env", ENVS, ids=["default", "one-sweep", "tile2", "tile3", "tile6", "tile9"])
def test_fused_equals_separate_and_oracle(model, n, kw, env, monkeypatch):
    cfg, rho, u, v = case(model, n, **kw)
    print(f"fused {model} {n} {kw} {env}", flush=True)
    fused = cycles(cfg, rho, u, v, 3, dict(env, HFZ_FUSE="1"), monkeypatch)
    sep = cycles(cfg, rho, u, v, 3, dict(env, HFZ_FUSE="0"), monkeypatch)
    for k, (a, b) in enumerate(zip(fused, sep)):
        for c, (x, y) in enumerate(zip(a, b)):
            assert rel_err(x, y) < 1e-13, (k, c, rel_err(x, y))
    if env == {}:
        ora = oracle_cycles(cfg, rho, u, v, 3)
        for k, (a, b) in enumerate(zip(fused, ora)):
            errs = [rel_err(x, y) for x, y in zip(a, b)]
            assert max(errs) < 1e-11, (k, errs)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
@pytest.mark.parametrize("variant", ["0", "1", "2", "3"])
def test_separate_restriction_variants_against_oracle(model, variant, monkeypatch):
    """HFZ_FUSE=0 with each FAS restriction variant forced: two V-cycles at
    128^2 against the oracle's."""
    cfg, rho, u, v = case(model, 128, seed=4)
    got = cycles(cfg, rho, u, v, 2, {"HFZ_FUSE": "0", "HFZ_RESTRICT": variant}, monkeypatch)
    ora = oracle_cycles(cfg, rho, u, v, 2)
    for k, (a, b) in enumerate(zip(got, ora)):
        errs = [rel_err(x, y) for x, y in zip(a, b)]
        assert max(errs) < 1e-11, (k, errs)


@pytest.mark.parametrize("model", ["pfc", "cdft"])
def test_fused_steps_equal_separate(model, monkeypatch):
    """Whole steps (graphs, device stop test): the same V-cycle counts and
    states within 1e-12 with and without the fused restriction."""
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v = case(model, 256, seed=5, coarsest_n=32)
    out = []
    for fuse in ("1", "0"):
        monkeypatch.setenv("HFZ_FUSE", fuse)
        sim = pkg.Simulation(cfg)
        sim.set_state(rho, u, v)
        st = sim.step(3)
        out.append((st.cycles_total, [np_(x) for x in sim.get_state()]))
    assert out[0][0] == out[1][0]
    for x, y in zip(out[0][1], out[1][1]):
        assert rel_err(x, y) < 1e-12


@pytest.mark.parametrize("model", ["pfc", "cdft", "pfc_gf", "cdft_gf"])
def test_fused_mixed_precision_steps(model, monkeypatch):
    """Mixed precision: the FP32 correction-form inner V-cycles with the fused
    restriction (the base state restricted along) against the separate
    restriction launches: the same outer iteration counts (within one) and
    final states within 1e-9, each meeting the FP64 tolerance."""
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v = case(model, 128, seed=6, precision="mixed", coarsest_n=16)
    out = []
    for fuse in ("1", "0"):
        monkeypatch.setenv("HFZ_FUSE", fuse)
        sim = pkg.Simulation(cfg)
        if cfg.gradflow:
            sim.set_state(rho)
        else:
            sim.set_state(rho, u, v)
        st = sim.step(3)
        assert st.residual_last <= cfg.tol
        out.append((st.cycles_total, [np_(x) for x in sim.get_state()]))
    assert abs(out[0][0] - out[1][0]) <= 3
    for x, y in zip(out[0][1], out[1][1]):
        if np.abs(y).max() > 0:
            assert rel_err(x, y) < 1e-9


FOLD_CASES = [("pfc", 256, {}), ("cdft", 256, {}), ("pfc_gf", 256, {}), ("cdft_gf", 128, {}),
              ("pfc", 128, dict(coarsest_n=16)), ("cdft", 128, dict(nu1=2, nu2=1))]


@pytest.mark.parametrize("model,n,kw", FOLD_CASES, ids=[f"{m}-{n}-{'-'.join(f'{k}{v}' for k, v in kw.items())}"
                                                        for m, n, kw in FOLD_CASES])
@pytest.mark.parametrize("tile", ["3", "6"])
def test_fold_rhs_equals_fas_rhs_launch(model, n, kw, tile, monkeypatch, capfd):
    """With every restriction folded (HFZ_FUSE=1) the coarse tiled levels
    complete f_c = R d + N_c(R g) in their own pre-sweep launch (RES = 4, the
    completed f read back by their post-sweep launch); HFZ_FOLD_RHS=0 leaves
    it to k_fas_rhs.  The same rows in the same order: three V-cycles agree
    to rounding, and both agree with the oracle's."""
    cfg, rho, u, v = case(model, n, seed=9, **kw)
    print(f"fold-rhs {model} {n} {kw} tile {tile}", flush=True)
    env = {"HFZ_FUSE": "1", "HFZ_TILE": tile, "HFZ_VERBOSE": "1"}
    capfd.readouterr()
    folded = cycles(cfg, rho, u, v, 3, env, monkeypatch)
    err = capfd.readouterr().err
    line = [x for x in err.splitlines() if "completed by the pre-sweep launch" in x]
    assert line and " 1" in line[-1].split(":")[-1], err
    launch = cycles(cfg, rho, u, v, 3, dict(env, HFZ_FOLD_RHS="0"), monkeypatch)
    for k, (a, b) in enumerate(zip(folded, launch)):
        for c, (x, y) in enumerate(zip(a, b)):
            assert rel_err(x, y) < 1e-13, (k, c, rel_err(x, y))
    ora = oracle_cycles(cfg, rho, u, v, 3)
    for k, (a, b) in enumerate(zip(folded, ora)):
        errs = [rel_err(x, y) for x, y in zip(a, b)]
        assert max(errs) < 1e-11, (k, errs)


@pytest.mark.parametrize("model,precision", [("pfc", "fp64"), ("cdft", "fp64"), ("pfc", "mixed"),
                                             ("cdft", "mixed")])
def test_fold_rhs_steps(model, precision, monkeypatch):
    """Whole steps (graphs, device stop test; mixed: the FP32 correction form)
    with the coarse right-hand sides completed in the pre-sweep launches
    against k_fas_rhs: the same V-cycle counts, states within 1e-12 (FP64) or
    1e-9 (mixed)."""
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v = case(model, 256, seed=12, precision=precision, coarsest_n=16)
    out = []
    for fold in ("1", "0"):
        monkeypatch.setenv("HFZ_FUSE", "1")
        monkeypatch.setenv("HFZ_TILE", "4")
        monkeypatch.setenv("HFZ_FOLD_RHS", fold)
        sim = pkg.Simulation(cfg)
        sim.set_state(rho, u, v)
        st = sim.step(3)
        assert st.residual_last <= cfg.tol
        out.append((st.cycles_total, [np_(x) for x in sim.get_state()]))
    tol = 1e-12 if precision == "fp64" else 1e-9
    if precision == "fp64":
        assert out[0][0] == out[1][0]
    else:
        assert abs(out[0][0] - out[1][0]) <= 3
    for x, y in zip(out[0][1], out[1][1]):
        if np.abs(y).max() > 0:
            assert rel_err(x, y) < tol
