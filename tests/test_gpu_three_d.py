"""GPU parity of the PFC step in three dimensions (hfz3_*) against the CPU
FP64 oracle (oracle/three_d.py): stage by stage, step by step, the uniform
fixed point, and at 128^3 the properties the oracle evaluates in one pass."""
import numpy as np
import pytest

import workloads
from oracle import three_d as t3
from tests.helpers import oracle_stepper, rel_err

pytestmark = pytest.mark.gpu


def np_(t):
    return t.cpu().numpy()


def setup(n, seed=0, uamp=0.02, **kw):
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v, w = workloads.pfc3d(n, seed=seed, uamp=uamp, **kw)
    sim = pkg.Simulation3(cfg)
    sim.set_state(rho, u, v, w)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v, w)
    return cfg, sim, ora


@pytest.mark.parametrize("n", [8, 16])
def test_source_and_coefficients(n):
    cfg, sim, ora = setup(n, seed=1)
    assert rel_err(np_(sim.read(5, 0, 0)), ora.g[4]) < 1e-12
    assert rel_err(np_(sim.read(5, 0, 1)), ora.g[5]) < 1e-12
    sim.begin_step()
    S, om = ora.build_source()
    for c in range(6):
        if np.abs(S[c]).max() > 0:
            assert rel_err(np_(sim.read(1, 0, c)), S[c]) < 1e-12, c
    sol = ora.solver(om)
    assert sim.levels() == len(sol.levels)
    for l, lev in enumerate(sol.levels):
        assert rel_err(np_(sim.read(3, l, 0)), lev.rho_k) < 1e-13, l
        for c in range(3):
            assert rel_err(np_(sim.read(3, l, 1 + c)), lev.omega_k[c]) < 1e-12, (l, c)


# levels from 128^3 up are swept by the z-marching tiled kernel, smaller ones
# by two per-colour launches; HFZ3_TILES=32 moves the switch down to 32^3
@pytest.mark.parametrize("n,tiles", [(8, None), (16, None), (32, None), (32, "32"), (64, None), (64, "32"),
                                     (128, None)])
def test_sweeps_and_residual(n, tiles, monkeypatch):
    if tiles:
        monkeypatch.setenv("HFZ3_TILES", tiles)
    cfg, sim, ora = setup(n, seed=2)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    lev = sol.levels[0]
    g = ora.g.copy()
    r0 = sol.resnorm(g, S, lev)
    assert abs(sim.residual() - r0) < 1e-11 * r0
    sim.smooth(0, 1)
    t3.sweep(g, S, lev, cfg.w)
    for c in range(6):
        assert rel_err(np_(sim.read(0, 0, c)), g[c]) < 1e-12, c
    sim.smooth(0, 2)
    t3.sweep(g, S, lev, cfg.w)
    t3.sweep(g, S, lev, cfg.w)
    for c in range(6):
        assert rel_err(np_(sim.read(0, 0, c)), g[c]) < 1e-12, c
    r2 = sol.resnorm(g, S, lev)
    assert abs(sim.residual() - r2) < 1e-10 * r2


def test_tiled_sweep_matches_per_colour_kernels(monkeypatch):
    """The z-marching tiled kernel (forced down to 32^3 by HFZ3_TILES=32) and
    the two per-colour launches (HFZ3_TILES=0) evaluate the same block update
    on the same values: an odd and an even sweep count (the odd one copies
    back from the second buffer)."""
    out = {}
    for tiles in ("32", "0"):
        monkeypatch.setenv("HFZ3_TILES", tiles)
        cfg, sim, _ = setup(64, seed=4)
        sim.begin_step()
        got = []
        for k in (3, 2):
            sim.smooth(0, k)
            got.append([np_(sim.read(0, 0, c)) for c in range(6)])
        out[tiles] = got
    for a, b in zip(out["32"], out["0"]):
        for c in range(6):
            assert rel_err(a[c], b[c]) < 1e-14, c


@pytest.mark.parametrize("n", [16, 32])
def test_tail_matches_per_level_kernels(n, monkeypatch):
    """The levels from 16^3 down run in one workgroup (k3_tail); with it
    switched off (HFZ3_TAIL=0) the per-level kernels run.  Both use the same
    per-node device code: three V-cycles agree to rounding."""
    out = {}
    for tail in ("1", "0"):
        monkeypatch.setenv("HFZ3_TAIL", tail)
        cfg, sim, _ = setup(n, seed=6)
        sim.begin_step()
        sim.vcycle(3)
        out[tail] = [np_(sim.read(0, 0, c)) for c in range(6)]
    for c in range(6):
        assert rel_err(out["1"][c], out["0"][c]) < 1e-14, c


@pytest.mark.parametrize("coarsest,nu1,nu2,sweeps", [(8, 2, 2, 4), (16, 2, 2, 6), (4, 1, 0, 4), (4, 0, 3, 3)])
def test_vcycle_variants(coarsest, nu1, nu2, sweeps):
    """Other cycle shapes at 32^3 against the oracle's V-cycles: coarsest grid
    8^3 (the one-workgroup tail is then only the coarsest sweeps), 16^3 (no
    tail), and V(1,0) and V(0,3) through the tail."""
    cfg, sim, ora = setup(32, seed=8, coarsest_n=coarsest, nu1=nu1, nu2=nu2, coarse_sweeps=sweeps)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    assert sim.levels() == len(sol.levels)
    g = ora.g.copy()
    for k in range(2):
        sim.vcycle(1)
        sol.vcycle(g, S)
        errs = [rel_err(np_(sim.read(0, 0, c)), g[c]) for c in range(6)]
        assert max(errs) < 1e-11, (k, errs)


@pytest.mark.parametrize("n,tiles", [(16, None), (32, None), (32, "32"), (64, "32")])
def test_vcycles(n, tiles, monkeypatch):
    if tiles:
        monkeypatch.setenv("HFZ3_TILES", tiles)
    cfg, sim, ora = setup(n, seed=3)
    sim.begin_step()
    S, om = ora.build_source()
    sol = ora.solver(om)
    g = ora.g.copy()
    for k in range(3):
        sim.vcycle(1)
        sol.vcycle(g, S)
        errs = [rel_err(np_(sim.read(0, 0, c)), g[c]) for c in range(6)]
        assert max(errs) < 1e-11, (k, errs)
    r = sol.resnorm(g, S, sol.levels[0])
    assert abs(sim.residual() - r) < 1e-9 * r


@pytest.mark.parametrize("n,tiles", [(16, None), (32, None), (32, "32")])
def test_steps(n, tiles, monkeypatch):
    if tiles:
        monkeypatch.setenv("HFZ3_TILES", tiles)
    cfg, sim, ora = setup(n, seed=4)
    m0 = sim.mass()
    for k in range(3):
        st = sim.step(1)
        c, r = ora.step()
        assert abs(st.cycles_last - c) <= 1, (k, st.cycles_last, c)
        assert st.residual_last <= cfg.tol
        rg, ug, vg, wg = [np_(x) for x in sim.get_state()]
        assert rel_err(rg, ora.g[0]) < 1e-10, k
        vs = np.abs(ora.g[1:4]).max()
        for x, y in zip((ug, vg, wg), ora.g[1:4]):
            assert np.abs(x - y).max() < 1e-10 * vs, k
    E, Eo = sim.energy(), ora.energy()
    assert abs(E[0] - Eo[0]) < 1e-10 * abs(Eo[0])
    assert abs(sim.mass() - m0) < 1e-13 * abs(m0)


def test_uniform_state_is_a_fixed_point():
    import paper_1503_07416_amd as pkg
    n = 16
    cfg, _, _, _, _ = workloads.pfc3d(n)
    sim = pkg.Simulation3(cfg)
    z = np.zeros((n, n, n))
    rho = np.full((n, n, n), 1.3)
    sim.set_state(rho, z + 0.1, z - 0.2, z + 0.05)
    st = sim.step(2)
    assert st.cycles_total == 0
    r, u, v, w = [np_(x) for x in sim.get_state()]
    assert np.abs(r - rho).max() < 1e-14 and np.abs(u - 0.1).max() < 1e-14


def test_full_size_step():
    """128^3: the GPU's iterate solves the oracle's system to tol, the end of the
    step is the oracle's continuity update, staged == benchmarked step."""
    import paper_1503_07416_amd as pkg
    n = 128
    cfg, rho, u, v, w = workloads.pfc3d(n)
    ora = oracle_stepper(cfg)
    ora.set_state(rho, u, v, w)
    S, om = ora.build_source()
    lev = ora.solver(om).levels[0]
    print("pfc3d 128: begin", flush=True)
    sim = pkg.Simulation3(cfg)
    sim.set_state(rho, u, v, w)
    sim.begin_step()
    for c in range(6):
        if np.abs(S[c]).max() > 0:
            assert rel_err(np_(sim.read(1, 0, c)), S[c]) < 1e-12, c
    r = sim.residual()
    cycles = 0
    while r > cfg.tol and cycles < cfg.max_cycles:
        sim.vcycle(1)
        cycles += 1
        r = sim.residual()
    assert r <= cfg.tol
    g = np.stack([np_(sim.read(0, 0, c)) for c in range(6)])
    dd = S - t3.N(g, lev)
    r_ora = np.sqrt(lev.h ** 3 * float(np.sum(dd * dd)))
    # the two evaluations of S - N(g) differ by rounding in each of the 6 x 2M
    # rows (terms up to ~1/h^2 cancelling to ~1e-11): a few 1e-13 in the norm
    assert r_ora <= cfg.tol and abs(r_ora - r) <= 1e-2 * r + 1e-12, (r_ora, r)
    sim.finish_step()
    staged = [np_(x) for x in sim.get_state()]
    rho1 = S[0] - cfg.s / (4 * cfg.h) * sum(t3.sh(rho * g[1 + a], t3.AX[a], 1) - t3.sh(rho * g[1 + a], t3.AX[a], -1)
                                            for a in range(3))
    assert rel_err(staged[0], rho1) < 1e-12
    sim.close()
    sim = pkg.Simulation3(cfg)
    sim.set_state(rho, u, v, w)
    st = sim.step(1)
    print(f"pfc3d 128: cycles {st.cycles_last} (staged {cycles}), residual {st.residual_last:.3e}", flush=True)
    assert st.cycles_last == cycles
    for x, y in zip([np_(t) for t in sim.get_state()], staged):
        assert np.abs(x - y).max() <= 1e-12 * max(np.abs(y).max(), 1e-30)
    sim.close()


def test_sweep_sampled_at_256():
    """256^3, one sweep of the z-marching tiled kernel in the launch bench.py
    times (2048 workgroups, 256 per XCD): at sampled nodes (random ones and
    ones on tile, z-chunk and periodic boundaries) the GPU's value equals the
    oracle's sweep of a 12^3 patch around the node.  A node's value after one
    red-black sweep depends on the state within two nodes of it (its red
    neighbours' new values read black values one node further, and S, omega^k,
    mu, kappa read one node beyond those), so the patch's periodic wrap, which
    corrupts values within two nodes of its edge, does not reach it; the patch
    origin keeps the colour (i + j + l) mod 2 of the global grid."""
    import paper_1503_07416_amd as pkg
    n, P = 256, 12
    cfg, rho, u, v, w = workloads.pfc3d(n, seed=3, uamp=0.02)
    sim = pkg.Simulation3(cfg)
    sim.set_state(rho, u, v, w)
    sim.begin_step()
    sim.smooth(0, 1)
    rng = np.random.default_rng(17)
    pts = [tuple(int(x) for x in rng.integers(0, n, 3)) for _ in range(48)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (31, 15, 15), (32, 16, 16), (95, 47, 111), (96, 48, 112),
            (63, 0, 255), (224, 255, 0), (1, 17, 33), (30, 14, 14)]
    idx = np.array([(l * n + j) * n + i for i, j, l in pts])
    gpu = np.stack([sim.read(0, 0, c).reshape(-1)[idx].cpu().numpy() for c in range(6)])
    for k, (i, j, l) in enumerate(pts):
        par = (i + j + l) & 1
        o = [i - 6 - par, j - 6, l - 6]          # origin with even coordinate sum: colours agree
        ii = (np.arange(P) + o[0]) % n
        jj = (np.arange(P) + o[1]) % n
        ll = (np.arange(P) + o[2]) % n
        cut = lambda f: f[np.ix_(ll, jj, ii)]
        st = t3.Stepper(P, cfg.h, cfg.s, cfg.alpha, gamma=cfg.gamma, sigma=cfg.sigma)
        st.set_state(cut(rho), cut(u), cut(v), cut(w))
        S, om = st.build_source()
        lev = t3.Level3(cfg.h, cfg.s, cfg.gamma, cfg.sigma, cfg.alpha, st.g[0], om)
        g = st.g.copy()
        t3.sweep(g, S, lev, cfg.w)
        lc = (6 + par, 6, 6)                     # the sample in the patch (x, y, z)
        inner = g[:, 2:-2, 2:-2, 2:-2]
        for c in range(6):
            ref = g[c, lc[2], lc[1], lc[0]]
            scale = max(np.abs(inner[c]).max(), 1e-300)
            assert abs(gpu[c, k] - ref) <= 1e-12 * scale, ((i, j, l), c, gpu[c, k], ref)


@pytest.mark.parametrize("n", [16, 128])
def test_step_that_does_not_converge_leaves_state(n):
    """A step that reaches max_cycles before the tolerance returns
    HFZ_ENOCONV, completes no step and leaves the state as it was (through
    the one-workgroup tail at 16^3, through the tiled sweep and the device
    stop test at 128^3); the next step with enough cycles then converges."""
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v, w = workloads.pfc3d(n, seed=9, uamp=0.02)
    cfg.max_cycles = 2
    sim = pkg.Simulation3(cfg)
    sim.set_state(rho, u, v, w)
    before = [np_(x) for x in sim.get_state()]
    rc, st = sim.step(1, raise_on_error=False)
    assert rc == -4 and st.steps_done == 0
    after = [np_(x) for x in sim.get_state()]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    cfg.max_cycles = 100
    sim2 = pkg.Simulation3(cfg)
    sim2.set_state(rho, u, v, w)
    st2 = sim2.step(1)
    assert st2.steps_done == 1 and st2.cycles_last > 2 and st2.residual_last <= cfg.tol
