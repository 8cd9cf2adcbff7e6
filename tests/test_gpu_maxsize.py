"""GPU at the largest grids the ABI accepts, in the launch configuration the
tuner picks there: PFC 8192^2 (two damped sweeps), the PFC gradient flow at
8192^2 (two sweeps), the channel at 8192 x 8193 (two sweeps; the patch takes
the true wall as its own where the node is near one, elsewhere both patch
walls are far from it) and the 3D step at 512^3
(one sweep of the z-marching tiled kernel).  At sampled nodes (random ones and
ones on tile and periodic boundaries) the GPU's value equals the oracle's
sweeps of a small patch around the node: after k red-black sweeps a node's
value depends on the state within 2k nodes of it, and S, omega^k and the
initial mu, kappa reach a few nodes further, so a patch wide enough is exact
at its centre (its periodic wrap corrupts only values near its edge), with its
origin chosen to keep the global colouring.  (CDFT's source holds a global
convolution, so a patch cannot stand in for it; its largest full-size test is
1024^2.)"""
import numpy as np
import pytest

import workloads
from oracle import fas, smoother
from oracle import gradflow as gf
from oracle import three_d as t3
from oracle import walls

pytestmark = pytest.mark.gpu


def test_pfc_8192_two_sweeps_sampled():
    import paper_1503_07416_amd as pkg
    n, P, R = 8192, 24, 8
    cfg, rho, _, _ = workloads.pfc_uniform_noise(n, 0.25, 0.01, 7)
    u, v = workloads.random_velocity(n, 8, 0.02)
    print("pfc 8192: init", flush=True)
    sim = pkg.Simulation(cfg)
    sim.set_state(rho, u, v)
    tx, ty, _ = sim.tile_shape(0)
    sim.begin_step()
    sim.smooth(0, 2)
    rng = np.random.default_rng(21)
    pts = [tuple(int(x) for x in rng.integers(0, n, 2)) for _ in range(40)]
    pts += [(0, 0), (n - 1, n - 1), (tx - 1, ty - 1), (tx, ty), (3 * tx - 1, 5 * ty), (n - 1, 0), (1, n - 2)]
    idx = np.array([j * n + i for i, j in pts])
    gpu = np.stack([sim.read(0, 0, c).reshape(-1)[idx].cpu().numpy() for c in range(5)])
    for k, (i, j) in enumerate(pts):
        par = (i + j) & 1
        ii = (np.arange(P) + i - R - par) % n
        jj = (np.arange(P) + j - R) % n
        cut = lambda f: f[np.ix_(jj, ii)]
        st = fas.Stepper(cfg.model, P, cfg.h, cfg.s, **cfg.oracle_kwargs())
        st.set_state(cut(rho), cut(u), cut(v))
        S, om = st.build_source()
        lev = st.solver(om).levels[0]
        g = st.initial_guess()
        smoother.sweep(g, S, lev, cfg.w)
        smoother.sweep(g, S, lev, cfg.w)
        inner = g[:, 6:-6, 6:-6]
        for c in range(5):
            ref = g[c, R, R + par]
            scale = max(np.abs(inner[c]).max(), 1e-300)
            assert abs(gpu[c, k] - ref) <= 1e-12 * scale, ((i, j), c, gpu[c, k], ref)


def test_pfc3d_512_sweep_sampled():
    import paper_1503_07416_amd as pkg
    n, P = 512, 12
    cfg, rho, u, v, w = workloads.pfc3d(n, seed=4, uamp=0.02)
    print("pfc3d 512: init", flush=True)
    sim = pkg.Simulation3(cfg)
    sim.set_state(rho, u, v, w)
    sim.begin_step()
    sim.smooth(0, 1)
    rng = np.random.default_rng(23)
    pts = [tuple(int(x) for x in rng.integers(0, n, 3)) for _ in range(32)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (31, 15, 15), (32, 16, 16), (n - 1, 0, n - 1), (255, 256, 257)]
    idx = np.array([(l * n + j) * n + i for i, j, l in pts])
    gpu = np.stack([sim.read(0, 0, c).reshape(-1)[idx].cpu().numpy() for c in range(6)])
    for k, (i, j, l) in enumerate(pts):
        par = (i + j + l) & 1
        ii = (np.arange(P) + i - 6 - par) % n
        jj = (np.arange(P) + j - 6) % n
        ll = (np.arange(P) + l - 6) % n
        cut = lambda f: f[np.ix_(ll, jj, ii)]
        st = t3.Stepper(P, cfg.h, cfg.s, cfg.alpha, gamma=cfg.gamma, sigma=cfg.sigma)
        st.set_state(cut(rho), cut(u), cut(v), cut(w))
        S, om = st.build_source()
        lev = t3.Level3(cfg.h, cfg.s, cfg.gamma, cfg.sigma, cfg.alpha, st.g[0], om)
        g = st.g.copy()
        t3.sweep(g, S, lev, cfg.w)
        inner = g[:, 2:-2, 2:-2, 2:-2]
        for c in range(6):
            ref = g[c, 6, 6, 6 + par]
            scale = max(np.abs(inner[c]).max(), 1e-300)
            assert abs(gpu[c, k] - ref) <= 1e-12 * scale, ((i, j, l), c, gpu[c, k], ref)


def test_pfc_gradflow_8192_two_sweeps_sampled():
    import paper_1503_07416_amd as pkg
    n, P, R = 8192, 24, 8
    cfg, rho, _, _ = workloads.gradflow("pfc_gf", n, 9)
    print("pfc_gf 8192: init", flush=True)
    sim = pkg.Simulation(cfg)
    sim.set_state(rho)
    tx, ty, _ = sim.tile_shape(0)
    sim.begin_step()
    sim.smooth(0, 2)
    rng = np.random.default_rng(25)
    pts = [tuple(int(x) for x in rng.integers(0, n, 2)) for _ in range(40)]
    pts += [(0, 0), (n - 1, n - 1), (tx - 1, ty - 1), (tx, ty), (n - 1, 0)]
    idx = np.array([j * n + i for i, j in pts])
    nc = 3
    gpu = np.stack([sim.read(0, 0, c).reshape(-1)[idx].cpu().numpy() for c in range(nc)])
    for k, (i, j) in enumerate(pts):
        par = (i + j) & 1
        ii = (np.arange(P) + i - R - par) % n
        jj = (np.arange(P) + j - R) % n
        st = gf.Stepper(cfg.base_model, P, cfg.h, cfg.s, **cfg.oracle_kwargs())
        st.set_state(rho[np.ix_(jj, ii)])
        S = st.build_source()
        lev = st.solver().levels[0]
        g = st.initial_guess()
        gf.sweep(g, S, lev, cfg.w)
        gf.sweep(g, S, lev, cfg.w)
        inner = g[:, 6:-6, 6:-6]
        for c in range(nc):
            ref = g[c, R, R + par]
            scale = max(np.abs(inner[c]).max(), 1e-300)
            assert abs(gpu[c, k] - ref) <= 1e-12 * scale, ((i, j), c, gpu[c, k], ref)


def test_channel_8192_two_sweeps_sampled():
    import paper_1503_07416_amd as pkg
    n, P, H = 8192, 24, 12
    cfg, rho, u, v = workloads.channel(n, u_wall=0.1, seed=6, amp=0.05)
    rng = np.random.default_rng(27)
    u = u + 0.02 * rng.standard_normal(u.shape)
    v = v + 0.02 * rng.standard_normal(v.shape)
    print("channel 8192: init", flush=True)
    sim = pkg.Simulation(cfg)
    sim.set_state(rho, u, v)
    sim.begin_step()
    sim.smooth(0, 2)
    pts = [(int(rng.integers(0, n)), int(rng.integers(0, n + 1))) for _ in range(32)]
    pts += [(0, 0), (5, 1), (n - 1, 3), (17, n - 2), (n - 7, n), (4096, 4096), (31, 15), (32, 16)]
    idx = np.array([j * n + i for i, j in pts])
    gpu = np.stack([sim.read(0, 0, c).reshape(-1)[idx].cpu().numpy() for c in range(5)])
    kw = cfg.wall_oracle_kwargs()
    for k, (i, j) in enumerate(pts):
        j0 = min(max(j - H, 0), n - P)
        ox = i - H
        ox -= (ox + j0) & 1                       # keeps the colour (i + j) mod 2
        ii = (np.arange(P) + ox) % n
        jj = np.arange(P + 1) + j0
        cut = lambda f: f[np.ix_(jj, ii)]
        st = walls.Stepper(P, cfg.h, cfg.s, cfg.alpha, **kw)
        st.set_state(cut(rho), cut(u), cut(v))
        S, om = st.build_source()
        lev = st.solver(om).levels[0]
        g = st.g.copy()
        walls.sweep(g, S, lev, cfg.w)
        walls.sweep(g, S, lev, cfg.w)
        for c in range(5):
            ref = g[c, j - j0, i - ox]
            scale = max(np.abs(g[c]).max(), 1e-300)
            assert abs(gpu[c, k] - ref) <= 1e-12 * scale, ((i, j), c, gpu[c, k], ref)
