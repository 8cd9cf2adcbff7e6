"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle
checks.  This module only draws random numbers and fixes the constants of each
workload; it holds none of the scheme's arithmetic.

Constants follow the paper's own runs (Sec. 6); where the printed value is
ambiguous, the reading taken and its reason are stated with it:

* PFC freezing run: eps = 0.025 (alpha = 1 - eps), gamma = 2, domain
  [0,32)^2 on 128^2 (h = 0.25), s = 0.01; mean density 3/2 - 0.07 sqrt(3)
  (the printed "+1/2" read as "+3/2", the offset of the map rho = sqrt(3) psi + 3/2
  of App. B).
* CDFT freezing run: nu = 2.362, gamma = 2, delta = 1e-10, domain [0,17)^2 on
  128^2 (h = 17/128), s = 0.02; mean density 6 * 0.6 / pi (number density at
  packing fraction 0.6; the printed "pi/6 x 0.6" makes the uniform state stable,
  against the text).
* Sheared-nanocrystal run: eps = 0.4, coexistence densities 0.72958 and 0.90073,
  h = pi / (2 sqrt 3), s = 0.02.
* Gradient-flow variant (Thm. thm_grad; the paper runs no experiment with it):
  the PFC and CDFT freezing runs' constants, grids and initial densities.
"""
import math
from dataclasses import dataclass, asdict

import numpy as np

PFC_EPS = 0.025
PFC_RHO_BAR = 1.5 - 0.07 * math.sqrt(3.0)
CDFT_NU = 2.362
CDFT_RHO_BAR = 6.0 * 0.6 / math.pi
NANO_EPS = 0.4
NANO_RHO_L = 0.72958
NANO_RHO_S = 0.90073
NANO_H = math.pi / (2.0 * math.sqrt(3.0))
# Coarsest grid of the benchmark workloads (FAS V(2,2) from n^2 down to 32^2,
# the largest level the one-workgroup tail holds).  On these workloads the
# levels below 32^2 do not change the V-cycles per step (measured with the
# oracle at 128^2 and 256^2: PFC eps = 0.025 and 0.4, CDFT, the gradient flows
# and the channel take the same cycle counts with coarsest 4^2 to 64^2).
BENCH_COARSEST_N = 32


@dataclass
class Config:
    """Parameters of one instance (the C ABI's parameter block carries the same
    values)."""
    model: str                 # "pfc", "cdft", or the gradient flow "pfc_gf", "cdft_gf"
    n: int
    h: float
    s: float
    gamma: float = 2.0
    alpha: float = 1.0 - PFC_EPS
    nu: float = CDFT_NU
    delta: float = 1e-10
    w: float = 0.5
    tol: float = 1e-10
    nu1: int = 2
    nu2: int = 2
    max_cycles: int = 200
    coarsest_n: int = 4
    coarse_sweeps: int = 4
    sigma: float = 1.0
    continuity_fix: bool = True
    precision: str = "fp64"    # "fp64" or "mixed"
    dims: int = 2              # 3: the PFC step on an n^3 grid
    walls: bool = False        # PFC in a channel: walls at y = 0 and y = n h
    u_bot: float = 0.0         # channel: wall speeds (u on the walls, v = 0)
    u_top: float = 0.0

    @property
    def gradflow(self):
        return self.model.endswith("_gf")

    @property
    def base_model(self):
        """"pfc" or "cdft": the free energy, whichever scheme."""
        return self.model[:-3] if self.gradflow else self.model

    def oracle_kwargs(self):
        d = asdict(self)
        d.pop("precision")
        d.pop("n"); d.pop("h"); d.pop("s"); d.pop("model")
        if self.base_model == "pfc":
            d.pop("nu"); d.pop("delta")
        else:
            d.pop("alpha")
        if self.gradflow:
            d.pop("gamma"); d.pop("sigma")
        d.pop("walls"); d.pop("u_bot"); d.pop("u_top"); d.pop("dims")
        return d

    def wall_oracle_kwargs(self):
        """Keyword arguments of oracle.walls.Stepper for a channel config."""
        d = self.oracle_kwargs()
        d.pop("alpha")
        return dict(d, u_bot=self.u_bot, u_top=self.u_top)


def pfc_uniform_noise(n, h, s, seed, rho_bar=PFC_RHO_BAR, amp=0.05, **kw):
    """rho = rho_bar + amp * U(-1, 1), u = v = 0."""
    rng = np.random.default_rng(seed)
    rho = rho_bar + amp * rng.uniform(-1.0, 1.0, (n, n))
    z = np.zeros((n, n))
    return Config("pfc", n, h, s, **kw), rho, z.copy(), z.copy()


def cdft_gauss_noise(n, h, s, seed, rho_bar=CDFT_RHO_BAR, amp=0.02, **kw):
    """rho = rho_bar + amp * N(0, 1), u = v = 0."""
    rng = np.random.default_rng(seed)
    rho = rho_bar + amp * rng.standard_normal((n, n))
    z = np.zeros((n, n))
    return Config("cdft", n, h, s, **kw), rho, z.copy(), z.copy()


def cdft_vacuum_lattice(n, seed=0, h=0.53125, period=4.25, rho_min=1e-3, amp=2.0, speed=0.6, s=0.03, **kw):
    """A CDFT state near vacuum between its peaks, for the positivity projection
    of Sec. 6: a square lattice of peaks of the given period,
    rho = rho_min + amp * b (1 + 0.05 U(-1, 1)), b = [(1 + cos kx)(1 + cos ky)/4]^2,
    k = 2 pi / period, so rho falls to rho_min in the troughs, and a flow out of
    the troughs, u = -speed sin(kx)(1 + 0.1 U(-1, 1)), v = -speed sin(ky)(...),
    strong enough (with s = 0.03) that the continuity update of the first
    V-cycle goes negative at some trough nodes.  n must be a multiple of
    period / h (8 at the defaults)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    k = 2.0 * math.pi / period
    bump = ((1.0 + np.cos(k * X)) * (1.0 + np.cos(k * Y)) / 4.0) ** 2
    rho = rho_min + amp * bump * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, (n, n)))
    u = -speed * np.sin(k * X) * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, (n, n)))
    v = -speed * np.sin(k * Y) * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, (n, n)))
    return Config("cdft", n, h, s, **kw), rho, u, v


def gradflow(model, n, seed=0, precision="fp64", **kw):
    """Gradient-flow workload: "pfc_gf" draws rho as the PFC freezing run
    (rho_bar + 0.05 U(-1, 1), h = 0.25, s = 0.01), "cdft_gf" as the CDFT run
    (rho_bar + 0.02 N(0, 1), h = 17/128, s = 0.02); u = v = 0."""
    if model == "pfc_gf":
        cfg, rho, u, v = pfc_uniform_noise(n, 0.25, 0.01, seed, precision=precision, **kw)
    elif model == "cdft_gf":
        cfg, rho, u, v = cdft_gauss_noise(n, 17.0 / 128.0, 0.02, seed, precision=precision, **kw)
    else:
        raise ValueError(model)
    cfg.model = model
    return cfg, rho, u, v


def nucleate(n, h, eps=NANO_EPS, rho_s=NANO_RHO_S, rho_l=NANO_RHO_L, diag_atoms=13.0):
    """The sheared-nanocrystal initial density (Sec. 6): the one-mode solid
    rho_s + A (cos(sqrt3/2 x + pi) cos(y/2) - cos(y)/2) inside a regular
    hexagon of long diagonal diag_atoms * a (a = 4 pi / sqrt 3, the solid's
    period in x), centred at (L/2, L/2) with that diagonal along x, and the
    uniform liquid rho_l outside; A is the one-mode amplitude the paper gives
    for eps and rho_s.  Shape (n + 1, n): the node rows y = j h, j = 0..n, of
    the channel (walls at j = 0 and j = n)."""
    L = n * h
    x = np.arange(n) * h
    y = np.arange(n + 1) * h
    X, Y = np.meshgrid(x, y)
    dp = rho_s - 1.5
    A = 4.0 / (5.0 * math.sqrt(3.0)) * dp - 4.0 * math.sqrt(3.0) / 15.0 * math.sqrt(15.0 * eps - 12.0 * dp * dp)
    solid = rho_s + A * (np.cos(math.sqrt(3.0) / 2.0 * X + math.pi) * np.cos(0.5 * Y) - 0.5 * np.cos(Y))
    a = 4.0 * math.pi / math.sqrt(3.0)
    R = 0.5 * diag_atoms * a
    dx, dy = np.abs(X - L / 2), np.abs(Y - L / 2)
    inside = (dy <= math.sqrt(3.0) / 2.0 * R) & (math.sqrt(3.0) * dx + dy <= math.sqrt(3.0) * R)
    return np.where(inside, solid, rho_l)


def channel(n=256, u_wall=0.1, seed=None, amp=0.0, **kw):
    """The sheared-nanocrystal run of Sec. 6 in a channel of n x (n + 1) node
    rows: eps = 0.4, h = pi/(2 sqrt 3), s = 0.02, walls at -u_wall (bottom) and
    +u_wall (top), the hexagonal nucleate of ``nucleate`` (13 atoms along its
    diagonal) in the liquid at rest; with seed given, amp * U(-1, 1) noise is
    added to rho (smaller grids for tests)."""
    rho = nucleate(n, NANO_H)
    if seed is not None:
        rho = rho + amp * np.random.default_rng(seed).uniform(-1.0, 1.0, rho.shape)
    z = np.zeros_like(rho)
    cfg = Config("pfc", n, NANO_H, 0.02, alpha=1.0 - NANO_EPS, walls=True, u_bot=-u_wall, u_top=u_wall, **kw)
    return cfg, rho, z.copy(), z.copy()


def pfc3d(n=128, seed=0, h=0.5, s=0.01, amp=0.05, uamp=0.0, **kw):
    """The PFC step in three dimensions: the PFC freezing run's law
    (eps = 0.025, rho = rho_bar + amp U(-1, 1)) on n^3 nodes, h = 0.5,
    s = 0.01 (s/h^4 = 0.16: the damped block smoother needs s/h^4 below about
    0.5 in 3D); with uamp, velocities uamp N(0, 1).  Fields [z, y, x]."""
    rng = np.random.default_rng(seed)
    rho = PFC_RHO_BAR + amp * rng.uniform(-1.0, 1.0, (n, n, n))
    if uamp:
        u, v, w = uamp * rng.standard_normal((3, n, n, n))
    else:
        u = v = w = np.zeros((n, n, n))
    cfg = Config("pfc", n, h, s, dims=3, **kw)
    return cfg, rho, u, v, w


def random_velocity(n, seed, amp):
    rng = np.random.default_rng(seed)
    return amp * rng.uniform(-1.0, 1.0, (n, n)), amp * rng.uniform(-1.0, 1.0, (n, n))


# ---- the workloads of the benchmark and parity suite ----------------------

def pfc_freezing_32(seed=0):
    """PFC, 32^2, h = 0.25, s = 0.01, 10 steps, FP64, V(2,2), tol 1e-10."""
    return pfc_uniform_noise(32, 0.25, 0.01, seed)


def pfc_freezing_512(seed=0, precision="fp64", n=512):
    """PFC, 512^2, h = 0.25, s = 0.01, 100 steps; FP64 or mixed precision;
    V(2,2) down to a 32^2 coarsest grid."""
    return pfc_uniform_noise(n, 0.25, 0.01, seed, precision=precision, coarsest_n=BENCH_COARSEST_N)


def cdft_freezing_1024(seed=0, n=1024):
    """CDFT, 1024^2, h = 17/128, s = 0.02, rho_bar + 0.02 N(0,1), 50 steps;
    V(2,2) down to a 32^2 coarsest grid."""
    return cdft_gauss_noise(n, 17.0 / 128.0, 0.02, seed, coarsest_n=BENCH_COARSEST_N)


def pfc_nanocrystal_batch(count=256, seed=0, sizes=(64, 128, 256), precision="mixed"):
    """Batch of independent PFC instances (eps = 0.4, h = pi/(2 sqrt 3), s = 0.02),
    n ~ U{sizes}, rho_bar ~ U(rho_l, rho_s), rho = rho_bar + 0.05 U(-1,1);
    instance i draws its field from seed 1000 + i."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    rbs = rng.uniform(NANO_RHO_L, NANO_RHO_S, size=count)
    out = []
    for i, (n, rb) in enumerate(zip(ns, rbs)):
        cfg, rho, u, v = pfc_uniform_noise(int(n), NANO_H, 0.02, 1000 + i,
                                           rho_bar=float(rb), alpha=1.0 - NANO_EPS,
                                           precision=precision,
                                           coarsest_n=min(BENCH_COARSEST_N, int(n) // 2))
        out.append((cfg, rho, u, v))
    return out


class Request:
    """One request of a serving stream: arrival time, steps, parameters, and
    its initial state, drawn from its own seed when first read (so a stream of
    thousands of requests holds no fields until they are served)."""

    def __init__(self, rid, arrival, steps, cfg, draw):
        self.rid, self.arrival, self.steps, self.cfg = rid, arrival, steps, cfg
        self._draw = draw
        self._state = None

    def state(self):
        if self._state is None:
            self._state = self._draw()
        return self._state

    @property
    def rho(self):
        return self.state()[0]

    @property
    def u(self):
        return self.state()[1]

    @property
    def v(self):
        return self.state()[2]

    def drop_state(self):
        """Forgets the drawn state (it is drawn again, identically, if read)."""
        self._state = None

    def fix_state(self, rho, u, v):
        """Replaces the state the request would draw (simulated backends)."""
        self._state = (rho, u, v)
        self._draw = lambda: (rho, u, v)

    def __repr__(self):
        return f"Request(rid={self.rid}, arrival={self.arrival:.4f}, steps={self.steps}, model={self.cfg.model}, n={self.cfg.n})"


def serving_stream(count, rate, seed=0, sizes=(64, 128, 256, 512, 1024),
                   steps=(10, 200), pfc_precision="mixed", cdft_precision="fp64"):
    """Poisson request stream: exponential inter-arrival times of mean 1/rate,
    model PFC or CDFT with probability 1/2 each, n ~ U{sizes},
    steps ~ U{steps[0]..steps[1]}.  PFC requests are drawn as in ``pfc_nanocrystal_batch``
    (mixed precision by default), CDFT requests as in ``cdft_freezing_1024`` at their own
    size (FP64 by default)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(np.asarray(sizes)))
        nst = int(rng.integers(steps[0], steps[1] + 1))
        cn = min(BENCH_COARSEST_N, n // 2)
        if rng.uniform() < 0.5:
            rb = float(rng.uniform(NANO_RHO_L, NANO_RHO_S))
            cfg = Config("pfc", n, NANO_H, 0.02, alpha=1.0 - NANO_EPS, precision=pfc_precision, coarsest_n=cn)
            draw = (lambda n=n, i=i, rb=rb: pfc_uniform_noise(n, NANO_H, 0.02, 5000 + i, rho_bar=rb)[1:])
        else:
            cfg = Config("cdft", n, 17.0 / 128.0, 0.02, precision=cdft_precision, coarsest_n=cn)
            draw = (lambda n=n, i=i: cdft_gauss_noise(n, 17.0 / 128.0, 0.02, 5000 + i)[1:])
        reqs.append(Request(i, t, nst, cfg, draw))
    return reqs


def paper_convergence_ic(n, model, L=32.0):
    """Smooth initial density of the paper's convergence tests (Sec. 6.1.1 for
    CDFT with mean 6*0.6/pi, Sec. 6.1.2 for PFC with offset 3/2); u = v = 0."""
    h = L / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    p = (-0.02 * np.cos(2 * np.pi * (X - 12) / 32) * np.sin(2 * np.pi * (Y - 1) / 32)
         + 0.02 * np.cos(np.pi * (X + 10) / 32) ** 2 * np.cos(np.pi * (Y + 3) / 32) ** 2
         - 0.01 * np.sin(4 * np.pi * X / 32) ** 2 * np.sin(4 * np.pi * (Y - 6) / 32) ** 2)
    if model == "pfc":
        rho = math.sqrt(3.0) * (-0.07 + p) + 1.5
    else:
        rho = CDFT_RHO_BAR + p
    z = np.zeros((n, n))
    return rho, z.copy(), z.copy()
