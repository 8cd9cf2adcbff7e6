"""ctypes binding of the hfz C ABI (include/hfz.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides the device memory (the workspace and state tensors) and the
stream.  Importing works without a GPU; creating a ``Simulation`` needs the
built library and a HIP device and raises otherwise.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhfz.so")

PFC, CDFT, PFC_GF, CDFT_GF = 0, 1, 2, 3
MODELS = {"pfc": PFC, "cdft": CDFT, "pfc_gf": PFC_GF, "cdft_gf": CDFT_GF}
FP64, MIXED = 0, 1
OK, EINVAL, ENOMEM, EDOMAIN, ENOCONV, ENAN, EHIP, ESTATE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8

ERRORS = {0: "HFZ_OK", -1: "HFZ_EINVAL", -2: "HFZ_ENOMEM", -3: "HFZ_EDOMAIN",
          -4: "HFZ_ENOCONV", -5: "HFZ_ENAN", -6: "HFZ_EHIP", -7: "HFZ_ESTATE", -8: "HFZ_ESCRATCH"}

# names exported by the library (include/hfz.h)
SYMBOLS = [
    "hfz_default_params", "hfz_workspace_bytes", "hfz_init", "hfz_set_state",
    "hfz_get_state", "hfz_get_aux", "hfz_step", "hfz_energy", "hfz_mass",
    "hfz_begin_step", "hfz_smooth", "hfz_vcycle", "hfz_residual", "hfz_finish_step",
    "hfz_read_field", "hfz_write_field", "hfz_info", "hfz_tile_shape", "hfz_destroy", "hfz_strerror",
    "hfz_step_noalloc",
    "hfz_batch_workspace_bytes", "hfz_batch_init", "hfz_batch_set_state", "hfz_batch_get_state",
    "hfz_batch_energy", "hfz_batch_release", "hfz_batch_step", "hfz_batch_destroy",
    "hfz3_workspace_bytes", "hfz3_init", "hfz3_set_state", "hfz3_get_state", "hfz3_step", "hfz3_energy",
    "hfz3_mass", "hfz3_begin_step", "hfz3_smooth", "hfz3_vcycle", "hfz3_residual", "hfz3_finish_step",
    "hfz3_read_field", "hfz3_levels", "hfz3_destroy",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int), ("n", ctypes.c_int),
        ("h", ctypes.c_double), ("s", ctypes.c_double), ("gamma", ctypes.c_double),
        ("alpha", ctypes.c_double), ("nu", ctypes.c_double), ("delta", ctypes.c_double),
        ("w_damp", ctypes.c_double), ("tol", ctypes.c_double),
        ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("max_cycles", ctypes.c_int),
        ("coarsest_n", ctypes.c_int), ("coarse_sweeps", ctypes.c_int),
        ("precision", ctypes.c_int), ("sigma", ctypes.c_int), ("continuity_fix", ctypes.c_int),
        ("walls", ctypes.c_int), ("u_wall_bottom", ctypes.c_double), ("u_wall_top", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int), ("cycles_last", ctypes.c_int),
                ("cycles_total", ctypes.c_longlong), ("residual_last", ctypes.c_double)]


class HfzError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {ERRORS.get(code, code)}")


_lib = None


def load():
    """Loads libhfz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "hfz_default_params": [i, P(Params)],
        "hfz_workspace_bytes": [P(Params), P(ctypes.c_size_t)],
        "hfz_init": [P(Params), vp, ctypes.c_size_t, vp, P(vp)],
        "hfz_set_state": [vp, vp, vp, vp],
        "hfz_get_state": [vp, vp, vp, vp],
        "hfz_get_aux": [vp, vp, vp],
        "hfz_step": [vp, i, P(Stats)],
        "hfz_energy": [vp, P(d)],
        "hfz_mass": [vp, P(d)],
        "hfz_begin_step": [vp],
        "hfz_smooth": [vp, i, i],
        "hfz_vcycle": [vp, i],
        "hfz_residual": [vp, P(d)],
        "hfz_finish_step": [vp],
        "hfz_read_field": [vp, i, i, i, vp],
        "hfz_write_field": [vp, i, i, i, vp],
        "hfz_info": [vp, P(i), P(d)],
        "hfz_tile_shape": [vp, i, P(i), P(i), P(i)],
        "hfz_destroy": [vp],
        "hfz_strerror": [i],
        "hfz_step_noalloc": [P(Params), vp, vp, vp, i, vp, P(Stats)],
        "hfz_batch_workspace_bytes": [P(Params), i, P(ctypes.c_size_t)],
        "hfz_batch_init": [P(Params), i, vp, ctypes.c_size_t, vp, P(vp)],
        "hfz_batch_set_state": [vp, i, vp, vp, vp],
        "hfz_batch_get_state": [vp, i, vp, vp, vp],
        "hfz_batch_energy": [vp, i, P(d)],
        "hfz_batch_release": [vp, i],
        "hfz_batch_step": [vp, i, P(Stats)],
        "hfz_batch_destroy": [vp],
        "hfz3_workspace_bytes": [P(Params), P(ctypes.c_size_t)],
        "hfz3_init": [P(Params), vp, ctypes.c_size_t, vp, P(vp)],
        "hfz3_set_state": [vp, vp, vp, vp, vp],
        "hfz3_get_state": [vp, vp, vp, vp, vp],
        "hfz3_step": [vp, i, P(Stats)],
        "hfz3_energy": [vp, P(d)],
        "hfz3_mass": [vp, P(d)],
        "hfz3_begin_step": [vp],
        "hfz3_smooth": [vp, i, i],
        "hfz3_vcycle": [vp, i],
        "hfz3_residual": [vp, P(d)],
        "hfz3_finish_step": [vp],
        "hfz3_read_field": [vp, i, i, i, vp],
        "hfz3_levels": [vp, P(i)],
        "hfz3_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "hfz_strerror" else ctypes.c_int
    _lib = lib
    return lib


def check(rc, what):
    if rc != 0:
        raise HfzError(rc, what)


def make_params(cfg):
    """Params from a mapping or object with the fields of workloads.Config."""
    get = (lambda k, dflt=None: cfg.get(k, dflt)) if isinstance(cfg, dict) else \
          (lambda k, dflt=None: getattr(cfg, k, dflt))
    lib = load()
    model = MODELS[get("model")]
    p = Params()
    check(lib.hfz_default_params(model, ctypes.byref(p)), "hfz_default_params")
    p.n = int(get("n"))
    p.h, p.s = float(get("h")), float(get("s"))
    for k, attr in [("gamma", "gamma"), ("alpha", "alpha"), ("nu", "nu"), ("delta", "delta"),
                    ("w", "w_damp"), ("tol", "tol")]:
        v = get(k)
        if v is not None:
            setattr(p, attr, float(v))
    for k in ["nu1", "nu2", "max_cycles", "coarsest_n", "coarse_sweeps"]:
        v = get(k)
        if v is not None:
            setattr(p, k, int(v))
    sg = get("sigma")
    if sg is not None:
        p.sigma = int(round(sg))
    cf = get("continuity_fix")
    if cf is not None:
        p.continuity_fix = int(bool(cf))
    prec = get("precision", "fp64")
    p.precision = MIXED if prec == "mixed" else FP64
    if get("walls"):
        p.walls = 1
        p.u_wall_bottom = float(get("u_bot", 0.0))
        p.u_wall_top = float(get("u_top", 0.0))
    return p


def workspace_bytes(p):
    nb = ctypes.c_size_t(0)
    check(load().hfz_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)), "hfz_workspace_bytes")
    return nb.value


def _ptr(t):
    return ctypes.c_void_p(None if t is None else t.data_ptr())


def step_noalloc(cfg, rho, u=None, v=None, nsteps=1, stream=None, raise_on_error=True):
    """hfz_step_noalloc: advances the state held in the float64 device tensors
    rho, u, v (contiguous, n x n; updated in place) by nsteps steps, with the
    library's static device scratch as workspace (no device allocation).
    Returns the step statistics, or (rc, stats) with raise_on_error=False."""
    lib = load()
    p = make_params(cfg)
    for t in (rho, u, v):
        if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError("state tensors must be contiguous float64 device tensors")
    s = stream if stream is not None else torch.cuda.current_stream(rho.device)
    torch.cuda.current_stream(rho.device).synchronize()
    st = Stats()
    rc = lib.hfz_step_noalloc(ctypes.byref(p), _ptr(rho), _ptr(u), _ptr(v), int(nsteps),
                              ctypes.c_void_p(s.cuda_stream), ctypes.byref(st))
    if raise_on_error:
        check(rc, "hfz_step_noalloc")
        return st
    return rc, st


class Simulation:
    """One instance: a handle over a torch-owned device workspace."""

    def __init__(self, cfg, device="cuda", stream=None):
        self.lib = load()
        self.p = make_params(cfg)
        self.n = self.p.n
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nbytes = workspace_bytes(self.p)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        check(self.lib.hfz_init(ctypes.byref(self.p), _ptr(self.ws), self.nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "hfz_init")
        self.h = h

    def _dev(self, a):
        t = torch.as_tensor(a, dtype=torch.float64)
        return t.to(self.device).contiguous()

    def _empty(self, n=None):
        """A field of a level of size n: n x n, or (n + 1) x n in a channel."""
        n = self.n if n is None else n
        return torch.empty((n + self.p.walls, n), dtype=torch.float64, device=self.device)

    @property
    def gradflow(self):
        return self.p.model in (PFC_GF, CDFT_GF)

    def set_state(self, rho, u=None, v=None):
        """(rho, u, v), each n x n (a channel: (n + 1) x n, rows 0..n); the
        gradient-flow models take rho alone (u, v ignored)."""
        shape = (self.n + self.p.walls, self.n)
        r = self._dev(rho)
        if self.gradflow:
            uu = vv = None
        else:
            uu, vv = self._dev(u), self._dev(v)
        for t in (r, uu, vv):
            if t is not None and tuple(t.shape) != shape:
                raise ValueError(f"state field of shape {tuple(t.shape)}, expected {shape}")
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.hfz_set_state(self.h, _ptr(r), _ptr(uu), _ptr(vv)), "hfz_set_state")

    def get_state(self):
        r, u, v = self._empty(), self._empty(), self._empty()
        check(self.lib.hfz_get_state(self.h, _ptr(r), _ptr(u), _ptr(v)), "hfz_get_state")
        return r, u, v

    def get_aux(self):
        """(mu, kappa) of the last solve; kappa is None for the CDFT gradient flow."""
        mu = self._empty()
        ka = None if self.p.model == CDFT_GF else self._empty()
        check(self.lib.hfz_get_aux(self.h, _ptr(mu), _ptr(ka)), "hfz_get_aux")
        return mu, ka

    def step(self, nsteps=1, raise_on_error=True):
        st = Stats()
        rc = self.lib.hfz_step(self.h, int(nsteps), ctypes.byref(st))
        if raise_on_error:
            check(rc, "hfz_step")
        return (rc, st) if not raise_on_error else st

    def energy(self):
        out = (ctypes.c_double * 5)()
        check(self.lib.hfz_energy(self.h, out), "hfz_energy")
        return list(out)

    def mass(self):
        m = ctypes.c_double()
        check(self.lib.hfz_mass(self.h, ctypes.byref(m)), "hfz_mass")
        return m.value

    # stage-level access
    def begin_step(self):
        check(self.lib.hfz_begin_step(self.h), "hfz_begin_step")

    def smooth(self, level, sweeps):
        check(self.lib.hfz_smooth(self.h, int(level), int(sweeps)), "hfz_smooth")

    def vcycle(self, count=1):
        check(self.lib.hfz_vcycle(self.h, int(count)), "hfz_vcycle")

    def residual(self):
        r = ctypes.c_double()
        check(self.lib.hfz_residual(self.h, ctypes.byref(r)), "hfz_residual")
        return r.value

    def finish_step(self):
        check(self.lib.hfz_finish_step(self.h), "hfz_finish_step")

    def levels(self):
        lv, ce = ctypes.c_int(), ctypes.c_double()
        check(self.lib.hfz_info(self.h, ctypes.byref(lv), ctypes.byref(ce)), "hfz_info")
        return lv.value

    def ce(self):
        lv, ce = ctypes.c_int(), ctypes.c_double()
        check(self.lib.hfz_info(self.h, ctypes.byref(lv), ctypes.byref(ce)), "hfz_info")
        return ce.value

    def tile_shape(self, level):
        """(tx, ty, threads) of the tiled sweep kernel on FP64 level `level`, or
        None where the coarse tail sweeps the level."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rc = self.lib.hfz_tile_shape(self.h, int(level), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return (a.value, b.value, c.value) if rc == 0 else None

    def read(self, which, level, comp):
        t = self._empty(self.n >> level)
        check(self.lib.hfz_read_field(self.h, which, level, comp, _ptr(t)), "hfz_read_field")
        return t

    def write(self, which, level, comp, arr):
        t = self._dev(arr)
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.hfz_write_field(self.h, which, level, comp, _ptr(t)), "hfz_write_field")

    def close(self):
        if self.h is not None:
            self.lib.hfz_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation3:
    """The PFC step in three dimensions (hfz3_*): one handle over a
    torch-owned device workspace; fields n x n x n, indexed [z, y, x]."""

    def __init__(self, cfg, device="cuda", stream=None):
        self.lib = load()
        self.p = make_params(cfg)
        self.n = self.p.n
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = ctypes.c_size_t(0)
        check(self.lib.hfz3_workspace_bytes(ctypes.byref(self.p), ctypes.byref(nb)), "hfz3_workspace_bytes")
        self.nbytes = nb.value
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        check(self.lib.hfz3_init(ctypes.byref(self.p), _ptr(self.ws), self.nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "hfz3_init")
        self.h = h

    def _dev(self, a):
        t = torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != (self.n,) * 3:
            raise ValueError(f"field of shape {tuple(t.shape)}, expected {(self.n,) * 3}")
        return t

    def _empty(self, n=None):
        n = self.n if n is None else n
        return torch.empty((n, n, n), dtype=torch.float64, device=self.device)

    def set_state(self, rho, u, v, w):
        t = [self._dev(x) for x in (rho, u, v, w)]
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.hfz3_set_state(self.h, *[_ptr(x) for x in t]), "hfz3_set_state")

    def get_state(self):
        out = [self._empty() for _ in range(4)]
        check(self.lib.hfz3_get_state(self.h, *[_ptr(x) for x in out]), "hfz3_get_state")
        return out

    def step(self, nsteps=1, raise_on_error=True):
        st = Stats()
        rc = self.lib.hfz3_step(self.h, int(nsteps), ctypes.byref(st))
        if raise_on_error:
            check(rc, "hfz3_step")
        return (rc, st) if not raise_on_error else st

    def energy(self):
        out = (ctypes.c_double * 3)()
        check(self.lib.hfz3_energy(self.h, out), "hfz3_energy")
        return tuple(out)

    def mass(self):
        m = ctypes.c_double()
        check(self.lib.hfz3_mass(self.h, ctypes.byref(m)), "hfz3_mass")
        return m.value

    def begin_step(self):
        check(self.lib.hfz3_begin_step(self.h), "hfz3_begin_step")

    def smooth(self, level, sweeps):
        check(self.lib.hfz3_smooth(self.h, int(level), int(sweeps)), "hfz3_smooth")

    def vcycle(self, count=1):
        check(self.lib.hfz3_vcycle(self.h, int(count)), "hfz3_vcycle")

    def residual(self):
        r = ctypes.c_double()
        check(self.lib.hfz3_residual(self.h, ctypes.byref(r)), "hfz3_residual")
        return r.value

    def finish_step(self):
        check(self.lib.hfz3_finish_step(self.h), "hfz3_finish_step")

    def levels(self):
        lv = ctypes.c_int()
        check(self.lib.hfz3_levels(self.h, ctypes.byref(lv)), "hfz3_levels")
        return lv.value

    def read(self, which, level, comp):
        t = self._empty(self.n >> level)
        check(self.lib.hfz3_read_field(self.h, which, level, comp, _ptr(t)), "hfz3_read_field")
        return t

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.hfz3_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many instances of one model and precision, of any grid sizes, stepped
    together (hfz_batch_* of the C ABI)."""

    def __init__(self, cfgs, device="cuda", stream=None):
        self.lib = load()
        self.count = len(cfgs)
        self.params = (Params * self.count)(*[make_params(c) for c in cfgs])
        self.ns = [p.n for p in self.params]
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = ctypes.c_size_t(0)
        check(self.lib.hfz_batch_workspace_bytes(self.params, self.count, ctypes.byref(nb)),
              "hfz_batch_workspace_bytes")
        self.nbytes = nb.value
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        check(self.lib.hfz_batch_init(self.params, self.count, _ptr(self.ws), self.nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "hfz_batch_init")
        self.h = h

    def set_state(self, i, rho, u, v):
        t = [torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous() for a in (rho, u, v)]
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.hfz_batch_set_state(self.h, i, *[_ptr(x) for x in t]), "hfz_batch_set_state")

    def get_state(self, i):
        n = self.ns[i]
        t = [torch.empty((n, n), dtype=torch.float64, device=self.device) for _ in range(3)]
        check(self.lib.hfz_batch_get_state(self.h, i, *[_ptr(x) for x in t]), "hfz_batch_get_state")
        return t

    def energy(self, i):
        out = (ctypes.c_double * 5)()
        check(self.lib.hfz_batch_energy(self.h, i, out), "hfz_batch_energy")
        return list(out)

    def release(self, i):
        check(self.lib.hfz_batch_release(self.h, i), "hfz_batch_release")

    def step(self, nsteps=1, raise_on_error=True):
        st = (Stats * self.count)()
        rc = self.lib.hfz_batch_step(self.h, int(nsteps), st)
        if raise_on_error:
            check(rc, "hfz_batch_step")
            return list(st)
        return rc, list(st)

    def close(self):
        if self.h is not None:
            self.lib.hfz_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
