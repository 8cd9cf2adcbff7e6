"""Shared test helpers: oracle construction from a workload config, error
metrics, and the GPU availability switch."""
import numpy as np

from oracle import gradflow, three_d, walls
from oracle.fas import Stepper


def oracle_stepper(cfg):
    """The oracle's stepper of a workload config (the hydrodynamic scheme or
    its gradient-flow variant)."""
    if getattr(cfg, "gradflow", False):
        return gradflow.Stepper(cfg.base_model, cfg.n, cfg.h, cfg.s, **cfg.oracle_kwargs())
    if getattr(cfg, "dims", 2) == 3:
        kw = cfg.oracle_kwargs()
        kw.pop("alpha")
        return three_d.Stepper(cfg.n, cfg.h, cfg.s, cfg.alpha, **kw)
    if getattr(cfg, "walls", False):
        return walls.Stepper(cfg.n, cfg.h, cfg.s, cfg.alpha, **cfg.wall_oracle_kwargs())
    return Stepper(cfg.model, cfg.n, cfg.h, cfg.s, **cfg.oracle_kwargs())


def rel_err(a, b):
    """||a - b||_inf / ||b||_inf (b is the oracle)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def state_errors(gpu_state, ora_state):
    """Per-field relative errors; the two velocity components share the scale
    max(|u|, |v|) of the oracle."""
    r, u, v = [np.asarray(x) for x in gpu_state]
    R, U, V = [np.asarray(x) for x in ora_state]
    vs = max(np.abs(U).max(), np.abs(V).max(), 1e-300)
    return (rel_err(r, R), float(np.abs(u - U).max() / vs), float(np.abs(v - V).max() / vs))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
