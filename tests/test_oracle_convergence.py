"""Refinement pins of the oracle (Sec. 6.1: the scheme is first order in time
and second order in space).

* The paper's convergence tables (golden fixture, Tables DFT1-3 and PFC1-3)
  are internally consistent: each printed rate is log2 of the ratio of the
  printed errors, and the finest rates are near 2.
* Second order in space, exactly measurable in the linear regime: one step of
  a small Fourier mode about the uniform PFC state, at fixed s and physical
  wavenumber, converges to the continuum amplification (the same 2x2 step with
  the continuum symbols k^2, k, written out here) at rate 2 as h halves.
* The paper's nonlinear protocol (smooth initial condition of Sec. 6.1,
  u = 0) on coarse grids: the Cauchy errors fall under refinement.  These
  grids are pre-asymptotic (the paper's own first rates are 7.5 and 2.4); the
  asymptotic rates and the comparison with the printed magnitudes come from
  the GPU path (tests/golden/README.md).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle.fas import Stepper

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "convergence_tables.json")


def test_golden_tables_consistent():
    d = json.load(open(GOLDEN))
    assert len(d["tables"]) == 6
    for name, t in d["tables"].items():
        e, r = t["error"], t["rate"]
        assert len(e) == len(r) == len(d["grids"])
        assert all(a > b for a, b in zip(e[:-1], e[1:])), name
        for k in range(1, len(e)):
            assert abs(math.log2(e[k - 1] / e[k]) - r[k]) < 2e-4, (name, k)
        assert 1.95 < r[-1] < 2.3, name   # second order at the finest pair


def _one_step_amplitude(n, L, s, rb, p, q, A=1e-5):
    """Cosine amplitude of rho after one step (odd part in A), oracle."""
    h = L / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    c = np.cos(2 * np.pi * (p * X + q * Y) / L)
    out = {}
    for sgn in (1, -1):
        st = Stepper("pfc", n, h, s, alpha=0.975, coarse_sweeps=60)
        st.set_state(rb + sgn * A * c, np.zeros((n, n)), np.zeros((n, n)))
        S, om = st.build_source()
        sol = st.solver(om)
        g = st.initial_guess()
        for _ in range(60):
            sol.vcycle(g, S)
        out[sgn] = g[0]
    odd = 0.5 * (out[1] - out[-1])
    return np.sum(odd * c) / np.sum(c * c) / A


def _continuum_amplitude(L, s, rb, p, q, gamma=2.0, alpha=0.975):
    # linearised step with the continuum symbols: Delta -> -k^2, grad -> k,
    # mu' = c_c r^{k+1} - c_e r^k with c_c = (rb - 3/2)^2 + alpha + k^4, c_e = 2 k^2
    k2 = (2 * np.pi / L) ** 2 * (p * p + q * q)
    k = math.sqrt(k2)
    cc, ce = (rb - 1.5) ** 2 + alpha + k2 * k2, 2 * k2
    lhs = np.array([[1.0, 0.5 * s * rb * k], [-s * rb * k * cc, rb + 0.5 * s * gamma * k2]])
    rhs = np.array([[1.0, -0.5 * s * rb * k], [-s * rb * k * ce, rb - 0.5 * s * gamma * k2]])
    return np.linalg.solve(lhs, rhs @ np.array([1.0, 0.0]))[0]


def test_linear_second_order_in_space():
    L, s, rb = 32.0, 0.05, workloads.PFC_RHO_BAR
    exact = _continuum_amplitude(L, s, rb, 1, 1)
    errs = [abs(_one_step_amplitude(n, L, s, rb, 1, 1) - exact) for n in (8, 16, 32, 64)]
    rates = [math.log2(a / b) for a, b in zip(errs[:-1], errs[1:])]
    assert rates[-1] > 1.95 and rates[-2] > 1.9, rates
    assert errs[-1] < 1e-6


@pytest.mark.slow
def test_paper_protocol_errors_fall():
    """Sec. 6.1 initial condition (PFC, offset 3/2), fixed s = 0.01, 10 steps,
    grids 16, 32, 64 on [0,32)^2: Cauchy errors e(16;32) > e(32;64)."""
    sol = {}
    for n in (16, 32, 64):
        rho, u, v = workloads.paper_convergence_ic(n, "pfc")
        st = Stepper("pfc", n, 32.0 / n, 0.01, alpha=1.0 - workloads.PFC_EPS)
        st.set_state(rho, u, v)
        for _ in range(10):
            st.step()
        sol[n] = (st.rho, st.u)
    e = []
    for a, b in ((16, 32), (32, 64)):
        hc = 32.0 / a
        e.append([math.sqrt(hc * hc * ((sol[a][k] - sol[b][k][::2, ::2]) ** 2).sum()) for k in range(2)])
    for k in range(2):
        assert e[1][k] < e[0][k] / 1.8, e
