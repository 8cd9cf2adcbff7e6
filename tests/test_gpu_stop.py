"""GPU: the device-side stop test (V-cycles enqueued in batches, each ending
in a kernel that raises a stop flag once ||S - N(g)||_2 <= tol; later cycles'
kernels return at once) runs exactly the cycles the host-tested loop runs:
same V-cycle counts, same final norms, bitwise the same states.  The host
loop is what runs without HIP graphs (HFZ_GRAPH=0)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def run(monkeypatch, graph, cfg, rho, u, v, steps, max_cycles=None):
    import paper_1503_07416_amd as pkg
    monkeypatch.setenv("HFZ_GRAPH", "1" if graph else "0")
    if max_cycles is not None:
        cfg = type(cfg)(**{**cfg.__dict__, "max_cycles": max_cycles})
    sim = pkg.Simulation(cfg)
    sim.set_state(rho, u, v)
    per = []
    for _ in range(steps):
        rc, st = sim.step(1, raise_on_error=False)
        per.append((rc, st.steps_done, st.cycles_last, st.residual_last))
    out = [x.cpu().numpy() for x in sim.get_state()]
    sim.close()
    return per, out


@pytest.mark.parametrize("model,precision", [("pfc", "fp64"), ("pfc", "mixed"), ("cdft", "fp64"),
                                             ("cdft", "mixed")])
def test_device_stop_equals_host_stop(monkeypatch, model, precision):
    if model == "pfc":
        cfg, rho, u, v = workloads.pfc_uniform_noise(128, 0.25, 0.01, 9, precision=precision)
    else:
        cfg, rho, u, v = workloads.cdft_gauss_noise(128, 17.0 / 64.0, 0.02, 9, precision=precision)
    a, sa = run(monkeypatch, True, cfg, rho, u, v, 4)
    b, sb = run(monkeypatch, False, cfg, rho, u, v, 4)
    assert a == b
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)


def test_device_stop_max_cycles(monkeypatch):
    """max_cycles reached: HFZ_ENOCONV after exactly max_cycles cycles, the
    state is that of the previous step, in both loops."""
    cfg, rho, u, v = workloads.pfc_uniform_noise(64, 0.25, 0.01, 3)
    a, sa = run(monkeypatch, True, cfg, rho, u, v, 2, max_cycles=3)
    b, sb = run(monkeypatch, False, cfg, rho, u, v, 2, max_cycles=3)
    assert a == b
    assert a[0][0] == -4 and a[0][1] == 0 and a[0][2] == 3
    for x, y, z in zip(sa, sb, (rho, u, v)):
        assert np.array_equal(x, y) and np.array_equal(x, z)
