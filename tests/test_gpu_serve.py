"""GPU: continuous batching.  Requests of both models and several grid sizes
stream through the server under a device-memory budget small enough that
requests wait for memory, pools are released and slots are reused; every
request's final state equals the one the single-instance solver gives for it
alone (same V-cycle count, fields within 1e-13 relative: the batched and the
single-instance kernels are compiled separately, so contraction may differ in
the last bit), and the discrete energy does not increase at any step."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_batch_skips_empty_and_released_slots():
    import paper_1503_07416_amd as pkg
    inst = [workloads.pfc_uniform_noise(64, workloads.NANO_H, 0.02, 40 + i, rho_bar=0.8,
                                        alpha=1.0 - workloads.NANO_EPS, precision="mixed") for i in range(3)]
    B = pkg.Batch([c for c, _, _, _ in inst])
    c, r, u, v = inst[0]
    B.set_state(0, r, u, v)                      # slots 1, 2 never filled
    st = B.step(2)
    assert [s.steps_done for s in st] == [2, 0, 0]
    B.set_state(2, *inst[2][1:])
    B.release(0)
    st = B.step(1)
    assert [s.steps_done for s in st] == [0, 0, 1]
    B.set_state(0, r, u, v)                      # a released slot takes a new request
    st = B.step(2)
    assert [s.steps_done for s in st] == [2, 0, 2]
    sim = pkg.Simulation(c)
    sim.set_state(r, u, v)
    sim.step(2)
    for x, y in zip(B.get_state(0), sim.get_state()):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1e-300)


def test_served_equals_alone():
    import paper_1503_07416_amd as pkg
    from paper_1503_07416_amd.serve import DeviceBackend, Server

    reqs = workloads.serving_stream(10, rate=400.0, seed=11, sizes=(64, 128), steps=(2, 5))
    be = DeviceBackend()
    # two slots per pool at most; the budget holds about three 128^2 pools
    big = max(be.pool_bytes(pkg.make_params(r.cfg), 2) for r in reqs)
    budget = 3 * big
    srv = Server(budget, backend=be, pool_target_bytes=big, max_slots=2, keep_results=True, check_energy=True)
    jobs, rep = srv.run(reqs, realtime=True)
    print(rep, flush=True)
    assert rep["completed"] == len(reqs) and rep["failed"] == 0
    assert rep["peak_reserved_bytes"] <= budget
    assert rep["energy_increases"] == 0
    for j in jobs:
        r = j.req
        sim = pkg.Simulation(r.cfg)
        sim.set_state(r.rho, r.u, r.v)
        st = sim.step(r.steps)
        assert st.cycles_total == j.cycles, (r.rid, st.cycles_total, j.cycles)
        for x, y in zip(j.result, sim.get_state()):
            y = y.cpu().numpy()
            assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1e-300), (r.rid, np.abs(x - y).max())
        sim.close()
