"""GPU: the batched solver gives, for every instance, the result the
single-instance solver gives for that instance alone (same device code, same
per-instance stop test, same V-cycle count; the two kernels are compiled
separately, so floating-point contraction may differ in the last bit), for
both precisions and both models; it also agrees with the CPU oracle."""
import numpy as np
import pytest

import workloads
from tests.helpers import oracle_stepper, state_errors

pytestmark = pytest.mark.gpu


def np_(t):
    return t.cpu().numpy()


def instances(model, n, count, precision, seed=0):
    out = []
    rng = np.random.default_rng(seed)
    for i in range(count):
        if model == "pfc":
            rb = float(rng.uniform(workloads.NANO_RHO_L, workloads.NANO_RHO_S))
            amp = 0.05 * (0.2 + i / count)   # uneven: different cycle counts
            out.append(workloads.pfc_uniform_noise(n, workloads.NANO_H, 0.02, 100 + i, rho_bar=rb, amp=amp,
                                                   alpha=1.0 - workloads.NANO_EPS, precision=precision))
        else:
            out.append(workloads.cdft_gauss_noise(n, 17.0 / 64.0, 0.02, 100 + i, amp=0.01 + 0.01 * i / count,
                                                  precision=precision))
    return out


@pytest.mark.parametrize("model,n,precision", [("pfc", 64, "fp64"), ("pfc", 128, "mixed"),
                                               ("pfc", 32, "mixed"), ("cdft", 64, "mixed"),
                                               ("cdft", 128, "fp64")])
def test_batch_equals_alone(model, n, precision):
    import paper_1503_07416_amd as pkg
    inst = instances(model, n, 5, precision)
    B = pkg.Batch([c for c, _, _, _ in inst])
    for i, (c, r, u, v) in enumerate(inst):
        B.set_state(i, r, u, v)
    stats = B.step(3)
    cyc = [s.cycles_total for s in stats]
    for i, (c, r, u, v) in enumerate(inst):
        sim = pkg.Simulation(c)
        sim.set_state(r, u, v)
        st = sim.step(3)
        assert st.cycles_total == cyc[i]
        a = [np_(x) for x in B.get_state(i)]
        b = [np_(x) for x in sim.get_state()]
        for x, y in zip(a, b):
            scale = max(np.abs(y).max(), 1e-300)
            assert np.abs(x - y).max() <= 1e-13 * scale, (i, np.abs(x - y).max())
        assert abs(B.energy(i)[0] - sim.energy()[0]) <= 1e-13 * abs(sim.energy()[0])


def test_batch_matches_oracle():
    import paper_1503_07416_amd as pkg
    inst = instances("pfc", 64, 3, "mixed", seed=5)
    B = pkg.Batch([c for c, _, _, _ in inst])
    for i, (c, r, u, v) in enumerate(inst):
        B.set_state(i, r, u, v)
    B.step(2)
    for i, (c, r, u, v) in enumerate(inst):
        ora = oracle_stepper(c)
        ora.set_state(r, u, v)
        ora.step()
        ora.step()
        errs = state_errors([np_(x) for x in B.get_state(i)], (ora.rho, ora.u, ora.v))
        assert max(errs) < 1e-6, (i, errs)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_tile_shapes_agree(precision, monkeypatch):
    """From 64^2 up the batched smoother runs 64x16 tiles of 512 threads;
    HFZ_BATCH_TILE=0 (read at batch init) forces the 32x16 tiles of 256.
    The swept values do not depend on the tile: three steps of a 128^2 batch
    agree to rounding, with the same V-cycle counts."""
    import paper_1503_07416_amd as pkg
    inst = instances("pfc", 128, 3, precision, seed=11)
    out = {}
    for tile in ("2", "0"):
        monkeypatch.setenv("HFZ_BATCH_TILE", tile)
        B = pkg.Batch([c for c, _, _, _ in inst])
        for i, (c, r, u, v) in enumerate(inst):
            B.set_state(i, r, u, v)
        stats = B.step(3)
        out[tile] = ([s.cycles_total for s in stats], [[np_(x) for x in B.get_state(i)] for i in range(len(inst))])
    assert out["2"][0] == out["0"][0]
    for a, b in zip(out["2"][1], out["0"][1]):
        for x, y in zip(a, b):
            assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1e-300)


def uneven(model, sizes, precision, seed=0, **kw):
    """Instances of the given grid sizes (in this order, not sorted), each with
    its own seed and amplitude."""
    out = []
    rng = np.random.default_rng(seed)
    for i, n in enumerate(sizes):
        if model == "pfc":
            rb = float(rng.uniform(workloads.NANO_RHO_L, workloads.NANO_RHO_S))
            out.append(workloads.pfc_uniform_noise(n, workloads.NANO_H, 0.02, 300 + i, rho_bar=rb,
                                                   amp=0.02 + 0.01 * i, alpha=1.0 - workloads.NANO_EPS,
                                                   precision=precision, **kw))
        else:
            out.append(workloads.cdft_gauss_noise(n, 17.0 / 64.0, 0.02, 300 + i, amp=0.01 + 0.002 * i,
                                                  precision=precision, **kw))
    return out


@pytest.mark.parametrize("model,precision", [("pfc", "fp64"), ("pfc", "mixed"), ("cdft", "fp64"),
                                             ("cdft", "mixed")])
def test_uneven_batch_equals_alone(model, precision):
    """Instances of 16^2 to 256^2 in one batch (one launch per level depth and
    phase; the 16^2 and 32^2 instances run only in the tail): every instance
    takes the V-cycles it takes alone and ends within 1e-13 of its result
    alone."""
    import paper_1503_07416_amd as pkg
    sizes = [64, 256, 16, 128, 32, 64, 256, 128]
    inst = uneven(model, sizes, precision)
    print(f"uneven batch {model} {precision} {sizes}", flush=True)
    B = pkg.Batch([c for c, _, _, _ in inst])
    for i, (c, r, u, v) in enumerate(inst):
        B.set_state(i, r, u, v)
    stats = B.step(3)
    for i, (c, r, u, v) in enumerate(inst):
        sim = pkg.Simulation(c)
        sim.set_state(r, u, v)
        st = sim.step(3)
        assert stats[i].steps_done == 3
        assert st.cycles_total == stats[i].cycles_total, (i, c.n, st.cycles_total, stats[i].cycles_total)
        a = [np_(x) for x in B.get_state(i)]
        b = [np_(x) for x in sim.get_state()]
        assert a[0].shape == (c.n, c.n)
        for x, y in zip(a, b):
            scale = max(np.abs(y).max(), 1e-300)
            assert np.abs(x - y).max() <= 1e-13 * scale, (i, c.n, np.abs(x - y).max())
        assert abs(B.energy(i)[0] - sim.energy()[0]) <= 1e-13 * abs(sim.energy()[0])


def test_uneven_batch_benchmark_mix_matches_oracle():
    """The benchmark's batch law (PFC eps = 0.4, n ~ U{64, 128, 256}, coarsest
    32^2, mixed precision) on a dozen instances, two steps against the FP64
    oracle (1e-6), and against each instance alone (same V-cycles)."""
    import paper_1503_07416_amd as pkg
    inst = workloads.pfc_nanocrystal_batch(count=12, seed=3)
    assert len({c.n for c, _, _, _ in inst}) == 3
    B = pkg.Batch([c for c, _, _, _ in inst])
    for i, (c, r, u, v) in enumerate(inst):
        B.set_state(i, r, u, v)
    stats = B.step(2)
    for i, (c, r, u, v) in enumerate(inst):
        if c.n <= 128:
            ora = oracle_stepper(c)
            ora.set_state(r, u, v)
            ora.step()
            ora.step()
            errs = state_errors([np_(x) for x in B.get_state(i)], (ora.rho, ora.u, ora.v))
            assert max(errs) < 1e-6, (i, c.n, errs)
        sim = pkg.Simulation(c)
        sim.set_state(r, u, v)
        st = sim.step(2)
        assert st.cycles_total == stats[i].cycles_total, (i, c.n)


def test_uneven_batch_release_and_refill():
    """A slot released and filled again with a new state (a serving pool's
    slot) in a batch of different sizes: the other instances are unaffected
    and the refilled one starts from its new state."""
    import paper_1503_07416_amd as pkg
    inst = uneven("pfc", [128, 64, 32], "mixed", seed=7)
    B = pkg.Batch([c for c, _, _, _ in inst])
    for i, (c, r, u, v) in enumerate(inst):
        B.set_state(i, r, u, v)
    B.step(1)
    B.release(1)
    st = B.step(1)
    assert st[1].steps_done == 0 and st[0].steps_done == 1 and st[2].steps_done == 1
    c, r, u, v = inst[1]
    B.set_state(1, r, u, v)
    B.step(2)
    sim = pkg.Simulation(c)
    sim.set_state(r, u, v)
    sim.step(2)
    for x, y in zip(B.get_state(1), sim.get_state()):
        x, y = np_(x), np_(y)
        assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1e-300)


@pytest.mark.parametrize("model,precision", [("pfc", "fp64"), ("pfc", "mixed"), ("cdft", "fp64"),
                                             ("cdft", "mixed")])
def test_batch_restriction_variants_agree(model, precision, monkeypatch):
    """The batched FAS restriction runs the staged kernel (the fine data under
    a coarse tile through LDS; HFZ_BATCH_RESTRICT=3, the default: coarse tiles
    of 16 and 512 threads; 2: 16 and 256; 1: 8 and 256) or the direct kernel
    (0); the variable is read at batch init.  The same arithmetic in the same
    order: three steps of an uneven batch agree to rounding, with the same
    V-cycle counts."""
    import paper_1503_07416_amd as pkg
    inst = uneven(model, [64, 256, 32, 128, 256], precision, seed=17)
    out = {}
    for mode in ("3", "2", "1", "0"):
        monkeypatch.setenv("HFZ_BATCH_RESTRICT", mode)
        B = pkg.Batch([c for c, _, _, _ in inst])
        for i, (c, r, u, v) in enumerate(inst):
            B.set_state(i, r, u, v)
        stats = B.step(3)
        out[mode] = ([s.cycles_total for s in stats], [[np_(x) for x in B.get_state(i)] for i in range(len(inst))])
        B.close()
    for mode in ("3", "2", "1"):
        assert out[mode][0] == out["0"][0], mode
        for a, b in zip(out[mode][1], out["0"][1]):
            for x, y in zip(a, b):
                assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1e-300), mode
