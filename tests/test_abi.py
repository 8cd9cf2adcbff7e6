"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and its pure host entry points validate parameters."""
import ctypes
import os
import re

import pytest

import paper_1503_07416_amd as pkg
from paper_1503_07416_amd import hfz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "hfz.h")).read()
    return sorted(set(re.findall(r"\b(hfz3?_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    lib = hfz.load()
    names = header_symbols()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(hfz.SYMBOLS) == names


def test_params_struct_matches_header_order():
    txt = open(os.path.join(ROOT, "include", "hfz.h")).read()
    body = txt[txt.index("typedef struct hfz_params"):txt.index("} hfz_params;")]
    fields = re.findall(r"\b(?:int|double)\s+([a-z_0-9, ]+);", body)
    names = [f.strip() for grp in fields for f in grp.split(",")]
    assert names == [f[0] for f in hfz.Params._fields_]


def ws(**kw):
    lib = hfz.load()
    p = hfz.Params()
    model = kw.pop("model", 0)
    assert lib.hfz_default_params(model if model in (0, 1, 2, 3) else 0, ctypes.byref(p)) == 0
    p.model = model
    for k, v in kw.items():
        setattr(p, k, v)
    nb = ctypes.c_size_t(0)
    return lib.hfz_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)), nb.value


def test_workspace_bytes_and_validation():
    rc, nb = ws(n=512)
    assert rc == 0 and nb > 17 * 512 * 512 * 8
    rc2, nb2 = ws(n=1024)
    assert rc2 == 0 and 3.5 < nb2 / nb < 4.5
    rc3, nb3 = ws(model=1, n=1024)
    assert rc3 == 0
    for bad in [dict(n=100), dict(n=4), dict(h=0.0), dict(s=-1.0), dict(gamma=0.0),
                dict(w_damp=1.0), dict(nu1=0, nu2=0), dict(max_cycles=0), dict(coarsest_n=2),
                dict(coarsest_n=64, n=32), dict(sigma=0), dict(precision=3), dict(tol=0.0),
                dict(model=1, n=4096), dict(model=7)]:
        rc, _ = ws(**bad)
        assert rc == -1, bad


def test_strerror():
    lib = hfz.load()
    for code in range(-7, 1):
        assert lib.hfz_strerror(code)


def test_simulation_fails_loudly_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(Exception):
        pkg.Simulation(dict(model="pfc", n=32, h=0.25, s=0.01))


def test_gradient_flow_models_validate():
    """Models 2 and 3 (the gradient flow) size a smaller workspace than their
    hydrodynamic counterparts (fewer unknowns per node), keep the CDFT size
    limit of the row FFT, and are refused by the batched solve."""
    lib = hfz.load()
    for model, base in [(2, 0), (3, 1)]:
        p = hfz.Params()
        assert lib.hfz_default_params(model, ctypes.byref(p)) == 0
        assert p.model == model
        assert (p.delta > 0) == (model == 3)
        rc, nb = ws(model=model, n=512)
        rcb, nbb = ws(model=base, n=512)
        assert rc == 0 and rcb == 0 and nb < nbb
        nbytes = ctypes.c_size_t(0)
        p.n = 64
        assert lib.hfz_batch_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(nbytes)) == -1
    assert ws(model=3, n=4096)[0] == -1
    assert ws(model=4, n=64)[0] == -1
    p = hfz.Params()
    assert lib.hfz_default_params(4, ctypes.byref(p)) == -1


def ws3(**kw):
    lib = hfz.load()
    p = hfz.Params()
    assert lib.hfz_default_params(0, ctypes.byref(p)) == 0
    for k, v in kw.items():
        setattr(p, k, v)
    nb = ctypes.c_size_t(0)
    return lib.hfz3_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)), nb.value


def test_three_d_workspace_and_validation():
    """hfz3_workspace_bytes (host only): the 3D step takes PFC, FP64, no walls,
    8 <= n <= 512; its workspace holds at least the finest level's 28 arrays
    (g, f, d, the tiled sweep's second iterate, rho^k, omega^k) and grows by
    about 8x per doubling of n."""
    rc, nb = ws3(n=128, h=0.5)
    assert rc == 0 and nb > 28 * 128 ** 3 * 8
    rc2, nb2 = ws3(n=256, h=0.5)
    assert rc2 == 0 and 7.5 < nb2 / nb < 8.5
    assert ws3(n=8, h=0.5)[0] == 0
    for bad in [dict(n=100), dict(n=4), dict(n=1024), dict(model=1), dict(walls=1), dict(precision=1),
                dict(coarsest_n=2), dict(coarsest_n=64, n=32), dict(h=0.0), dict(s=-1.0), dict(w_damp=1.0),
                dict(nu1=0, nu2=0), dict(coarse_sweeps=0), dict(sigma=0), dict(tol=0.0)]:
        rc, _ = ws3(**bad)
        assert rc == -1, bad


def test_cycle_shapes_the_tiled_paths_cannot_run_are_refused():
    """The FP32 correction-form inner solve (mixed precision), the channel and
    the batch run only on the tiled kernels, whose pre-sweep launch writes the
    residual field and whose first post-sweep launch applies the coarse-grid
    correction, and on the one-workgroup tail (levels <= 32^2), which must hold
    the coarsest level.  So nu1 = 0, nu2 = 0 and coarsest_n > 32 are refused
    there (HFZ_EINVAL, host only), while the FP64 periodic solve, which has
    per-level kernels for them, accepts them."""
    lib = hfz.load()
    for kw in [dict(nu1=0), dict(nu2=0), dict(coarsest_n=64)]:
        assert ws(n=256, precision=1, **kw)[0] == -1, kw
        assert ws(n=256, walls=1, **kw)[0] == -1, kw
        assert ws(n=256, **kw)[0] == 0, kw
    assert ws(n=256, precision=1, coarsest_n=32)[0] == 0
    assert ws(n=256, precision=1, nu1=1, nu2=1)[0] == 0
    assert ws(model=1, n=256, precision=1, nu1=0, nu2=3)[0] == -1
    for kw, want in [(dict(coarsest_n=64), -1), (dict(coarsest_n=32), 0), (dict(nu1=0), -1),
                     (dict(coarsest_n=8), 0)]:
        for precision in (0, 1):
            p = hfz.Params()
            assert lib.hfz_default_params(0, ctypes.byref(p)) == 0
            p.n, p.precision = 256, precision
            for k, v in kw.items():
                setattr(p, k, v)
            arr = (hfz.Params * 2)(p, p)
            nb = ctypes.c_size_t(0)
            assert lib.hfz_batch_workspace_bytes(arr, 2, ctypes.byref(nb)) == want, (kw, precision)


def test_workspace_too_small_is_enomem():
    """hfz_init, hfz_batch_init and hfz3_init refuse a workspace smaller than
    the size the *_workspace_bytes call reports with HFZ_ENOMEM, before any
    device work (the pointer is never dereferenced)."""
    lib = hfz.load()
    fake = ctypes.c_void_p(1 << 20)  # a 256-byte aligned address nothing reads
    out = ctypes.c_void_p(None)
    for model in (0, 1, 2, 3):
        p = hfz.Params()
        assert lib.hfz_default_params(model, ctypes.byref(p)) == 0
        p.n = 64
        nb = ctypes.c_size_t(0)
        assert lib.hfz_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == 0
        assert lib.hfz_init(ctypes.byref(p), fake, nb.value - 1, None, ctypes.byref(out)) == -2
        assert not out.value
        assert lib.hfz_init(ctypes.byref(p), None, nb.value, None, ctypes.byref(out)) == -2
        if model < 2:
            arr = (hfz.Params * 3)(p, p, p)
            assert lib.hfz_batch_workspace_bytes(arr, 3, ctypes.byref(nb)) == 0
            assert lib.hfz_batch_init(arr, 3, fake, nb.value - 1, None, ctypes.byref(out)) == -2
            assert not out.value
    p = hfz.Params()
    assert lib.hfz_default_params(0, ctypes.byref(p)) == 0
    p.n, p.h = 16, 0.5
    nb = ctypes.c_size_t(0)
    assert lib.hfz3_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == 0
    assert lib.hfz3_init(ctypes.byref(p), fake, nb.value - 1, None, ctypes.byref(out)) == -2
    assert not out.value


def test_batch_accepts_uneven_sizes():
    """The batch takes instances of different grid sizes (host-side sizing);
    it refuses instances that differ in model, precision, cycle shape,
    coarsest grid or coarse sweeps."""
    lib = hfz.load()

    def params(**kw):
        p = hfz.Params()
        assert lib.hfz_default_params(kw.pop("model", 0), ctypes.byref(p)) == 0
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    nb = ctypes.c_size_t(0)
    arr = (hfz.Params * 4)(params(n=64), params(n=256), params(n=16), params(n=128))
    assert lib.hfz_batch_workspace_bytes(arr, 4, ctypes.byref(nb)) == 0
    single = 0
    for n in (64, 256, 16, 128):
        s = ctypes.c_size_t(0)
        assert lib.hfz_workspace_bytes(ctypes.byref(params(n=n)), ctypes.byref(s)) == 0
        single += s.value
    assert nb.value > single
    for bad in [dict(precision=1), dict(nu1=3), dict(coarsest_n=8), dict(coarse_sweeps=5), dict(model=1),
                dict(continuity_fix=0)]:
        arr = (hfz.Params * 2)(params(n=64), params(n=128, **bad))
        assert lib.hfz_batch_workspace_bytes(arr, 2, ctypes.byref(nb)) == -1, bad
