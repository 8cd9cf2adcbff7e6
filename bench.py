"""Benchmark of the energy-stable FAS step on one MI355X.

Headline (`value`): time steps per second of the PFC 512^2 workload: the
paper's PFC freezing run scaled to 512^2, eps = 0.025, gamma = 2, h = 0.25,
s = 0.01, rho = (3/2 - 0.07 sqrt 3) + 0.05 U(-1,1) (seed 0), u = v = 0, FAS
V(2,2) with the damped red-black smoother to ||S - N(g)||_2 <= 1e-10, FP64.

Also reported on the same JSON line:
  roofline      the finest-level smoother (the LDS-tiled kernel doing two damped
                red-black sweeps), algorithmic bytes / average launch time from
                HIP events on the library's stream; `traffic` from the committed
                FETCH_SIZE / WRITE_SIZE counter summary when it was taken from
                the current kernel sources, else null;
  cpu_baseline  the CPU oracle (NumPy FP64) on a bounded sample;
  mixed         the same workload with FP32 smoothing inside FP64 defect
                correction: steps/s and its distance from the FP64 result;
  precision_sweep  FP64 against mixed precision on the same law at 512^2,
                1024^2 and 2048^2 (steps/s, V-cycles, time per V-cycle);
  batched       256 PFC instances (eps = 0.4, n ~ U{64,128,256}, 20 steps,
                mixed precision) in one batch: instance-steps/s against the
                unbatched FP64 path, and the per-step energy check;
  serving       a Poisson stream of PFC and CDFT requests (n ~ U{64..1024},
                10-200 steps) through the continuous-batching server under a
                budget of 80 % of the device memory, the arrival rate from
                Little's law for that occupancy: p50/p99 per-step latency,
                throughput, peak reserved memory;
  cdft          CDFT 1024^2 (h = 17/128, s = 0.02), 50 steps with the energy
                and mass read after every step;
  gradflow      the gradient-flow variant of the scheme (Thm. thm_grad) with the
                PFC free energy at 512^2 and the CDFT free energy at 1024^2 (the
                freezing runs' constants and initial densities), FP64 and mixed:
                steps/s, V-cycles per step, F and mass checks, and the roofline of
                its finest-level smoother;
  channel       the sheared-nanocrystal run of Sec. 6: PFC (eps = 0.4) in a
                channel of 256 x 257 nodes with walls at rest and at -+0.1 and
                -+0.5, the 13-atom hexagonal nucleate in the liquid: steps/s,
                V-cycles per step, energy (non-increasing with resting walls),
                and the roofline of its finest-level smoother;
  three_d       the PFC step in three dimensions at 128^3 (h = 0.5, s = 0.01):
                steps/s, V-cycles per step, energy and mass checks, and the
                roofline of its smoother (and at 256^3).
"""
import argparse
import dataclasses
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one damped red-black sweep per fine node: read g (5),
# f (5), rho^k, omega^k, write g (5), FP64
SWEEP_BYTES_PFC = 17 * 8
# 3D PFC: read g 6, f 6, rho^k, omega^k 3; write g 6
SWEEP_BYTES_3D = 22 * 8
# the gradient flow: read g, f and write g with 3 (PFC) or 2 (CDFT) unknowns
SWEEP_BYTES_GF = {"pfc_gf": 9 * 8, "cdft_gf": 6 * 8}
KERNEL_SOURCES = ["paper_1503_07416_amd/csrc/tile.hpp", "paper_1503_07416_amd/csrc/stencil.hpp",
                  "paper_1503_07416_amd/csrc/kernels.hpp"]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "smoother_pfc512_fp64_hbm_counters.md")
KERNEL_SOURCES_3D = ["paper_1503_07416_amd/csrc/hfz3.hip"]
TRAFFIC_SUMMARY_3D = os.path.join(ROOT, "profiles", "pfc3d128_fp64_kernels.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="headline and roofline only")
    ap.add_argument("--cpu-cycles", type=int, default=10, help="V-cycles of the oracle sample")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="processes of the parallel oracle sample (0: min(16, host CPUs))")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-hbm-frac", type=float, default=0.8,
                    help="serving budget as a fraction of the device memory")
    ap.add_argument("--serving-only", action="store_true", help="only the serving workload")
    ap.add_argument("--precision-sweep-only", action="store_true",
                    help="only FP64 against mixed precision at 512^2, 1024^2, 2048^2")
    ap.add_argument("--cdft-only", action="store_true", help="only the CDFT 1024^2 workload (for profiles)")
    ap.add_argument("--mixed-only", action="store_true", help="only the mixed-precision PFC workload (for profiles)")
    ap.add_argument("--batched-only", action="store_true", help="only the batched workload (for profiles)")
    ap.add_argument("--gradflow-only", action="store_true", help="only the gradient-flow workloads (for profiles)")
    ap.add_argument("--channel-only", action="store_true", help="only the channel workloads (for profiles)")
    ap.add_argument("--three-d-only", action="store_true", help="only the 3D workload (for profiles)")
    ap.add_argument("--size-sweep-only", action="store_true",
                    help="only the headline smoother at 1024^2, 2048^2, 4096^2")
    ap.add_argument("--counter-probe-3d", action="store_true",
                    help="only launch the 3D smoothers at 128^3 and a reference copy kernel (for counter runs)")
    ap.add_argument("--convergence", action="store_true",
                    help="the paper's convergence study instead of the benchmark (minutes of GPU time)")
    ap.add_argument("--conv-sizes", default="16,32,64,128,256,512")
    ap.add_argument("--conv-tf", type=float, default=10.0)
    ap.add_argument("--probe-tile-shape", type=int, default=9,
                    help="tile shape of the counter probe (9: 64x16/1024, 8: 32x32/1024, the two the "
                         "tuner picks between at 512^2)")
    ap.add_argument("--counter-probe", action="store_true",
                    help="only launch the smoother and a reference copy kernel (for counter runs)")
    return ap.parse_args()


def source_hash(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic_3d(n):
    """HBM bytes per 3D smoother sweep at n^3 from the committed counter
    summary, or None if it is missing, was taken from other sources or at
    another size."""
    try:
        with open(TRAFFIC_SUMMARY_3D) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"source_hash_3d:\s*([0-9a-f]+)", text)
    t = re.search(r"traffic_bytes_per_sweep_%d:\s*([0-9.eE+]+)" % n, text)
    if not m or not t or m.group(1) != source_hash(KERNEL_SOURCES_3D):
        return None
    return float(t.group(1))


def committed_traffic(shape):
    """HBM bytes per smoother launch in tile shape `shape` ("64x16x1024") from
    the committed counter summary (a line traffic_bytes_per_launch_<shape>,
    or tile_shape + traffic_bytes_per_launch), or None if it is missing, was
    taken from other kernel sources or for another tile shape."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != source_hash():
        return None
    t = re.search(r"traffic_bytes_per_launch_%s:\s*([0-9.eE+]+)" % re.escape(shape), text)
    if t:
        return float(t.group(1))
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    sh = re.search(r"tile_shape:\s*([0-9x]+)", text)
    if not t or not sh or sh.group(1) != shape:
        return None
    return float(t.group(1))


def smoother_roofline(sim, n, launches=25, sweep_bytes=SWEEP_BYTES_PFC, model="PFC"):
    """Average duration of one finest-level smoother launch (two damped
    red-black sweeps, as in the V-cycle's smoothing), measured with HIP
    events on the stream the library launches on."""
    import torch
    stream = sim.stream
    sim.begin_step()
    sim.smooth(0, 2)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    sim.smooth(0, 2 * launches)
    stop.record(stream)
    stop.synchronize()
    ms = start.elapsed_time(stop)
    t_launch = ms * 1e-3 / launches
    bytes_launch = 2 * sweep_bytes * n * n
    achieved = bytes_launch / t_launch / 1e9
    tx, ty, nt = sim.tile_shape(0)
    traffic = committed_traffic(f"{tx}x{ty}x{nt}") if (n == 512 and model == "PFC") else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"k_sweeps_tile<{model}, double, 2 sweeps, {tx}x{ty} tile, {nt} threads>",
            "launch_us": round(t_launch * 1e6, 3), "bytes_per_launch": bytes_launch}


def counter_probe(n, shape):
    """Five smoother launches at n^2 in tile shape `shape` (forced: the tuner's
    timings are distorted under a counter-collecting profiler) and three
    launches of a reference copy kernel (torch elementwise multiply, 1 GiB
    read + 1 GiB written), for the FETCH_SIZE / WRITE_SIZE counter runs."""
    os.environ["HFZ_TILE"] = str(shape)
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v = workloads.pfc_uniform_noise(n, 0.25, 0.01, 0)
    sim = pkg.Simulation(cfg, device="cuda:0")
    sim.set_state(rho, u, v)
    sim.begin_step()
    sim.smooth(0, 10)
    x = torch.ones(2**27, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"counter_probe": True, "n": n, "smoother_launches": 5, "copy_bytes_each_way": 2**30,
                      "tile_shape": "x".join(map(str, sim.tile_shape(0))), "source_hash": source_hash()}))


def counter_probe_3d(n=128):
    """Four sweeps at n^3 by the z-marching tiled kernel, four by the two
    per-colour kernels (HFZ3_TILES=0), and three launches of the reference copy
    kernel, for the FETCH_SIZE / WRITE_SIZE counter runs of the 3D smoother."""
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    for tiles in ("128", "0"):
        os.environ["HFZ3_TILES"] = tiles
        cfg, rho, u, v, w = workloads.pfc3d(n)
        sim = pkg.Simulation3(cfg, device="cuda:0")
        sim.set_state(rho, u, v, w)
        sim.begin_step()
        sim.smooth(0, 4)
        torch.cuda.synchronize()
        sim.close()
    os.environ.pop("HFZ3_TILES")
    x = torch.ones(2**27, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"counter_probe_3d": True, "n": n, "sweeps_each": 4, "copy_bytes_each_way": 2**30,
                      "source_hash_3d": source_hash(KERNEL_SOURCES_3D)}))


def oracle_sample(n, vcycles):
    """The oracle (NumPy FP64, one thread) on the headline workload: seconds to
    set up step 1 (source, hierarchy) and seconds per V-cycle over `vcycles`
    V-cycles of it."""
    import workloads
    from oracle.fas import Stepper
    cfg, rho, u, v = workloads.pfc_freezing_512(0, n=n)
    st = Stepper(cfg.model, cfg.n, cfg.h, cfg.s, **cfg.oracle_kwargs())
    st.set_state(rho, u, v)
    t0 = time.perf_counter()
    S, om = st.build_source()
    sol = st.solver(om)
    g = st.initial_guess()
    t1 = time.perf_counter()
    for _ in range(vcycles):
        sol.vcycle(g, S)
    t2 = time.perf_counter()
    return t1 - t0, (t2 - t1) / vcycles


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sample(n, vcycles, processes):
    """Times the oracle sample in this process (one thread), then in
    `processes` child processes at once (each an independent copy, one thread
    each).  Runs before the GPU is used, so the host cores are otherwise idle."""
    import subprocess
    setup, per_cycle = oracle_sample(n, vcycles)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = ("import json, bench; s, c = bench.oracle_sample(%d, %d); print(json.dumps([s, c]))" % (n, vcycles))
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, "-c", code], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                              stderr=subprocess.DEVNULL, text=True) for _ in range(processes)]
    outs = [json.loads(p.communicate()[0].strip().splitlines()[-1]) for p in procs]
    wall = time.perf_counter() - t0
    return {"setup_s": setup, "per_cycle_s": per_cycle, "processes": processes, "parallel_wall_s": wall,
            "parallel_per_cycle_s": [o[1] for o in outs], "parallel_setup_s": [o[0] for o in outs]}


def cpu_baseline(sample, n, cycles_per_step, vcycles):
    """steps/s of the oracle from the sample, extrapolated with the GPU's mean
    V-cycles per step: one process (one thread), and the aggregate of
    `processes` independent copies running at once."""
    per_step = sample["setup_s"] + sample["per_cycle_s"] * cycles_per_step
    par = [s + c * cycles_per_step for s, c in zip(sample["parallel_setup_s"], sample["parallel_per_cycle_s"])]
    return {"value": round(1.0 / per_step, 6), "unit": "time steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{vcycles} V-cycles of step 1 of the {n}^2 workload "
                      f"({sample['setup_s'] + vcycles * sample['per_cycle_s']:.1f} s, one thread), "
                      f"scaled by {cycles_per_step:.2f} V-cycles/step",
            "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
            "parallel": {"processes": sample["processes"], "threads_each": 1,
                         "value": round(sum(1.0 / t for t in par), 6), "unit": "time steps/s (aggregate)",
                         "note": f"{sample['processes']} independent copies of the sample at once "
                                 f"({sample['parallel_wall_s']:.1f} s wall); the oracle itself is single-threaded"}}


def rel_diff(a, b):
    import torch
    out = []
    for x, y in zip(a, b):
        out.append(float((x - y).abs().max() / max(float(y.abs().max()), 1e-300)))
    return max(out)


def run_mixed(a, ref_state):
    """The PFC 512^2 workload in mixed precision: steps/s and max relative distance of the
    final state from the FP64 run's."""
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v = workloads.pfc_freezing_512(0, precision="mixed", n=a.n)
    sim = pkg.Simulation(cfg, device="cuda:0")
    sim.set_state(rho, u, v)
    E = [sim.energy()[0]]
    if a.warmup:
        sim.step(a.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.step(a.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    E.append(sim.energy()[0])
    return {"steps_per_s": round(a.steps / dt, 3), "ms_per_step": round(1e3 * dt / a.steps, 4),
            "outer_cycles_per_step": round(st.cycles_total / max(1, st.steps_done), 3),
            "max_rel_diff_vs_fp64": rel_diff(sim.get_state(), ref_state),
            "energy_decreased": bool(E[1] <= E[0]), "tol": 1e-10}


def run_precision_sweep(sizes=(512, 1024, 2048), steps=5, warmup=2):
    """The headline law (PFC, h = 0.25, s = 0.01, coarsest 32^2, tol 1e-10) at
    growing grid sizes in FP64 and in mixed precision: where the V-cycle is
    bound by latency (the coarse levels) the FP32 inner solve gains little,
    where it is bound by bandwidth it moves half the bytes."""
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    out = {}
    for n in sizes:
        row = {}
        for prec in ("fp64", "mixed"):
            cfg, rho, u, v = workloads.pfc_freezing_512(0, precision=prec, n=n)
            sim = pkg.Simulation(cfg, device="cuda:0")
            sim.set_state(rho, u, v)
            sim.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row[prec] = {"steps_per_s": round(steps / dt, 3),
                         "cycles_per_step": round(st.cycles_total / steps, 3),
                         "us_per_cycle": round(1e6 * dt / max(1, st.cycles_total), 2)}
            sim.close()
            del sim
            torch.cuda.empty_cache()
        row["mixed_over_fp64"] = round(row["mixed"]["steps_per_s"] / row["fp64"]["steps_per_s"], 3)
        out[str(n)] = row
    return out


def run_batched(steps=20, count=256):
    """The batched workload: all instances (grid sizes mixed) in one batch, one launch per
    level depth and phase; then the same instances one at a time through the
    unbatched FP64 path (a sample of 16), and an untimed rerun one step at a
    time reading every instance's energy after each step."""
    import numpy as np
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    inst = workloads.pfc_nanocrystal_batch(count)
    B = pkg.Batch([c for c, _, _, _ in inst], device="cuda:0")

    def load():
        for k, (c, r, u, v) in enumerate(inst):
            B.set_state(k, r, u, v)
        torch.cuda.synchronize()

    load()
    B.step(1)          # warm-up step (captures the batch's V-cycle graph)
    load()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = B.step(steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    cycles = np.mean([s.cycles_total / steps for s in res])
    # unbatched FP64 path on a sample
    sub = inst[::count // 16]
    tu = 0.0
    for c, r, u, v in sub:
        sim = pkg.Simulation(dataclasses.replace(c, precision="fp64"))
        sim.set_state(r, u, v)
        sim.step(1)
        sim.set_state(r, u, v)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        tu += time.perf_counter() - t1
        sim.close()
    unb = len(sub) * steps / tu
    # energy check, untimed: the same instances again, one step at a time
    load()
    viol = 0
    E = [B.energy(i)[0] for i in range(B.count)]
    for _ in range(steps):
        B.step(1)
        for i in range(B.count):
            e = B.energy(i)[0]
            if e > E[i] + 1e-10 * max(1.0, abs(E[i])):
                viol += 1
            E[i] = e
    B.close()
    sizes = {n: sum(1 for c, _, _, _ in inst if c.n == n) for n in sorted({c.n for c, _, _, _ in inst})}
    return {"workload": f"{count} PFC instances, eps=0.4, h=pi/(2 sqrt 3), s=0.02, n~U{{64,128,256}} "
                        f"({', '.join(f'{v} x {k}^2' for k, v in sizes.items())}), one batch, "
                        f"{steps} steps, mixed precision, tol 1e-10",
            "solves_per_s": round(count * steps / T, 1), "seconds": round(T, 4),
            "unbatched_fp64_solves_per_s": round(unb, 1), "unbatched_sample": len(sub),
            "speedup_vs_unbatched_fp64": round(count * steps / T / unb, 2),
            "mean_cycles_per_step": round(float(cycles), 3),
            "energy_increases": viol, "energy_checks": count * steps}


def run_serving(requests, hbm_frac):
    """The serving workload: the budget is hbm_frac (80 %) of the device's memory; a pilot
    per class (alone, mixed PFC / FP64 CDFT) gives the mean residence time,
    and the arrival rate follows Little's law for a mean occupancy of that
    budget, lambda = budget / (E[bytes per request] E[residence]); then the
    Poisson stream through the server."""
    import numpy as np
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    from paper_1503_07416_amd.serve import DeviceBackend, Server
    be = DeviceBackend("cuda:0")
    hbm = torch.cuda.get_device_properties(0).total_memory
    budget = int(hbm_frac * hbm)
    sizes = (64, 128, 256, 512, 1024)
    t_alone, slot = {}, {}
    for model in ("pfc", "cdft"):
        for n in sizes:
            if model == "pfc":
                cfg, r, u, v = workloads.pfc_uniform_noise(n, workloads.NANO_H, 0.02, 77, rho_bar=0.8,
                                                           alpha=1 - workloads.NANO_EPS, precision="mixed",
                                                           coarsest_n=workloads.BENCH_COARSEST_N)
            else:
                cfg, r, u, v = workloads.cdft_gauss_noise(n, 17 / 128, 0.02, 77,
                                                          coarsest_n=workloads.BENCH_COARSEST_N)
            sim = pkg.Simulation(cfg, device="cuda:0")
            sim.set_state(r, u, v)
            sim.step(1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            sim.step(3)
            torch.cuda.synchronize()
            t_alone[(model, n)] = (time.perf_counter() - t) / 3
            slot[(model, n)] = be.pool_bytes(pkg.make_params(cfg), 1)
            sim.close()
    e_bytes = float(np.mean(list(slot.values())))
    e_res = 105.0 * float(np.mean(list(t_alone.values())))
    lam = budget / (e_bytes * e_res)
    reqs = workloads.serving_stream(requests, rate=lam, seed=0)
    alone = sum(t_alone[(r.cfg.model, r.cfg.n)] * r.steps for r in reqs)
    srv = Server(budget, backend=be, check_energy=True)
    _, rep = srv.run(reqs, realtime=True, progress_every=20.0, log=sys.stderr)
    rep = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()}
    rep.update({"workload": f"{requests} requests, PFC (mixed, as the batched workload) / CDFT (FP64, h=17/128, "
                            "s=0.02) 50/50, n~U{64..1024}, steps~U{10..200}, Poisson arrivals, seed 0; "
                            f"budget {hbm_frac:g} of the device memory",
                "device_memory_bytes": hbm, "peak_reserved_frac_of_device": round(rep["peak_reserved_bytes"] / hbm, 4),
                "arrival_rate_per_s": round(lam, 3), "mean_slot_bytes": int(e_bytes),
                "mean_residence_alone_s": round(e_res, 4),
                "sequential_alone_s": round(alone, 3),
                "speedup_vs_sequential_alone": round(alone / rep["makespan_s"], 3)})
    return rep


def run_cdft(steps=50, n=1024):
    """The CDFT workload: 1024^2 FP64, energy and mass read after every step
    (inside the timed region: they are part of this workload)."""
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v = workloads.cdft_freezing_1024(0, n=n)
    sim = pkg.Simulation(cfg, device="cuda:0")
    sim.set_state(rho, u, v)
    E = [sim.energy()]
    M = [sim.mass()]
    cyc = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = sim.step(1)
        cyc += st.cycles_total
        E.append(sim.energy())
        M.append(sim.mass())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inc = sum(1 for a, b in zip(E[:-1], E[1:]) if b[0] > a[0] + 1e-10 * max(1.0, abs(a[0])))
    return {"workload": f"CDFT {n}^2 h=17/128 s=0.02 nu=2.362 FP64 tol 1e-10, {steps} steps",
            "steps_per_s": round(steps / dt, 3), "vcycles_per_step": round(cyc / steps, 3),
            "E_first": E[0][0], "E_last": E[-1][0], "F_id_last": E[-1][3], "F_ex_last": E[-1][4],
            "KE_last": E[-1][1], "energy_increases": inc,
            "mass_rel_drift": max(abs(m - M[0]) for m in M) / abs(M[0])}


def run_gradflow(steps=50, check_steps=10):
    """The gradient-flow variant: PFC free energy at 512^2 and CDFT at 1024^2,
    FP64 and mixed precision.  `steps` timed steps, then `check_steps` more
    with F and the mass read after each (not timed)."""
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    out = {}
    for model, n, kname in [("pfc_gf", 512, "GPFC"), ("cdft_gf", 1024, "GCDFT")]:
        res = {}
        for prec in ("fp64", "mixed"):
            cfg, rho, _, _ = workloads.gradflow(model, n, 0, precision=prec, coarsest_n=workloads.BENCH_COARSEST_N)
            sim = pkg.Simulation(cfg, device="cuda:0")
            sim.set_state(rho)
            sim.step(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            F = [sim.energy()[2]]
            M = [sim.mass()]
            for _ in range(check_steps):
                sim.step(1)
                F.append(sim.energy()[2])
                M.append(sim.mass())
            r = {"steps_per_s": round(steps / dt, 3), "ms_per_step": round(1e3 * dt / steps, 4),
                 "vcycles_per_step": round(st.cycles_total / steps, 3), "final_residual": st.residual_last,
                 "F_last": F[-1],
                 "energy_increases": sum(1 for a, b in zip(F[:-1], F[1:]) if b > a + 1e-12 * abs(a)),
                 "mass_rel_drift": max(abs(m - M[0]) for m in M) / abs(M[0])}
            if prec == "fp64":
                r["roofline"] = smoother_roofline(sim, n, sweep_bytes=SWEEP_BYTES_GF[model], model=kname)
                ref = sim.get_state()[0]
            else:
                r["max_rel_diff_vs_fp64"] = rel_diff([sim.get_state()[0]], [ref])
            sim.close()
            del sim
            torch.cuda.empty_cache()
            res[prec] = r
        h, s_ = (0.25, 0.01) if model == "pfc_gf" else (17.0 / 128.0, 0.02)
        res["workload"] = (f"{model} {n}^2 h={h:g} s={s_:g} FAS V(2,2) tol 1e-10, {steps} timed steps "
                           f"(+{check_steps} checked)")
        out[model] = res
    return out


def run_channel(steps=50, check_steps=10, n=256):
    """The sheared-nanocrystal channel (Sec. 6) at wall speeds 0, 0.1, 0.5:
    `steps` timed steps, then `check_steps` with the energy read after each
    (not timed).  With resting walls the energy must not increase."""
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    out = {"workload": f"PFC eps=0.4 channel {n}x{n + 1} nodes, h=pi/(2 sqrt3), s=0.02, 13-atom hexagonal "
                       f"nucleate, FAS V(2,2) tol 1e-10 FP64, {steps} timed steps (+{check_steps} checked)"}
    for uw in (0.0, 0.1, 0.5):
        cfg, rho, u, v = workloads.channel(n, u_wall=uw, coarsest_n=workloads.BENCH_COARSEST_N)
        sim = pkg.Simulation(cfg, device="cuda:0")
        sim.set_state(rho, u, v)
        sim.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        E = [sim.energy()]
        for _ in range(check_steps):
            sim.step(1)
            E.append(sim.energy())
        r = {"steps_per_s": round(steps / dt, 3), "ms_per_step": round(1e3 * dt / steps, 4),
             "vcycles_per_step": round(st.cycles_total / steps, 3), "final_residual": st.residual_last,
             "E_last": E[-1][0], "KE_last": E[-1][1],
             "energy_increases": sum(1 for a, b in zip(E[:-1], E[1:]) if b[0] > a[0] + 1e-12 * abs(a[0]))}
        if uw == 0.1:
            # algorithmic bytes: the interior nodes n x (n - 1)
            r["roofline"] = smoother_roofline(sim, n, model="WPFC")
            r["roofline"]["bytes_per_launch"] = 2 * SWEEP_BYTES_PFC * n * (n - 1)
            t = r["roofline"]["launch_us"] * 1e-6
            r["roofline"]["achieved"] = round(r["roofline"]["bytes_per_launch"] / t / 1e9, 1)
            r["roofline"]["frac"] = round(r["roofline"]["achieved"] / HBM_PEAK_GBS, 4)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        out[f"u_wall_{uw:g}"] = r
    # the channel smoother past the 256 MB cache (a grid that fills the device)
    sweep = {}
    for m in (1024, 2048):
        cfg, rho, u, v = workloads.channel(m, u_wall=0.1)
        sim = pkg.Simulation(cfg, device="cuda:0")
        sim.set_state(rho, u, v)
        rl = smoother_roofline(sim, m, model="WPFC")
        nbytes = 2 * SWEEP_BYTES_PFC * m * (m - 1)
        sweep[str(m)] = {"launch_us": rl["launch_us"], "achieved": round(nbytes / (rl["launch_us"] * 1e-6) / 1e9, 1),
                         "kernel": rl["kernel"]}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out["smoother_size_sweep_GBs"] = sweep
    return out


def run_size_sweep(sizes=(1024, 2048, 4096), shapes=(0, 1, 2, 7, 8, 9)):
    """The headline smoother (PFC, FP64, two fused sweeps per launch) on grids
    past the 256 MB Infinity Cache: at 2048^2 one launch moves 2.3 GB of
    algorithmic bytes, at 4096^2 9.1 GB.  In the tuner's tile shape (chosen
    for the V-cycle's pre- and post-smoothing launches together), and in each
    of the large shapes forced (HFZ_TILE, no tuning), with the best of them."""
    import torch
    import workloads
    import paper_1503_07416_amd as pkg

    def one(m):
        cfg, rho, u, v = workloads.pfc_uniform_noise(m, 0.25, 0.01, 0)
        sim = pkg.Simulation(cfg, device="cuda:0")
        sim.set_state(rho, u, v)
        rl = smoother_roofline(sim, m, launches=10)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        return rl

    out = {}
    for m in sizes:
        rl = one(m)
        out[str(m)] = {"launch_us": rl["launch_us"], "achieved": rl["achieved"], "frac": rl["frac"],
                       "kernel": rl["kernel"], "by_shape_GBs": {}}
        saved = {k: os.environ.get(k) for k in ("HFZ_TILE", "HFZ_TUNE")}
        try:
            os.environ["HFZ_TUNE"] = "0"
            for ts in shapes:
                os.environ["HFZ_TILE"] = str(ts)
                r = one(m)
                out[str(m)]["by_shape_GBs"][r["kernel"]] = r["achieved"]
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        best = max(out[str(m)]["by_shape_GBs"].items(), key=lambda kv: kv[1])
        out[str(m)]["best"] = {"kernel": best[0], "achieved": best[1], "frac": round(best[1] / HBM_PEAK_GBS, 4)}
    return out


def smoother3_roofline(sim, n, sweeps=10):
    """Average time of one damped red-black sweep of the 3D smoother (one
    launch of the z-marching tiled kernel from 32^3 up), HIP events on the
    library's stream."""
    import torch
    sim.begin_step()
    sim.smooth(0, 1)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    sim.smooth(0, sweeps)
    stop.record(sim.stream)
    stop.synchronize()
    t = start.elapsed_time(stop) * 1e-3 / sweeps
    nbytes = SWEEP_BYTES_3D * n ** 3
    ach = nbytes / t / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": committed_traffic_3d(n),
            "kernel": "k3_sweep_tile (both colours of one sweep)", "sweep_us": round(t * 1e6, 3),
            "bytes_per_sweep": nbytes}


def run_three_d(steps=20, check_steps=5, n=128):
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    cfg, rho, u, v, w = workloads.pfc3d(n)
    sim = pkg.Simulation3(cfg, device="cuda:0")
    sim.set_state(rho, u, v, w)
    sim.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    E, M = [sim.energy()[0]], [sim.mass()]
    for _ in range(check_steps):
        sim.step(1)
        E.append(sim.energy()[0])
        M.append(sim.mass())
    out = {"workload": f"PFC 3D {n}^3 h=0.5 s=0.01 eps=0.025 FAS V(2,2) tol 1e-10 FP64, {steps} timed steps "
                       f"(+{check_steps} checked)",
           "steps_per_s": round(steps / dt, 3), "ms_per_step": round(1e3 * dt / steps, 3),
           "vcycles_per_step": round(st.cycles_total / steps, 3), "final_residual": st.residual_last,
           "energy_increases": sum(1 for a, b in zip(E[:-1], E[1:]) if b > a + 1e-12 * abs(a)),
           "mass_rel_drift": max(abs(m - M[0]) for m in M) / abs(M[0]),
           "roofline": smoother3_roofline(sim, n)}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    cfg2, rho2, u2, v2, w2 = workloads.pfc3d(256)
    sim = pkg.Simulation3(cfg2, device="cuda:0")
    sim.set_state(rho2, u2, v2, w2)
    out["roofline_256"] = smoother3_roofline(sim, 256, sweeps=4)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def run_convergence(sizes, tf):
    """The paper's convergence study (Sec. 6.1): smooth initial density on
    [0,32)^2, u = 0, refinement path s = 0.025 h^2 to t_f; CDFT with nu = 1 and
    mean 6*0.6/pi, PFC with eps = 0.025 and offset 3/2.  Cauchy errors
    e_ij = rho^h_ij - rho^{h/2}_{2i,2j} in the h_c^2-weighted 2-norm and the
    rates log2(e_prev / e), beside the paper's printed tables.  Stop test: tol
    1e-10 (CDFT), 2e-9 (PFC)."""
    import math
    import numpy as np
    import torch
    import workloads
    import paper_1503_07416_amd as pkg
    with open(os.path.join(ROOT, "tests", "golden", "convergence_tables.json")) as f:
        printed = json.load(f)["tables"]
    out = {}
    for model in ("cdft", "pfc"):
        sol, runs = {}, []
        for n in sizes:
            h = 32.0 / n
            s = 0.025 * h * h
            nst = int(round(tf / s))
            rho, u, v = workloads.paper_convergence_ic(n, model)
            # PFC at 512^2 on this path (s/h^4 = 6.4): the residual's FP64 rounding floor is ~6e-10, so
            # the PFC runs stop at 2e-9 (three times that floor); the Cauchy errors are ~1e-5 and above
            cfg = (workloads.Config(model, n, h, s, tol=2e-9) if model == "pfc"
                   else workloads.Config(model, n, h, s, nu=1.0))
            sim = pkg.Simulation(cfg, device="cuda:0")
            sim.set_state(rho, u, v)
            E0 = sim.energy()[0]
            t0 = time.perf_counter()
            done, cycles = 0, 0
            while done < nst:
                k = min(5000, nst - done)
                st = sim.step(k)
                done += k
                cycles += st.cycles_total
                print(f"convergence {model} {n}^2: {done}/{nst} steps, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sol[n] = [x.cpu().numpy() for x in sim.get_state()]
            runs.append({"n": n, "steps": nst, "seconds": round(dt, 2), "steps_per_s": round(nst / dt, 1),
                         "vcycles_per_step": round(cycles / nst, 3), "E0": E0, "E_tf": sim.energy()[0]})
            sim.close()
        errs = []
        for a, b in zip(sizes[:-1], sizes[1:]):
            hc = 32.0 / a
            errs.append([math.sqrt(hc * hc * float(np.sum((sol[a][k] - sol[b][k][::2, ::2]) ** 2)))
                         for k in range(3)])
        rates = [[round(math.log2(p / q), 4) for p, q in zip(x, y)] for x, y in zip(errs[:-1], errs[1:])]
        key = "DFT" if model == "cdft" else "PFC"
        paper = {f: printed[f"{key}{i}_{f}"] for i, f in ((1, "rho"), (2, "u"), (3, "v"))}
        out[model] = {"grids": [[a, b] for a, b in zip(sizes[:-1], sizes[1:])],
                      "error_rho_u_v": [[float(f"{e:.4e}") for e in x] for x in errs], "rate_rho_u_v": rates,
                      "paper_error_rho": paper["rho"]["error"][:len(errs)],
                      "paper_rate_rho": paper["rho"]["rate"][:len(errs)], "runs": runs}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: the solver runs on a single device; --gpus must be 1"}))
        sys.exit(2)
    if a.counter_probe_3d:
        counter_probe_3d()
        return
    if a.counter_probe:
        counter_probe(a.n, a.probe_tile_shape)
        return
    if a.convergence:
        print(json.dumps({"convergence": run_convergence([int(x) for x in a.conv_sizes.split(",")], a.conv_tf)}))
        return
    if a.cdft_only:
        print(json.dumps({"cdft": run_cdft()}))
        return
    if a.batched_only:
        print(json.dumps({"batched": run_batched()}))
        return
    if a.precision_sweep_only:
        print(json.dumps({"precision_sweep": run_precision_sweep()}))
        return
    if a.serving_only:
        print(json.dumps({"serving": run_serving(a.serve_requests, a.serve_hbm_frac)}))
        return
    if a.gradflow_only:
        print(json.dumps({"gradflow": run_gradflow()}))
        return
    if a.channel_only:
        print(json.dumps({"channel": run_channel()}))
        return
    if a.size_sweep_only:
        print(json.dumps({"smoother_size_sweep": run_size_sweep()}))
        return
    if a.three_d_only:
        print(json.dumps({"three_d": run_three_d()}))
        return
    if a.mixed_only:
        import torch
        import workloads
        import paper_1503_07416_amd as pkg
        cfg, rho, u, v = workloads.pfc_freezing_512(0, n=a.n)
        sim = pkg.Simulation(cfg, device="cuda:0")
        sim.set_state(rho, u, v)
        sim.step(a.warmup + a.steps)
        print(json.dumps({"mixed": run_mixed(a, sim.get_state())}))
        return
    sample = None
    if not a.no_cpu:
        procs = a.cpu_procs if a.cpu_procs > 0 else max(1, min(16, os.cpu_count() or 1))
        sample = cpu_sample(a.n, a.cpu_cycles, procs)
    import torch
    import workloads
    import paper_1503_07416_amd as pkg

    cfg, rho, u, v = workloads.pfc_freezing_512(0, n=a.n)
    sim = pkg.Simulation(cfg, device="cuda:0")
    sim.set_state(rho, u, v)
    E0 = sim.energy()[0]
    if a.warmup:
        sim.step(a.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sim.step(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    E1 = sim.energy()[0]
    mass = sim.mass()
    state = sim.get_state()
    dt = t1 - t0
    cps = st.cycles_total / max(1, st.steps_done)
    roof = smoother_roofline(sim, a.n)
    out = {
        "metric": "time steps/sec + smoother HBM GB/s at 512^2; batched solves/sec, p50/p99 latency",
        "value": round(a.steps / dt, 3), "unit": "time steps/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(1e3 * dt / a.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"PFC {a.n}^2 h=0.25 s=0.01 eps=0.025 FAS V(2,2) to a {cfg.coarsest_n}^2 coarsest "
                               f"grid, tol 1e-10, FP64",
                   "n": a.n, "vcycles_per_step": round(cps, 3),
                   "us_per_vcycle": round(1e6 * dt / max(1, st.cycles_total), 2),
                   "final_residual": st.residual_last,
                   "energy_decreased": bool(E1 <= E0), "mass": mass},
        "roofline": roof,
    }
    if sample is not None:
        out["cpu_baseline"] = cpu_baseline(sample, a.n, cps, a.cpu_cycles)
    if not a.no_extras:
        sim.close()
        out["mixed"] = run_mixed(a, state)
        del state
        torch.cuda.empty_cache()
        out["precision_sweep"] = run_precision_sweep()
        torch.cuda.empty_cache()
        out["batched"] = run_batched()
        torch.cuda.empty_cache()
        out["cdft"] = run_cdft()
        torch.cuda.empty_cache()
        out["serving"] = run_serving(a.serve_requests, a.serve_hbm_frac)
        torch.cuda.empty_cache()
        out["gradflow"] = run_gradflow()
        torch.cuda.empty_cache()
        out["channel"] = run_channel()
        torch.cuda.empty_cache()
        out["three_d"] = run_three_d()
        torch.cuda.empty_cache()
        out["smoother_size_sweep"] = run_size_sweep()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
