"""Benchmark: time steps per second of the PFC 512^2 workload on one MI355X.

Workload (the paper's PFC freezing run scaled to 512^2): eps = 0.025, gamma = 2,
h = 0.25, s = 0.01, rho = (3/2 - 0.07 sqrt 3) + 0.05 U(-1,1) (seed 0), u = v = 0,
FAS V(2,2) with the damped red-black smoother to ||S - N(g)||_2 <= 1e-10, FP64.

Prints ONE JSON line with the step throughput, the roofline figure of the
dominant kernel (the finest-level smoother, timed with HIP events on the
library's stream) and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one damped red-black sweep per fine node: read g (5),
# f (5), rho^k, omega^k, write g (5), FP64
SWEEP_BYTES_PFC = 17 * 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-cycles", type=int, default=10,
                    help="V-cycles of the oracle sample")
    return ap.parse_args()


def smoother_roofline(sim, n, launches=25):
    """Average duration of one finest-level smoother launch (the LDS-tiled
    kernel doing two damped red-black sweeps, as in the V-cycle's
    pre-smoothing), measured with HIP events on the stream the library
    launches on."""
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
    bytes_launch = 2 * SWEEP_BYTES_PFC * n * n
    achieved = bytes_launch / t_launch / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_sweeps_tile<PFC,double,2 sweeps>", "launch_us": round(t_launch * 1e6, 3),
            "bytes_per_launch": bytes_launch}


def cpu_baseline(cfg, rho, u, v, cycles_per_step, vcycles):
    """The oracle (NumPy FP64, one thread) on a bounded sample: `vcycles`
    V-cycles of the first step of the same workload; steps/s extrapolated with
    the GPU's mean V-cycles per step."""
    from oracle.fas import Stepper
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
    per_cycle = (t2 - t1) / vcycles
    per_step = (t1 - t0) + per_cycle * cycles_per_step
    return {"value": round(1.0 / per_step, 6), "unit": "time steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{vcycles} V-cycles of step 1 of the {cfg.n}^2 workload "
                      f"({t2 - t0:.1f} s), scaled by {cycles_per_step:.2f} V-cycles/step"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads
    import paper_1503_07416_amd as pkg

    cfg, rho, u, v = workloads.pfc_uniform_noise(a.n, 0.25, 0.01, 0, precision=a.precision)
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
    dt = t1 - t0
    steps_per_s = a.steps / dt
    cps = st.cycles_total / max(1, st.steps_done)
    roof = smoother_roofline(sim, a.n)
    out = {
        "metric": "time steps/sec + smoother HBM GB/s at 512^2; batched solves/sec, p50/p99 latency",
        "value": round(steps_per_s, 3), "unit": "time steps/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(1e3 * dt / a.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if a.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"PFC {a.n}^2 h=0.25 s=0.01 eps=0.025 FAS V(2,2) tol 1e-10 {a.precision}",
                   "n": a.n, "precision": a.precision, "vcycles_per_step": round(cps, 3),
                   "final_residual": st.residual_last, "energy_decreased": bool(E1 <= E0),
                   "mass": mass},
        "roofline": roof,
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, rho, u, v, cps, a.cpu_cycles)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
