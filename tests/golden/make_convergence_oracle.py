"""Writes convergence_oracle_16_64.json: the oracle's Cauchy errors for the
paper's convergence protocol (Sec. 6.1: smooth initial density on [0,32)^2,
u = 0, s = 0.025 h^2, t_f = 10) on 16^2, 32^2 and 64^2, for both models, under
the readings this repository takes (CDFT mean 6 * 0.6 / pi with nu = 1, PFC
offset 3/2 with eps = 0.025; gamma = 2; FAS V(2,2), 4 coarsest sweeps, tol
1e-10), and a summary of each final state.  Calls only the oracle.

    python tests/golden/make_convergence_oracle.py      (about 10 minutes on 4 cores)
"""
import json
import math
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SIZES = (16, 32, 64)


def run(args):
    model, n = args
    import numpy as np
    import workloads
    from oracle.fas import Stepper
    h = 32.0 / n
    s = 0.025 * h * h
    nst = int(round(10.0 / s))
    rho, u, v = workloads.paper_convergence_ic(n, model)
    if model == "pfc":
        st = Stepper("pfc", n, h, s, alpha=1.0 - workloads.PFC_EPS, tol=1e-10, coarse_sweeps=4, max_cycles=400)
    else:
        st = Stepper("cdft", n, h, s, nu=1.0, tol=1e-10, coarse_sweeps=4, max_cycles=400)
    st.set_state(rho, u, v)
    for _ in range(nst):
        st.step()
    return model, n, nst, [st.rho.tolist(), st.u.tolist(), st.v.tolist()]


def main():
    import numpy as np
    jobs = [(m, n) for m in ("cdft", "pfc") for n in SIZES]
    with Pool(min(len(jobs), 6)) as pool:
        res = {(m, n): (nst, [np.array(x) for x in f]) for m, n, nst, f in pool.map(run, jobs)}
    out = {"protocol": "Sec. 6.1, [0,32)^2, s = 0.025 h^2, t_f = 10, u0 = 0; CDFT rho_o = 6*0.6/pi, nu = 1; "
                       "PFC offset 3/2, eps = 0.025; gamma = 2; FAS V(2,2), 4 coarsest sweeps, tol 1e-10",
           "norm": "e_ij = f^{h_c}_ij - f^{h_f}_{2i,2j}, ||e|| = (h_c^2 sum e^2)^(1/2)", "models": {}}
    for m in ("cdft", "pfc"):
        errs = []
        for a, b in zip(SIZES[:-1], SIZES[1:]):
            hc = 32.0 / a
            fa, fb = res[(m, a)][1], res[(m, b)][1]
            errs.append([math.sqrt(hc * hc * float(np.sum((fa[k] - fb[k][::2, ::2]) ** 2))) for k in range(3)])
        summ = {str(n): {"steps": res[(m, n)][0],
                         "rho_mean": float(res[(m, n)][1][0].mean()), "rho_min": float(res[(m, n)][1][0].min()),
                         "rho_max": float(res[(m, n)][1][0].max()),
                         "u_absmax": float(np.abs(res[(m, n)][1][1]).max())} for n in SIZES}
        out["models"][m] = {"grids": [[a, b] for a, b in zip(SIZES[:-1], SIZES[1:])],
                            "error_rho_u_v": errs, "final_states": summ}
    with open(os.path.join(HERE, "convergence_oracle_16_64.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["models"], indent=1))


if __name__ == "__main__":
    main()
