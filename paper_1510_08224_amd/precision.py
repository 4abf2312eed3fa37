"""Precision report: FP32 and FP16 deviation storage against FP64 storage.

    python -m paper_1510_08224_amd.precision [--nx 4096 --ny 1024 --steps 50000]

Runs the Rayleigh-Benard cell (periodic in x, hot bottom T = 1, cold top
T = 0, no-slip, Ra = 1e5, Pr = 0.71, u_c = 0.1) from the linear conduction
profile plus seeded uniform noise of +-1e-3 (PCG64, seed 1510) in each
storage mode on the GPU, and reports the errors of the FP32/FP16 runs
against the FP64 run (whose own agreement with the FP64 oracle is the
parity test): the relative global errors of Eq. 35 (velocity) and Eq. 38
(temperature), the largest pointwise |du| and |dT|, the relative error of
the bottom and top wall Nusselt numbers, and the relative drift of total
mass.  Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import lbm
from . import workloads as W


def run(pb, T0, storage: str, steps: int, chunk: int = 5000) -> dict:
    S = lbm.Solver(pb.nx, pb.ny, storage)
    S.set_params(pb)
    S.init_temperature(T0)
    mass0 = float(np.sum(S.moments()[0]))
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        S.step(k)
        done += k
        _, bad = S.residual(raise_unstable=False)
        if bad:
            break
    S.synchronize()
    wall = time.perf_counter() - t0
    rho, ux, uy, T = S.moments()
    out = {"storage": storage, "steps": done, "seconds": wall, "nonfinite": bad,
           "rho": rho, "ux": ux, "uy": uy, "T": T, "mass0": mass0, "mass1": float(np.sum(rho)),
           "nu_bottom": S.nusselt(W.BOTTOM)[0], "nu_top": S.nusselt(W.TOP)[0]}
    S.close()
    return out


def compare(ref: dict, r: dict, u_scale: float, t_scale: float) -> dict:
    du = np.sqrt((r["ux"] - ref["ux"]) ** 2 + (r["uy"] - ref["uy"]) ** 2)
    e_u = float(np.sum(du) / np.sum(np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2)))          # Eq. 35 form
    e_t = float(np.sqrt(np.sum((r["T"] - ref["T"]) ** 2)) / np.sqrt(np.sum(ref["T"] ** 2)))  # Eq. 38 form
    return {
        "E_u": e_u,
        "E_T": e_t,
        "max_du_over_uc": float(np.max(du)) / u_scale,
        "max_dT_over_dT": float(np.max(np.abs(r["T"] - ref["T"]))) / t_scale,
        "rel_err_nu_bottom": abs(r["nu_bottom"] - ref["nu_bottom"]) / abs(ref["nu_bottom"]),
        "rel_err_nu_top": abs(r["nu_top"] - ref["nu_top"]) / abs(ref["nu_top"]),
        "mass_drift": (r["mass1"] - r["mass0"]) / r["mass0"],
        "nonfinite": r["nonfinite"],
        "steps": r["steps"],
        "seconds": r["seconds"],
    }


def report(nx: int, ny: int, steps: int, ra: float = 1e5, storages=("f32", "f16")) -> dict:
    pb = W.rayleigh_benard(nx, ny, ra, 0.71, 0.1)
    T0 = W.rb_initial_temperature(nx, ny, 1.0, 0.0, amp=1e-3, seed=1510)
    ref = run(pb, T0, "f64", steps)
    res = {"workload": f"rb{nx}x{ny}_ra{ra:g}_pr0.71_uc0.1", "steps": steps,
           "f64": {"nu_bottom": ref["nu_bottom"], "nu_top": ref["nu_top"],
                   "mass_drift": (ref["mass1"] - ref["mass0"]) / ref["mass0"],
                   "max_u": float(np.max(np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2))),
                   "seconds": ref["seconds"]}}
    for s in storages:
        res[s] = compare(ref, run(pb, T0, s, steps), 0.1, 1.0)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--ra", type=float, default=1e5)
    ap.add_argument("--steps-list", default="",
                    help="comma-separated step counts: one report (JSON line) per count, each from the start")
    args = ap.parse_args()
    counts = [int(v) for v in args.steps_list.split(",") if v] or [args.steps]
    for n in counts:
        print(json.dumps(report(args.nx, args.ny, n, args.ra)), flush=True)


if __name__ == "__main__":
    main()
