"""The collision-operator comparison of Sec. 3.2 on MI355X.

    python -m paper_1510_08224_amd.comparison [--n 2048] [--steps 2000]

1. Cost.  The paper reports its non-orthogonal MRT step about 4% cheaper
   than the classical orthogonal MRT (on a CPU).  Here the three operators
   (the paper's MRT, BGK and the orthogonal MRT) are timed as the fused GPU
   step on the 2048^2 heated cavity in every storage (HIP events on the
   solver's stream), reported as MLUPS and algorithmic GB/s.

2. Stability.  The paper runs the lid-driven cavity at Re = 1200 on an
   80 x 80 lattice and finds BGK streamlines oscillating where the MRT ones
   are smooth.  The same case (walls by non-equilibrium extrapolation, lid
   speed 0.1, FP64) is run with each operator; reported are whether the run
   stays finite, the steady-state residual, and a grid-scale roughness of
   the velocity field: the RMS of the discrete Laplacian of u_x and u_y over
   the interior, relative to the RMS velocity (a smooth field gives a small
   value; node-to-node oscillations a large one).

Prints one JSON line per measurement and a final summary line.
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import lbm
from . import workloads as W

BYTES = {"f64": 8, "f32": 4, "f16": 2}
OPS = {"mrt": W.COLL_MRT, "bgk": W.COLL_BGK, "ortho_mrt": W.COLL_ORTHO}


def time_operator(n: int, storage: str, coll: int, steps: int) -> dict:
    import torch
    pb = W.cavity(n, 1e6).replace(collision=coll)
    S = lbm.Solver(n, n, storage)
    S.set_params(pb)
    S.step(20)
    S.synchronize()
    st = torch.cuda.ExternalStream(S.stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    S.step(steps)
    e1.record(st)
    S.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / steps
    launch = S.get_launch()
    S.close()
    return {"us_per_step": round(t * 1e6, 2), "mlups": round(n * n / t / 1e6, 1),
            "GBs": round(28 * BYTES[storage] * n * n / t / 1e9, 1), "launch": list(launch)}


def roughness(ux: np.ndarray, uy: np.ndarray) -> float:
    """RMS of the 5-point Laplacian of (u_x, u_y) over interior nodes over
    the RMS speed."""
    def lap(a):
        return a[1:-1, 2:] + a[1:-1, :-2] + a[2:, 1:-1] + a[:-2, 1:-1] - 4 * a[1:-1, 1:-1]
    num = np.sqrt(np.mean(lap(ux) ** 2 + lap(uy) ** 2))
    den = np.sqrt(np.mean(ux ** 2 + uy ** 2))
    return float(num / den)


def lid_cavity_run(coll: int, n: int = 80, re: float = 1200.0, u0: float = 0.1, steps: int = 400000,
                   check_every: int = 10000) -> dict:
    # walls through the edge nodes: the cavity side is n - 1 spacings
    pb = W.with_nee_walls(W.lid_cavity(n, lbm.viscous_rate(re, n - 1, u0), u0)).replace(collision=coll)
    S = lbm.Solver(n, n, "f64", model="isothermal")
    S.set_params(pb)
    S.residual()
    done, r, bad = 0, float("inf"), 0
    while done < steps:
        S.step(check_every)
        done += check_every
        r, bad = S.residual(raise_unstable=False)
        if bad or r < 1e-12:
            break
    out = {"steps": done, "finite": not bad, "residual": r}
    if not bad:
        _, ux, uy, _ = S.moments()
        out["roughness"] = roughness(ux, uy)
        out["u_max"] = float(np.max(np.hypot(ux, uy)))
        # u_x on the vertical centre line, sampled every 8 nodes
        out["ux_centerline"] = [round(float(v), 5) for v in ux[::8, n // 2]]
    S.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--storages", default="f64,f32,f16")
    ap.add_argument("--lid-steps", type=int, default=400000)
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    cost = {}
    for st in a.storages.split(","):
        cost[st] = {}
        for name, coll in OPS.items():
            cost[st][name] = time_operator(a.n, st, coll, a.steps)
            print(json.dumps({"cost": name, "storage": st, "n": a.n, **cost[st][name]}), flush=True)
    stab = {}
    for name, coll in OPS.items():
        stab[name] = lid_cavity_run(coll, steps=a.lid_steps)
        print(json.dumps({"stability": name, **stab[name]}), flush=True)
    summary = {"cost_ratio_ortho_over_mrt": {st: round(cost[st]["ortho_mrt"]["us_per_step"] /
                                                       cost[st]["mrt"]["us_per_step"], 4) for st in cost},
               "cost_ratio_bgk_over_mrt": {st: round(cost[st]["bgk"]["us_per_step"] /
                                                     cost[st]["mrt"]["us_per_step"], 4) for st in cost},
               "roughness": {k: v.get("roughness") for k, v in stab.items()}}
    print(json.dumps({"summary": summary}), flush=True)


if __name__ == "__main__":
    main()
