"""The collision-operator comparison of Sec. 3.2 on MI355X.

    python -m paper_1510_08224_amd.comparison [--n 2048] [--steps 1992]

1. Cost.  The paper reports its non-orthogonal MRT step about 4% cheaper
   than the classical orthogonal MRT (on a CPU).  Here the three operators
   (the paper's MRT, BGK and the orthogonal MRT) are timed on the 2048^2
   heated cavity in every storage (HIP events on the solver's stream), in
   the library's default launch (four steps per launch for FP64 and FP32,
   fused pairs for FP16; bound by latency and arithmetic) and one step per launch (bound by
   bandwidth), reported as MLUPS and algorithmic GB/s.

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


def time_operator(n: int, storage: str, coll: int, steps: int, single: bool = False) -> dict:
    import torch
    pb = W.cavity(n, 1e6).replace(collision=coll)
    S = lbm.Solver(n, n, storage)
    S.set_params(pb)
    if single:
        S.set_launch(policy=S.get_launch()[3] & ~(lbm.LBM_POLICY_FUSE2 | lbm.LBM_POLICY_FUSEK))
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
    launch, spl = S.get_launch(), S.steps_per_launch
    S.close()
    return {"us_per_step": round(t * 1e6, 2), "mlups": round(n * n / t / 1e6, 1),
            "GBs": round(28 * BYTES[storage] * n * n / t / 1e9, 1), "launch": list(launch),
            "steps_per_launch": spl}


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
    pb = W.with_nee_walls(W.lid_cavity(n, lbm.lbm_rate_for_reynolds(re, n - 1, u0), u0)).replace(collision=coll)
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


def markdown(cost: dict, cost1: dict, stab: dict, n: int, lid_steps: int) -> str:
    """Cost and stability tables as Markdown."""
    out = ["# Collision operators compared on MI355X (Sec. 3.2)", "", "Command:", "", "```",
           "python -m paper_1510_08224_amd.comparison", "```", "",
           f"## Cost of the step ({n} x {n} heated cavity, HIP events)", "",
           "Default launch (four steps per launch for FP64 and FP32, fused pairs for FP16) and one "
           "step per launch.  Algorithmic GB/s: 28 stored values per node and step.", "",
           "| storage | operator | steps / launch | us / step | MLUPS | algorithmic GB/s | one step per launch: "
           "us / step | MLUPS |",
           "|---|---|---:|---:|---:|---:|---:|---:|"]
    for st in cost:
        for op in cost[st]:
            c, c1 = cost[st][op], cost1[st][op]
            out.append(f"| {st} | {op} | {c['steps_per_launch']} | {c['us_per_step']} | {c['mlups']} | {c['GBs']} "
                       f"| {c1['us_per_step']} | {c1['mlups']} |")
    r = lambda c, op: ", ".join(f"{st} {c[st][op]['us_per_step'] / c[st]['mrt']['us_per_step']:.4f}" for st in c)
    out += ["", "Step time relative to the paper's non-orthogonal MRT, default launch: orthogonal MRT "
                f"{r(cost, 'ortho_mrt')}; BGK {r(cost, 'bgk')}.  One step per launch: orthogonal MRT "
                f"{r(cost1, 'ortho_mrt')}; BGK {r(cost1, 'bgk')}.", "",
            f"## Stability: lid-driven cavity, Re = 1200, 80 x 80, NEE walls, lid speed 0.1, FP64 "
            f"(at most {lid_steps} steps, stop at residual 1e-12)", "",
            "| operator | steps | finite | final residual | roughness (RMS Laplacian of u / RMS u) |",
            "|---|---:|---|---:|---:|"]
    for op, v in stab.items():
        rough = f"{v['roughness']:.4f}" if "roughness" in v else "-"
        out.append(f"| {op} | {v['steps']} | {v['finite']} | {v['residual']:.3g} | {rough} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=1992, help="a multiple of 12: whole pairs and quadruples")
    ap.add_argument("--storages", default="f64,f32,f16")
    ap.add_argument("--lid-steps", type=int, default=400000)
    ap.add_argument("--md", default=None, help="also write the tables as Markdown to this file")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    cost, cost1 = {}, {}
    for st in a.storages.split(","):
        cost[st], cost1[st] = {}, {}
        for name, coll in OPS.items():
            cost[st][name] = time_operator(a.n, st, coll, a.steps)
            cost1[st][name] = time_operator(a.n, st, coll, a.steps, single=True)
            print(json.dumps({"cost": name, "storage": st, "n": a.n, "default_launch": cost[st][name],
                              "single_steps": cost1[st][name]}), flush=True)
    stab = {}
    for name, coll in OPS.items():
        stab[name] = lid_cavity_run(coll, steps=a.lid_steps)
        print(json.dumps({"stability": name, **stab[name]}), flush=True)
    ratio = lambda c, op: {st: round(c[st][op]["us_per_step"] / c[st]["mrt"]["us_per_step"], 4) for st in c}
    summary = {"cost_ratio_ortho_over_mrt": ratio(cost, "ortho_mrt"),
               "cost_ratio_bgk_over_mrt": ratio(cost, "bgk"),
               "single_step_cost_ratio_ortho_over_mrt": ratio(cost1, "ortho_mrt"),
               "single_step_cost_ratio_bgk_over_mrt": ratio(cost1, "bgk"),
               "roughness": {k: v.get("roughness") for k, v in stab.items()}}
    print(json.dumps({"summary": summary}), flush=True)
    if a.md:
        with open(a.md, "w") as fh:
            fh.write(markdown(cost, cost1, stab, a.n, a.lid_steps))


if __name__ == "__main__":
    main()
