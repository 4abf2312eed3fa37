"""Launch-shape and memory-policy tuning of the step kernel.

    python -m paper_1510_08224_amd.tuning [--sizes 1024,2048,4096]
                                          [--models d2q5,d2q9t,isothermal]
                                          [--storages f64,f32,f16]

For every lattice size, temperature model and storage, times the step
kernel (HIP events on the solver's stream) for each block width
(64 x 4, 128 x 2, 256 x 1) and each memory policy of single steps (XCD
order round robin, bands or strips; kept or non-temporal stores), and for
fused pairs of steps (LBM_POLICY_FUSE2) and K steps per launch
(LBM_POLICY_FUSEK, where that kernel exists; fused tiles do not use the
block width) in each XCD order and store policy, and prints one JSON line
with the library's default choice, the best choice and every figure
(algorithmic GB/s: 2 (9 + NG) stored values per node and step).  Results
do not depend on the shape or the policy; only the time does.

:func:`autotune` does the same on a live solver and keeps the fastest
setting; the solver's state is saved first and restored afterwards.
"""
from __future__ import annotations

import argparse
import json

from . import lbm
from . import workloads as W

BYTES = {"f64": 8, "f32": 4, "f16": 2}
NG = {"d2q5": 5, "d2q9t": 9, "isothermal": 0}
SHAPES = (64, 128, 256)
POLICIES = tuple(order | keep for order in (0, lbm.LBM_POLICY_XCD_BANDS, lbm.LBM_POLICY_XCD_STRIPS)
                 for keep in (0, lbm.LBM_POLICY_KEEP_STORES))
FUSED = tuple(lbm.LBM_POLICY_FUSE2 | p for p in POLICIES)
FUSEDK = tuple(lbm.LBM_POLICY_FUSEK | lbm.LBM_POLICY_FUSE2 | p for p in POLICIES)
FUSE_ANY = lbm.LBM_POLICY_FUSE2 | lbm.LBM_POLICY_FUSEK


def _time_steps(S, steps: int) -> float:
    """Seconds per step of `steps` steps on the solver's stream."""
    import torch
    st = torch.cuda.ExternalStream(S.stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    S.step(steps)
    e1.record(st)
    S.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def _steps_for(S) -> int:
    # about 2 GB of algorithmic traffic per setting, at least 48 steps, a
    # multiple of 12 (whole pairs and whole launches of four)
    per_step = 2 * (9 + S.ng) * BYTES[{0: "f64", 1: "f32", 2: "f16"}[S.storage]] * S.nx * S.ny
    return max(48, int(2e9 / per_step)) // 12 * 12


def measure(S, steps: int | None = None) -> dict:
    """Algorithmic GB/s of every (block width, policy) on solver S, fused
    policies under block width 64.  The solver ends on its original shape
    and policy, with its state advanced."""
    keep = S.get_launch()
    steps = steps or _steps_for(S)
    per_step = 2 * (9 + S.ng) * BYTES[{0: "f64", 1: "f32", 2: "f16"}[S.storage]] * S.nx * S.ny
    out = {}
    trials = [(bx, pol) for bx in SHAPES for pol in POLICIES] + [(64, pol) for pol in FUSED]
    S.set_launch(64, 4, 1, lbm.LBM_POLICY_FUSEK)
    if S.steps_per_launch > 2:
        trials += [(64, pol) for pol in FUSEDK]
    for bx, pol in trials:
        S.set_launch(bx, 256 // bx, 1, pol)
        S.step(12)
        out[(bx, pol)] = per_step / _time_steps(S, steps) / 1e9
    S.set_launch(*keep)
    return out


def autotune(S, steps: int | None = None) -> tuple:
    """Pick the fastest (block width, policy) for solver S and keep it.
    The state is saved before and restored after the trial steps."""
    blob = S.save_state()
    res = measure(S, steps)
    S.load_state(blob)
    bx, pol = max(res, key=res.get)
    S.set_launch(bx, 256 // bx, 1, pol)
    return bx, pol, res[(bx, pol)]


def _key(bx: int, pol: int) -> tuple:
    # fused policies are measured under block width 64 (their tiles do not use it)
    return (64, pol) if pol & FUSE_ANY else (bx, pol)


def sweep(sizes, models, storages, md: str | None = None):
    import torch
    torch.cuda.set_device(0)
    rows = []
    for n in sizes:
        for model in models:
            pb = (W.cavity(n, 1e6) if model != "isothermal"
                  else W.lid_cavity(n, lbm.lbm_rate_for_reynolds(1000.0, n, 0.1), 0.1))
            for st in storages:
                S = lbm.Solver(n, n, st, model=model)
                S.set_params(pb)
                d = S.get_launch()
                res = measure(S)
                best = max(res, key=res.get)
                single = max((k for k in res if not k[1] & FUSE_ANY), key=res.get)
                dk = _key(d[0], d[3])
                rec = {"n": n, "model": model, "storage": st,
                       "footprint_MB": round(lbm.lbm_required_bytes(n, n, S.storage, S.model) / 1e6, 1),
                       "default": f"{dk[0]}/{dk[1]}", "default_GBs": round(res[dk], 1),
                       "best": f"{best[0]}/{best[1]}", "best_GBs": round(res[best], 1),
                       "best_single": f"{single[0]}/{single[1]}", "best_single_GBs": round(res[single], 1),
                       "all": {f"{k[0]}/{k[1]}": round(v, 1) for k, v in res.items()}}
                print(json.dumps(rec), flush=True)
                rows.append(rec)
                S.close()
    if md:
        with open(md, "w") as fh:
            fh.write(markdown(rows, sizes, models, storages))


def markdown(rows, sizes, models, storages) -> str:
    cmd = (f"python -m paper_1510_08224_amd.tuning --sizes {','.join(map(str, sizes))} "
           f"--models {','.join(models)} --storages {','.join(storages)}")
    out = ["# Launch shape and memory policy of the step kernel on MI355X", "", "Command:", "", "```", cmd, "```",
           "",
           "Algorithmic GB/s (2 (9 + NG) stored values per node and step) for block width bx (64 x 4, 128 x 2, "
           "256 x 1 threads) and policy mask p (1 XCD bands, 2 kept stores, 4 XCD strips, 8 fused pairs of "
           "steps, 16 K = 4 steps per launch (with 8: remainders as pairs), 0 round-robin XCD order with "
           "non-temporal stores, one step per launch).  Fused policies are listed under bx 64: their tiles "
           "do not use the block width.", "",
           "| n | model | storage | footprint MB | default bx/p | GB/s | best bx/p | GB/s | best single step bx/p | GB/s |",
           "|---:|---|---|---:|---|---:|---|---:|---|---:|"]
    for r in rows:
        out.append(f"| {r['n']} | {r['model']} | {r['storage']} | {r['footprint_MB']} | {r['default']} | "
                   f"{r['default_GBs']} | {r['best']} | {r['best_GBs']} | {r['best_single']} | "
                   f"{r['best_single_GBs']} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="1024,2048,4096")
    ap.add_argument("--models", default="d2q5,d2q9t,isothermal")
    ap.add_argument("--storages", default="f64,f32,f16")
    ap.add_argument("--md", default=None, help="also write a Markdown table to this file")
    a = ap.parse_args()
    sweep([int(v) for v in a.sizes.split(",")], a.models.split(","), a.storages.split(","), a.md)


if __name__ == "__main__":
    main()
