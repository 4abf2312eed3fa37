"""Launch-shape and memory-policy tuning of the step kernel.

    python -m paper_1510_08224_amd.tuning [--sizes 1024,2048,4096]
                                          [--models d2q5,d2q9t,isothermal]
                                          [--storages f64,f32,f16]

For every lattice size, temperature model and storage, times the step
kernel (HIP events on the solver's stream) for each block width
(64 x 4, 128 x 2, 256 x 1) and each memory policy (XCD bands on/off,
kept/non-temporal stores), and prints one JSON line with the library's
default choice, the best choice and every figure (algorithmic GB/s:
2 (9 + NG) stored values per node and step).  Results do not depend on the
shape or the policy; only the time does.

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
    # about 2 GB of algorithmic traffic per setting, at least 40 steps
    per_step = 2 * (9 + S.ng) * BYTES[{0: "f64", 1: "f32", 2: "f16"}[S.storage]] * S.nx * S.ny
    return max(40, int(2e9 / per_step))


def measure(S, steps: int | None = None) -> dict:
    """Algorithmic GB/s of every (block width, policy) on solver S.  The
    solver ends on its original shape and policy, with its state advanced."""
    keep = S.get_launch()
    steps = steps or _steps_for(S)
    per_step = 2 * (9 + S.ng) * BYTES[{0: "f64", 1: "f32", 2: "f16"}[S.storage]] * S.nx * S.ny
    out = {}
    for bx in SHAPES:
        for pol in POLICIES:
            S.set_launch(bx, 256 // bx, 1, pol)
            S.step(10)
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


def sweep(sizes, models, storages):
    import torch
    torch.cuda.set_device(0)
    for n in sizes:
        for model in models:
            pb = (W.cavity(n, 1e6) if model != "isothermal"
                  else W.lid_cavity(n, lbm.viscous_rate(1000.0, n, 0.1), 0.1))
            for st in storages:
                S = lbm.Solver(n, n, st, model=model)
                S.set_params(pb)
                d = S.get_launch()
                res = measure(S)
                best = max(res, key=res.get)
                rec = {"n": n, "model": model, "storage": st,
                       "footprint_MB": round(lbm.lbm_required_bytes(n, n, S.storage, S.model) / 1e6, 1),
                       "default": f"{d[0]}/{d[3]}", "default_GBs": round(res[(d[0], d[3])], 1),
                       "best": f"{best[0]}/{best[1]}", "best_GBs": round(res[best], 1),
                       "all": {f"{k[0]}/{k[1]}": round(v, 1) for k, v in res.items()}}
                print(json.dumps(rec), flush=True)
                S.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="1024,2048,4096")
    ap.add_argument("--models", default="d2q5,d2q9t,isothermal")
    ap.add_argument("--storages", default="f64,f32,f16")
    a = ap.parse_args()
    sweep([int(v) for v in a.sizes.split(",")], a.models.split(","), a.storages.split(","))


if __name__ == "__main__":
    main()
