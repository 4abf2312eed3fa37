"""Batched solves and the tile autotuner.

    python -m paper_1510_08224_amd.batching [--count 256 --seed 3 --steps 2000]
    python -m paper_1510_08224_amd.batching --size-sweep

Builds the batch workload (independent differentially heated cavities,
side uniform over {64, 96, 128, 192, 256}, Ra log-uniform in [1e3, 1e6],
Pr in {0.71, 7.0}, u_c = 0.1, FP32 storage), tunes the tile width of every
size class, and reports aggregate MLUPS of the batched step (one launch
for all members per time step, or per pair of steps with fused pairs,
replayed from captured graphs) against one launch per instance per step
on the same GPU.

Autotuner, on the measured time of the whole batched step: for each size
class (lattice shape) the tile width block_x in {64, 128, 256} of the
one-step kernel (never wider than the lattice), by coordinate descent with
the other classes held fixed; then the launch the batched step runs with:
fused pairs or one step per launch, the XCD order of the tile tables, kept
or non-temporal stores, and the members' order in the tables (as added, or
largest first).  Choices are cached in a JSON file keyed by GPU
architecture, storage and size class (tile widths) or mix of size classes
(launch); cached choices are applied, not re-measured.  The report gives
the library's untuned default beside the tuned step.
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import lbm
from . import workloads as W

DEFAULT_CACHE = os.environ.get("LBM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "lbm_tiles.json"))


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_batch(B: lbm.Batch, steps: int) -> float:
    """Seconds per batched step, from HIP events on the batch's stream."""
    import torch
    st = torch.cuda.ExternalStream(B.stream)
    B.step(2)
    B.synchronize()
    e0, e1 = _events()
    e0.record(st)
    B.step(steps)
    e1.record(st)
    B.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def time_per_instance(solvers, steps: int) -> float:
    """Seconds per time step when every instance gets its own launch."""
    import torch
    for S in solvers:
        S.set_graph_steps(0)
    st = torch.cuda.ExternalStream(solvers[0].stream)
    for S in solvers:
        S.step(1)
    solvers[0].synchronize()
    e0, e1 = _events()
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        for S in solvers:
            S.step(1)
    e1.record(st)
    solvers[0].synchronize()
    wall = time.perf_counter() - t0
    return max(e0.elapsed_time(e1) / 1e3, wall) / steps


def build(problems, storage: str = "f32", graph_steps: int = 50):
    B = lbm.Batch(storage)
    B.set_graph_steps(graph_steps)
    solvers = []
    for pb in problems:
        S = B.new_solver(pb.nx, pb.ny)
        S.set_params(pb)
        B.add(S)
        solvers.append(S)
    return B, solvers


def size_classes(solvers) -> dict:
    cls: dict = {}
    for S in solvers:
        cls.setdefault(f"{S.nx}x{S.ny}", []).append(S)
    return cls


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", "gpu").split(":")[0]


def autotune(B: lbm.Batch, solvers, candidates=(64, 128, 256), steps: int = 60, cache_path: str | None = None,
             passes: int = 1) -> dict:
    """Choose block_x per size class; returns {class: block_x} and applies it."""
    cache_path = cache_path or DEFAULT_CACHE
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    key = f"{_arch()}/{B.storage_name}"
    known = cache.get(key, {})
    classes = size_classes(solvers)
    choice = {}

    def apply(c, bx):
        for S in classes[c]:
            S.set_launch(bx, 256 // bx, 1)

    for c, members in classes.items():
        bx = known.get(c)
        if bx is None:
            nx = members[0].nx
            bx = 64
            while bx < 256 and bx < nx:
                bx *= 2
        choice[c] = bx
        apply(c, bx)
    trials = []
    for _ in range(passes):
        for c, members in sorted(classes.items()):
            if c in known:
                continue
            nx = members[0].nx
            best_bx, best_t = choice[c], None
            for bx in candidates:
                if bx > 64 and bx // 2 >= nx:      # half the tile would be off the lattice
                    continue
                apply(c, bx)
                t = time_batch(B, steps)
                trials.append({"class": c, "block_x": bx, "us_per_step": round(t * 1e6, 2)})
                if best_t is None or t < best_t:
                    best_t, best_bx = t, bx
            choice[c] = best_bx
            apply(c, best_bx)
    if cache_path:
        cache.setdefault(key, {}).update(choice)
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return {"choice": choice, "trials": trials, "cache_key": key}


def mix_key(solvers) -> str:
    """The batch's size classes and their member counts, as a cache key."""
    return ",".join(f"{c}:{len(v)}" for c, v in sorted(size_classes(solvers).items()))


def autotune_launch(B: lbm.Batch, solvers, steps: int = 100, cache_path: str | None = None) -> dict:
    """Choose the launch the batched step runs with: K steps per launch,
    fused pairs or one step per launch, the XCD order of the tile tables, kept or non-temporal
    stores, and the members' order in the tables (as added, or largest
    lattice first), by the measured time of the whole batched step (best of
    two runs per setting).  The one-step kernel's tile widths per size class
    come from `autotune` first.  Choices are cached per GPU architecture,
    storage and mix of size classes; a cached mix is applied, not
    re-measured.  Returns the choice and the trials."""
    cache_path = cache_path or DEFAULT_CACHE
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    key = f"{_arch()}/{B.storage_name}/launch/{mix_key(solvers)}"
    known = cache.get(key)
    trials = []
    if known is None:
        best, best_t = None, None
        for policy in (lbm.LBM_POLICY_FUSEK | lbm.LBM_POLICY_FUSE2, lbm.LBM_POLICY_FUSE2, 0):
            B.set_policy(policy)
            if policy & lbm.LBM_POLICY_FUSEK and B.steps_per_launch <= 2:
                continue   # no multi-step kernel for this storage
            for order in (1, 0):
                for keep in (0, 1):
                    for largest in (0, 1):
                        B.set_policy(policy)
                        B.set_tuning(order, keep, largest)
                        t = min(time_batch(B, steps), time_batch(B, steps))
                        c = {"policy": policy, "xcd_order": order, "keep_stores": keep, "largest_first": largest}
                        trials.append(dict(c, us_per_step=round(t * 1e6, 2)))
                        if best_t is None or t < best_t:
                            best, best_t = c, t
        known = best
        if cache_path:
            cache[key] = known
            os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
            with open(cache_path, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
    B.set_policy(known["policy"])
    B.set_tuning(known["xcd_order"], known["keep_stores"], known["largest_first"])
    return {"choice": known, "trials": trials, "cache_key": key}


def report(count: int = 256, seed: int = 3, steps: int = 2000, base_steps: int = 200,
           storage: str = "f32", tune: bool = True, cache_path: str | None = None) -> dict:
    problems = W.batch_mix(count, seed)
    nodes = sum(p.nx * p.ny for p in problems)
    B, solvers = build(problems, storage)
    # the library's default launch, untuned
    B.set_policy(lbm.LBM_POLICY_DEFAULT)
    default_tuning = B.get_tuning()
    spl_default = B.steps_per_launch
    t_default = time_batch(B, steps)
    # tile widths of the one-step kernel per size class, timed alone
    B.set_policy(0)
    tuned = autotune(B, solvers, cache_path=cache_path) if tune else {"choice": {}, "trials": []}
    t_single = time_batch(B, steps)
    # the launch the batched step runs with
    launch = autotune_launch(B, solvers, cache_path=cache_path) if tune else None
    if not tune:
        B.set_policy(lbm.LBM_POLICY_DEFAULT)
    spl = B.steps_per_launch
    t_batch = time_batch(B, steps)
    t_inst = time_per_instance(solvers, base_steps)
    r, bad = B.residual()
    out = {
        "workload": f"batch{count}_cavities_seed{seed}",
        "storage": storage,
        "members": count,
        "nodes": nodes,
        "size_classes": {c: len(v) for c, v in size_classes(solvers).items()},
        "batched": {"us_per_step": round(t_batch * 1e6, 2), "mlups": round(nodes / t_batch / 1e6, 1),
                    "steps": steps, "graph_steps": 50, "steps_per_launch": spl,
                    "launch": None if launch is None else launch["choice"]},
        "batched_untuned_default": {"us_per_step": round(t_default * 1e6, 2),
                                    "mlups": round(nodes / t_default / 1e6, 1),
                                    "steps_per_launch": spl_default, "tuning": default_tuning},
        "tuned_over_default": round(t_default / t_batch, 3),
        "batched_one_step_per_launch": {"us_per_step": round(t_single * 1e6, 2),
                                        "mlups": round(nodes / t_single / 1e6, 1)},
        "one_launch_per_instance": {"us_per_step": round(t_inst * 1e6, 2), "mlups": round(nodes / t_inst / 1e6, 1),
                                    "steps": base_steps},
        "speedup": round(t_inst / t_batch, 2),
        # the state read and written once per launch (of steps_per_launch steps)
        "hbm_GBs_batched": round(28 * {"f64": 8, "f32": 4, "f16": 2}[storage] * nodes / (spl * t_batch) / 1e9, 1),
        # what one-step launches would move for the same steps
        "effective_GBs_batched": round(28 * {"f64": 8, "f32": 4, "f16": 2}[storage] * nodes / t_batch / 1e9, 1),
        "nonfinite_members": int((bad > 0).sum()),
        "autotune": tuned,
        "autotune_launch": launch,
    }
    B.close()
    for S in solvers:
        S.close()
    return out


def size_sweep(storages=("f32", "f64"), sides=(64, 96, 128, 192, 256, 384, 512, 1024), total: float = 6.7e6,
               steps: int = 400):
    """Fused pairs against one step per launch for batches of equal square
    cavities of each side (about `total` nodes per batch); one JSON line
    per (storage, side)."""
    import torch
    torch.cuda.set_device(0)
    for storage in storages:
        for side in sides:
            count = max(1, int(round(total / side ** 2)))
            B, sols = build([W.cavity(side, 1e5)] * count, storage)
            t = {}
            multi = lbm.LBM_POLICY_FUSEK | lbm.LBM_POLICY_FUSE2
            for pol in (0, lbm.LBM_POLICY_FUSE2, multi):
                B.set_policy(pol)
                t[pol] = time_batch(B, steps)
            B.set_policy(lbm.LBM_POLICY_DEFAULT)
            nodes = count * side * side
            print(json.dumps({"storage": storage, "side": side, "members": count,
                              "single_us": round(t[0] * 1e6, 2),
                              "fused_us": round(t[lbm.LBM_POLICY_FUSE2] * 1e6, 2),
                              "multi_us": round(t[multi] * 1e6, 2),
                              "single_over_fused": round(t[0] / t[lbm.LBM_POLICY_FUSE2], 3),
                              "fused_over_multi": round(t[lbm.LBM_POLICY_FUSE2] / t[multi], 3),
                              "single_mlups": round(nodes / t[0] / 1e6),
                              "fused_mlups": round(nodes / t[lbm.LBM_POLICY_FUSE2] / 1e6),
                              "default_steps_per_launch": B.steps_per_launch}), flush=True)
            B.close()
            for S in sols:
                S.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--base-steps", type=int, default=200)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cache", default=None)
    ap.add_argument("--size-sweep", action="store_true",
                    help="fused pairs vs one step per launch by member size, then exit")
    args = ap.parse_args()
    if args.size_sweep:
        size_sweep()
        return
    print(json.dumps(report(args.count, args.seed, args.steps, args.base_steps, args.storage,
                            not args.no_tune, args.cache)), flush=True)


if __name__ == "__main__":
    main()
