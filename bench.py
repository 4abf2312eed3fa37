#!/usr/bin/env python3
"""Throughput of the fused D2Q9 + D2Q5 non-orthogonal MRT step on one MI355X.

Workload: the differentially heated square cavity, 2048 x 2048 nodes,
Ra = 1e6, Pr = 0.71, u_c = 0.1, from rest at T = 0.5, synthetic (the
paper's problem of Sec. 3.4 at a production size).  One benchmark "step" is
one time step of the whole lattice; every 1000 steps the run also takes the
wall Nusselt numbers (both walls) and the steady-state residual, as a real
solve does.  Inputs are resident in HBM before timing starts.

Prints one JSON line: MLUPS for FP64 storage (the plain method) with the
roofline of the step kernel measured with HIP events on the solver's
stream, the same figures for FP32 and FP16 deviation storage and for the
other temperature models in FP64 (the D2Q9 thermal model on the same
cavity; the flow alone on a lid-driven cavity of the same size, Re = 1000),
the step time of the comparison collision operators of Sec. 3.2 (BGK,
orthogonal MRT) relative to the paper's, fused and one step per launch,
and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--storage f64] [--variants f32,f16]
                    [--models d2q9t,isothermal] [--collisions bgk,ortho_mrt] [--slabs 2,4,8]

`slab_variants` times one GPU's share of the same lattice cut into 2, 4 or 8
y-slabs (2048 x 1024 / 512 / 256), with periodic rows standing in for the
halo rows a neighbour would send: the kernel at the shape each GPU of a
sharded run would sweep.  No figure at several GPUs is measured.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0              # MI355X HBM3E, published peak
LLC_BYTES = 256 * 2 ** 20          # MI355X last-level (Infinity) cache
BYTES = {"f64": 8, "f32": 4, "f16": 2}
NG = {"d2q5": 5, "d2q9t": 9, "isothermal": 0}   # temperature populations per node
REDUCE_EVERY = 1000


def values_per_node(model: str) -> int:
    """Populations read plus written per node and step: 9 + NG each way."""
    return 2 * (9 + NG[model])


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1510_08224_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.startswith("lbm_") and name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str, nodes: int, steps_per_launch: int):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter runs (key: storage for the D2Q5 model, model_storage for the
    others), if they were taken on the current kernel sources with the same
    number of time steps per launch."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get("kernels", {}).get(f"{key}/{steps_per_launch}")
    if (not ent or rec.get("source_hash") != kernel_source_hash() or ent.get("nodes") != nodes
            or ent.get("steps_per_launch", 1) != steps_per_launch):
        return None
    return ent.get("bytes_per_launch")


def time_storage(storage: str, pb, steps: int, warmup: int, launch=None, model: str = "d2q5",
                 single_steps: bool = False) -> dict:
    import torch
    from paper_1510_08224_amd import lbm

    S = lbm.Solver(pb.nx, pb.ny, storage, torch_memory=True, model=model)
    S.set_params(pb)
    if launch:
        S.set_launch(*launch)
    if single_steps:
        S.set_launch(policy=S.get_launch()[3] & ~(lbm.LBM_POLICY_FUSE2 | lbm.LBM_POLICY_FUSEK))
    shape = S.get_launch()
    spl = S.steps_per_launch
    thermal = NG[model] > 0
    st = torch.cuda.ExternalStream(S.stream)
    S.step(warmup)
    S.residual()
    S.synchronize()
    torch.cuda.synchronize()
    nodes = pb.nx * pb.ny
    segs = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(REDUCE_EVERY, steps - done)
        # whole launches of spl steps between e0 and e1 (the roofline's launch
        # time), the steps left over (shorter launches) between e1 and e2
        kk = k - k % spl
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(st)
        S.step(kk)
        e1.record(st)
        S.step(k - kk)
        e2.record(st)
        segs.append((e0, e1, e2, kk))
        done += k
        if done % REDUCE_EVERY == 0 or done == steps:
            if thermal:
                S.nusselt(0)
                S.nusselt(1)
            r, bad = S.residual(raise_unstable=False)
    S.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep_ms = sum(a.elapsed_time(c) for a, _, c, _ in segs)
    whole_ms = sum(a.elapsed_time(b) for a, b, _, kk in segs if kk)
    launches = sum(kk for *_, kk in segs) // spl
    nu = S.nusselt(1)[0] if thermal else None
    S.close()
    avg_step_s = sweep_ms / 1e3 / steps
    avg_launch_s = whole_ms / 1e3 / launches if launches else spl * avg_step_s
    traffic = measured_traffic(storage if model == "d2q5" else f"{model}_{storage}", nodes, spl)
    return {
        "storage": storage,
        "model": model,
        "launch": {"block_x": shape[0], "block_y": shape[1], "rows": shape[2], "policy": shape[3],
                   "steps_per_launch": spl},
        "mlups": nodes * steps / wall / 1e6,
        "ms_per_step": wall * 1e3 / steps,
        "sweep_us_per_launch": avg_launch_s * 1e6,
        "sweep_us_per_step": avg_step_s * 1e6,
        "sweep_mlups": nodes / avg_step_s / 1e6,
        "residual_last": r,
        "nonfinite": bad,
        "nu_right_mean": nu,
        "roofline": roofline(storage, model, nodes, spl, avg_launch_s, traffic),
    }


def roofline(storage: str, model: str, nodes: int, spl: int, launch_s: float, traffic) -> dict:
    """Roofline of one launch of the step kernel.  A launch advances `spl`
    steps (4 or 2 when fused) and must read and write the whole state once:
    its algorithmic HBM bytes are 2 (9 + NG) values per node whatever `spl`
    is, and `achieved` is those bytes over the launch time.  The
    single-step equivalent (spl times that: the bytes one-step launches
    would move for the same steps) is reported beside it as `effective`.
    `traffic` is the counter-measured HBM bytes of a launch, or None."""
    alg_bytes = values_per_node(model) * BYTES[storage] * nodes
    achieved = alg_bytes / launch_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
            "steps_per_launch": spl,
            # HBM bytes the counters measured per launch, over the same launch time
            "traffic_GBs": None if traffic is None else round(traffic / launch_s / 1e9, 1),
            # the bytes one-step launches would move for the same steps, over the same time
            "effective_GBs": round(spl * achieved, 1),
            "effective_frac": round(spl * achieved / HBM_PEAK_GBS, 4),
            # both buffers (one read and one written: alg_bytes) within the
            # 256 MB last-level cache: the bytes are then not all HBM traffic
            "state_in_last_level_cache": alg_bytes <= LLC_BYTES}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pb, steps: int, steps_all: int) -> dict:
    """The oracle timed on the host: its serial build on one core, and its
    OpenMP build (the same source, loops over nodes and rows split across
    threads, results bitwise equal) on all the cores OpenMP is given."""
    import oracle

    def run(library, n):
        L = oracle.Lattice(pb, library=library)
        t0 = time.perf_counter()
        L.step(n)
        return time.perf_counter() - t0

    dt1 = run(oracle.lib(), steps)
    omp = oracle.lib_openmp()
    threads = int(omp.orc_threads())
    dtn = run(omp, steps_all)
    mlups1 = pb.nx * pb.ny * steps / dt1 / 1e6
    mlupsn = pb.nx * pb.ny * steps_all / dtn / 1e6
    return {"value": round(mlupsn, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{pb.nx}x{pb.ny} cavity Ra={pb.ra:g}, FP64, from rest: {steps_all} steps on {threads} "
                      f"OpenMP threads in {dtn:.1f} s; {steps} steps on one thread in {dt1:.1f} s",
            "single_core": {"value": round(mlups1, 3), "unit": "MLUPS", "cores": 1},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f64", choices=list(BYTES))
    ap.add_argument("--variants", default="f32,f16", help="other storages to time ('none' for none)")
    ap.add_argument("--models", default="d2q9t,isothermal",
                    help="other temperature models to time in the main storage ('none' for none)")
    ap.add_argument("--collisions", default="bgk,ortho_mrt",
                    help="comparison collision operators to time in the main storage ('none' for none)")
    ap.add_argument("--slabs", default="2,4,8",
                    help="GPU counts whose y-slab share of the lattice to time on this GPU ('none' for none)")
    ap.add_argument("--cpu-steps", type=int, default=32, help="oracle steps on one core (~12 s)")
    ap.add_argument("--cpu-steps-all", type=int, default=160,
                    help="oracle steps on all cores (OpenMP build; ~5 s on 16 cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--n", type=int, default=2048, help="cavity side")
    ap.add_argument("--launch", default="", help="block_x,block_y,rows[,policy]")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one elementwise pass over 1 GiB (reference kernel for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(a single lattice would shard as y-slabs with a halo exchange, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1510_08224_amd import lbm
    from paper_1510_08224_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    pb = W.cavity(args.n, 1e6, 0.71, 0.1)
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    main_res = time_storage(args.storage, pb, args.steps, args.warmup, launch)
    variants = {}
    if args.variants != "none":
        for s in args.variants.split(","):
            if s and s != args.storage:
                variants[s] = time_storage(s, pb, args.steps, args.warmup, launch)
    models = {}
    if args.models != "none":
        for m in args.models.split(","):
            if m and m != "d2q5":
                mpb = pb if m != "isothermal" else W.lid_cavity(args.n, lbm.lbm_rate_for_reynolds(1000.0, args.n, 0.1), 0.1)
                models[m] = time_storage(args.storage, mpb, args.steps, args.warmup, launch, model=m)
                models[m]["workload"] = mpb.name
    colls, colls1 = {}, {}
    if args.collisions != "none":
        # every operator in the default launch (fused steps: bound by latency
        # and arithmetic, so operator costs can show) and one step per launch
        # (bound by bandwidth)
        colls["mrt"] = main_res
        colls1["mrt"] = time_storage(args.storage, pb, args.steps, args.warmup, launch, single_steps=True)
        codes = {"bgk": W.COLL_BGK, "ortho_mrt": W.COLL_ORTHO}
        for c in args.collisions.split(","):
            if c in codes:
                cpb = pb.replace(collision=codes[c])
                colls[c] = time_storage(args.storage, cpb, args.steps, args.warmup, launch)
                colls1[c] = time_storage(args.storage, cpb, args.steps, args.warmup, launch, single_steps=True)
    slabs = {}
    if args.slabs != "none":
        # one GPU's share of the lattice cut into k y-slabs: the same rates
        # (length of the whole cavity), walls left and right, and periodic
        # rows standing in for the halo rows a neighbour would send
        for k in (int(v) for v in args.slabs.split(",")):
            spb = pb.replace(ny=args.n // k, length=float(args.n), name=f"slab{args.n}x{args.n // k}",
                             bc_flow=(W.FLOW_WALL, W.FLOW_WALL, W.FLOW_PERIODIC, W.FLOW_PERIODIC),
                             bc_temp=(W.TEMP_DIRICHLET, W.TEMP_DIRICHLET, W.TEMP_PERIODIC, W.TEMP_PERIODIC))
            slabs[k] = time_storage(args.storage, spb, args.steps, args.warmup, launch)
            slabs[k]["shape"] = f"{args.n}x{args.n // k}"
    if args.calibrate_copy:
        # reference for counter runs: one dispatch reading and writing 1 GiB
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    cpu = None if args.no_cpu else cpu_baseline(pb, args.cpu_steps, args.cpu_steps_all)
    out = {
        "metric": "MLUPS & %HBM roofline, FP64 vs FP32/FP16 store; served p50/p99 latency",
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"cavity{args.n}_ra1e6_pr0.71_uc0.1", "nx": args.n, "ny": args.n,
                   "storage": args.storage, "model": "d2q5", "reduce_every": REDUCE_EVERY,
                   "launch": main_res["launch"], "device": torch.cuda.get_device_name(0)},
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "sweep_mlups": round(main_res["sweep_mlups"], 1),
        "sweep_us_per_launch": round(main_res["sweep_us_per_launch"], 3),
        "sweep_us_per_step": round(main_res["sweep_us_per_step"], 3),
        "nu_right_mean": main_res["nu_right_mean"],
        "storage_variants": {k: {"mlups": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 5),
                                 "sweep_mlups": round(v["sweep_mlups"], 1), "roofline": v["roofline"],
                                 "nu_right_mean": v["nu_right_mean"], "launch": v["launch"]}
                             for k, v in variants.items()},
        "model_variants": {k: {"workload": v["workload"], "storage": args.storage, "mlups": round(v["mlups"], 1),
                               "sweep_mlups": round(v["sweep_mlups"], 1), "roofline": v["roofline"],
                               "launch": v["launch"]}
                           for k, v in models.items()},
        "collision_variants": {k: {"storage": args.storage, "mlups": round(v["mlups"], 1),
                                   "steps_per_launch": v["launch"]["steps_per_launch"],
                                   "sweep_us_per_step": round(v["sweep_us_per_step"], 3),
                                   "ratio_to_mrt": round(v["sweep_us_per_step"] / colls["mrt"]["sweep_us_per_step"], 4),
                                   "single_step_us": round(colls1[k]["sweep_us_per_step"], 3),
                                   "single_step_ratio_to_mrt": round(colls1[k]["sweep_us_per_step"] /
                                                                     colls1["mrt"]["sweep_us_per_step"], 4)}
                               for k, v in colls.items()},
        "slab_variants": {f"{k}_gpus": {"shape": v["shape"], "storage": args.storage,
                                        "sweep_mlups": round(v["sweep_mlups"], 1),
                                        "sweep_us_per_step": round(v["sweep_us_per_step"], 3),
                                        "roofline": v["roofline"]}
                          for k, v in slabs.items()},
        "source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
