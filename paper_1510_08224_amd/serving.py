"""Continuous-batching solve server.

    python -m paper_1510_08224_amd.serving [--count 32 --rates 0.5,1,2,4 --cap 100000]

Requests (cavity and Rayleigh-Benard solves of different sizes, Poisson
arrivals) are admitted as slots in one :class:`lbm.Batch` while an HBM
budget and a slot limit allow; their lattices stay resident on the GPU and
advance together, one launch per time step for all of them.  Every
``check_every`` steps each member's steady-state residual (max |du|, |dT|
over the interval) is taken; a member retires when it falls below ``tol``,
when it hits the step cap, or when its lattice holds non-finite values.
New requests join at those boundaries, so work that arrives while others
run overlaps with them on the device.

The baseline is the plain method: FIFO, one solve at a time, one kernel
launch per time step, the same stopping rule.

Each request's stopping step depends only on its own residual history, and
a batch member's state is bitwise the state it has alone, so every result
of the server equals the result of the same request solved alone.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm
from . import workloads as W

SNAPSHOT_BYTES = 3 * 8            # residual snapshot per node
STORAGE = {"f64": lbm.LBM_F64, "f32": lbm.LBM_F32, "f16": lbm.LBM_F16}


def request_bytes(pb, storage: str) -> int:
    """HBM a resident solve needs in the given storage ("f64", "f32",
    "f16"): population buffers and residual state."""
    return lbm.lbm_required_bytes(pb.nx, pb.ny, STORAGE[storage]) + SNAPSHOT_BYTES * pb.nx * pb.ny + 64 * 1024


def initial_temperature(req: W.Request):
    """Rayleigh-Benard solves start from the conduction profile with seeded
    noise (seed 1510 + request id); cavities from rest at T0."""
    if req.kind == "rb":
        pb = req.problem
        return W.rb_initial_temperature(pb.nx, pb.ny, pb.t_hot, pb.t_cold, amp=1e-3, seed=1510 + req.rid)
    return None


@dataclass
class Result:
    rid: int
    kind: str
    nx: int
    ny: int
    arrival: float
    start: float = 0.0
    finish: float = 0.0
    steps: int = 0
    status: str = ""
    residual: float = float("nan")
    nu: float = float("nan")
    fields: tuple | None = None

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def _nu_of(S, req) -> float:
    side = lbm.LBM_RIGHT if req.kind == "cavity" else lbm.LBM_BOTTOM
    return S.nusselt(side)[0]


def solve_alone(req: W.Request, tol: float, check_every: int, cap: int, storage: str = "f32",
                keep_fields: bool = False, graph: bool = False) -> Result:
    """The plain method: one solve, one launch per step (unless graph)."""
    pb = req.problem
    S = lbm.Solver(pb.nx, pb.ny, storage)
    S.set_params(pb)
    if not graph:
        S.set_graph_steps(0)
    T = initial_temperature(req)
    if T is not None:
        S.init_temperature(T)
    S.residual()
    res = Result(req.rid, req.kind, pb.nx, pb.ny, req.arrival)
    while True:
        S.step(check_every)
        r, bad = S.residual(raise_unstable=False)
        res.steps += check_every
        res.residual = r
        if bad:
            res.status = "nonfinite"
            break
        if r < tol:
            res.status = "converged"
            break
        if res.steps >= cap:
            res.status = "capped"
            break
    if res.status != "nonfinite":
        res.nu = _nu_of(S, req)
    if keep_fields:
        res.fields = S.moments()
    S.close()
    return res


def serve_serial(requests, tol, check_every, cap, storage="f32") -> list[Result]:
    """FIFO, one solve at a time, live in wall-clock time."""
    out = []
    t0 = time.perf_counter()
    for req in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if now < req.arrival:
            time.sleep(req.arrival - now)
        start = time.perf_counter() - t0
        res = solve_alone(req, tol, check_every, cap, storage)
        res.start = start
        res.finish = time.perf_counter() - t0
        out.append(res)
    return out


def fifo_latencies(requests, service: dict) -> list[float]:
    """Latencies of a single-server FIFO queue with the measured service
    time of each request (for arrival rates not run live)."""
    t = 0.0
    lat = []
    for req in sorted(requests, key=lambda r: r.arrival):
        t = max(t, req.arrival) + service[req.rid]
        lat.append(t - req.arrival)
    return lat


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 64, storage: str = "f32", tol: float = 1e-7,
                 check_every: int = 1000, cap: int = 30000, graph_steps: int = 50, keep_fields: bool = False):
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.storage = storage
        self.tol, self.check_every, self.cap = tol, check_every, cap
        self.keep_fields = keep_fields
        self.B = lbm.Batch(storage)
        self.B.set_graph_steps(graph_steps)
        self.used = 0
        self.active: dict[int, tuple] = {}     # slot -> (solver, request, result, bytes)
        self.refused = 0

    def fits(self, req) -> bool:
        return len(self.active) < self.max_slots and self.used + request_bytes(req.problem, self.storage) <= self.budget

    def admit(self, req, now: float) -> int:
        pb = req.problem
        S = self.B.new_solver(pb.nx, pb.ny)
        S.set_params(pb)
        T = initial_temperature(req)
        if T is not None:
            S.init_temperature(T)
        S.residual()
        slot = self.B.add(S)
        nbytes = request_bytes(pb, self.storage)
        self.used += nbytes
        res = Result(req.rid, req.kind, pb.nx, pb.ny, req.arrival, start=now)
        self.active[slot] = (S, req, res, nbytes)
        return slot

    def retire(self, slot: int, now: float, status: str) -> Result:
        S, req, res, nbytes = self.active.pop(slot)
        res.finish = now
        res.status = status
        if status != "nonfinite":
            res.nu = _nu_of(S, req)
        if self.keep_fields:
            res.fields = S.moments()
        self.B.remove(slot)
        S.close()
        self.used -= nbytes
        return res

    def run(self, requests) -> dict:
        pending = sorted(requests, key=lambda r: r.arrival)
        never = [r for r in pending if request_bytes(r.problem, self.storage) > self.budget]
        pending = [r for r in pending if request_bytes(r.problem, self.storage) <= self.budget]
        self.refused = len(never)
        done: list[Result] = []
        t0 = time.perf_counter()
        busy = 0.0
        lup = 0
        while pending or self.active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now and self.fits(pending[0]):
                self.admit(pending.pop(0), now)
            if not self.active:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now, 0.05)))
                continue
            tb = time.perf_counter()
            self.B.step(self.check_every)
            r, bad = self.B.residual()          # synchronizes
            busy += time.perf_counter() - tb
            now = time.perf_counter() - t0
            for slot in list(self.active):
                S, req, res, _ = self.active[slot]
                res.steps += self.check_every
                res.residual = float(r[slot])
                lup += S.nx * S.ny * self.check_every
                if bad[slot] > 0:
                    done.append(self.retire(slot, now, "nonfinite"))
                elif r[slot] < self.tol:
                    done.append(self.retire(slot, now, "converged"))
                elif res.steps >= self.cap:
                    done.append(self.retire(slot, now, "capped"))
        wall = time.perf_counter() - t0
        return {"results": done, "wall": wall, "busy": busy, "lup": lup, "refused": self.refused}

    def close(self):
        for slot in list(self.active):
            self.retire(slot, 0.0, "cancelled")
        self.B.close()


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def summarize(results, wall, lup) -> dict:
    lat = [r.latency for r in results]
    return {"requests": len(results), "p50_latency_s": round(_pct(lat, 50), 4),
            "p99_latency_s": round(_pct(lat, 99), 4), "mean_latency_s": round(float(np.mean(lat)), 4),
            "solves_per_s": round(len(results) / wall, 4), "mlups": round(lup / wall / 1e6, 1),
            "wall_s": round(wall, 3),
            "status": {s: sum(r.status == s for r in results) for s in sorted({r.status for r in results})}}


def benchmark(count: int = 32, rates=(0.5, 1.0, 2.0, 4.0), seed: int = 4, cap: int = 100000,
              tol: float = 1e-7, check_every: int = 1000, budget_gib: float = 2.0, max_slots: int = 64,
              n_range=(64, 1024), live_serial_rate: float | None = 1.0, ra_range=(1e3, 1e6),
              storage: str = "f32") -> dict:
    base = W.request_stream(count, 1.0, seed=seed, n_range=n_range, ra_range=ra_range)
    # service time of each request alone (the plain method), measured once
    service, lup_serial, serial_results = {}, 0, {}
    for req in base:
        t0 = time.perf_counter()
        res = solve_alone(req, tol, check_every, cap, storage)
        service[req.rid] = time.perf_counter() - t0
        lup_serial += req.problem.nx * req.problem.ny * res.steps
        serial_results[req.rid] = res
    mu = count / sum(service.values())     # serial solves per second
    out = {"workload": f"serve{count}_seed{seed}_cap{cap}", "count": count, "sides": list(n_range),
           "ra_range": list(ra_range), "storage": storage, "cap_steps": cap, "tol": tol,
           "check_every": check_every, "hbm_budget_bytes": int(budget_gib * 2 ** 30), "max_slots": max_slots,
           "serial_service_rate_per_s": round(mu, 4),
           "serial_mlups": round(lup_serial / sum(service.values()) / 1e6, 1),
           "serial_status": {s: sum(r.status == s for r in serial_results.values())
                             for s in sorted({r.status for r in serial_results.values()})},
           "rates": []}
    for f in rates:
        lam = f * mu
        reqs = W.request_stream(count, lam, seed=seed, n_range=n_range, ra_range=ra_range)
        srv = Server(int(budget_gib * 2 ** 30), max_slots, storage=storage, tol=tol, check_every=check_every,
                     cap=cap)
        run = srv.run(reqs)
        srv.close()
        batched = summarize(run["results"], run["wall"], run["lup"])
        batched["refused"] = run["refused"]
        lat = fifo_latencies(reqs, service)
        serial = {"p50_latency_s": round(_pct(lat, 50), 4), "p99_latency_s": round(_pct(lat, 99), 4),
                  "mean_latency_s": round(float(np.mean(lat)), 4), "mlups": out["serial_mlups"],
                  "method": "FIFO queue over the measured one-launch-per-step service times"}
        # equality of stopping: the server's steps per request match the plain method's
        same = sum(r.steps == serial_results[r.rid].steps and r.status == serial_results[r.rid].status
                   for r in run["results"])
        entry = {"rate_factor": f, "arrival_rate_per_s": round(lam, 4), "batched": batched,
                 "serial": serial, "same_steps_as_alone": f"{same}/{len(run['results'])}"}
        if live_serial_rate is not None and abs(f - live_serial_rate) < 1e-12:
            # the plain method run live at this rate, to check the FIFO model
            live = serve_serial(reqs, tol, check_every, cap, storage)
            wall = max(r.finish for r in live)
            lup = sum(r.nx * r.ny * r.steps for r in live)
            entry["serial_live"] = summarize(live, wall, lup)
        out["rates"].append(entry)
        print(json.dumps(out["rates"][-1]), flush=True)
    return out


def markdown(res: dict, command: str) -> str:
    """The benchmark's result as a Markdown summary (the table of every
    rate factor and the live check of the FIFO model)."""
    out = ["# Continuous-batching solve server vs the plain method (MI355X)", "", "Command:", "", "```", command,
           "```", "",
           f"Workload `{res['workload']}`: {res['count']} requests (cavity and Rayleigh-Benard solves, 50/50, "
           f"sides {res['sides'][0]}-{res['sides'][1]}, Ra log-uniform in [{res['ra_range'][0]:g}, "
           f"{res['ra_range'][1]:g}], {res['storage'].upper()} storage), Poisson arrivals at a rate factor times the "
           f"measured serial service rate "
           f"({res['serial_service_rate_per_s']} solves/s). A request stops when its residual over "
           f"{res['check_every']} steps falls below {res['tol']:g} or at {res['cap_steps']} steps (serial status "
           f"{res['serial_status']}). HBM budget {res['hbm_budget_bytes'] / 2 ** 30:g} GiB, at most "
           f"{res['max_slots']} slots. The plain method: FIFO, one solve at a time, each with the library's "
           f"default launch; its latencies follow a FIFO queue over the measured per-request service times.",
           "",
           "| rate factor | arrivals/s | batched p50 s | batched p99 s | batched solves/s | batched MLUPS "
           "| plain p50 s | plain p99 s | plain MLUPS | same steps as alone | batched status |",
           "|---:|---:|---:|---:|---:|---:|---:|---:|---:|---|---|"]
    for e in res["rates"]:
        b, s = e["batched"], e["serial"]
        out.append(f"| {e['rate_factor']} | {e['arrival_rate_per_s']} | {b['p50_latency_s']} | {b['p99_latency_s']} "
                   f"| {b['solves_per_s']} | {b['mlups']} | {s['p50_latency_s']} | {s['p99_latency_s']} "
                   f"| {s['mlups']} | {e['same_steps_as_alone']} | {b['status']} |")
    for e in res["rates"]:
        if "serial_live" in e:
            lv, s = e["serial_live"], e["serial"]
            out += ["", f"Plain method run live at rate factor {e['rate_factor']}: p50 {lv['p50_latency_s']} s, "
                        f"p99 {lv['p99_latency_s']} s, {lv['solves_per_s']} solves/s, {lv['mlups']} MLUPS "
                        f"(FIFO model: p50 {s['p50_latency_s']} s, p99 {s['p99_latency_s']} s)."]
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=32)
    ap.add_argument("--rates", default="0.5,1,2,4")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--cap", type=int, default=100000)
    ap.add_argument("--budget-gib", type=float, default=2.0)
    ap.add_argument("--max-slots", type=int, default=64)
    ap.add_argument("--nmin", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=1024)
    ap.add_argument("--ra-min", type=float, default=1e3)
    ap.add_argument("--ra-max", type=float, default=1e6)
    ap.add_argument("--storage", default="f32", choices=list(STORAGE))
    ap.add_argument("--md", default=None, help="also write a Markdown summary to this file")
    args = ap.parse_args()
    rates = tuple(float(v) for v in args.rates.split(","))
    res = benchmark(args.count, rates, args.seed, args.cap, budget_gib=args.budget_gib,
                    max_slots=args.max_slots, n_range=(args.nmin, args.nmax), ra_range=(args.ra_min, args.ra_max),
                    storage=args.storage)
    print(json.dumps(res), flush=True)
    if args.md:
        with open(args.md, "w") as fh:
            fh.write(markdown(res, "python -m paper_1510_08224_amd.serving " + " ".join(sys.argv[1:])))


if __name__ == "__main__":
    main()
