"""Continuous-batching server: each request's result is the same alone and
in the mix (bitwise, FP32 storage: a batch member's state is bitwise its
state alone and the stopping rule depends only on its own residuals), the
HBM budget and slot limit bound what is resident, and requests that can
never fit are refused."""
import numpy as np
import pytest

from paper_1510_08224_amd import lbm, serving
from paper_1510_08224_amd import workloads as W

pytestmark = pytest.mark.gpu


def _requests():
    reqs = W.request_stream(7, rate=50.0, seed=11, n_range=(64, 160))
    return reqs


def test_each_result_equals_the_solve_alone():
    reqs = _requests()
    srv = serving.Server(hbm_budget=1 << 30, max_slots=4, tol=1e-6, check_every=500, cap=3000,
                         keep_fields=True)
    run = srv.run(reqs)
    srv.close()
    assert len(run["results"]) == len(reqs)
    for res in run["results"]:
        req = next(r for r in reqs if r.rid == res.rid)
        alone = serving.solve_alone(req, 1e-6, 500, 3000, keep_fields=True)
        assert res.steps == alone.steps and res.status == alone.status, res.rid
        for a, b in zip(res.fields, alone.fields):
            assert np.array_equal(a, b), res.rid
        assert res.nu == alone.nu


def test_budget_and_slots_bound_residency():
    reqs = _requests()
    need = sorted(serving.request_bytes(r.problem, "f32") for r in reqs)
    budget = need[-1] + need[-2] // 2        # never two of the largest at once
    srv = serving.Server(hbm_budget=budget, max_slots=2, tol=1e-6, check_every=500, cap=1500)
    peak_slots, peak_bytes = 0, 0
    orig = srv.admit

    def admit(req, now):
        slot = orig(req, now)
        nonlocal peak_slots, peak_bytes
        peak_slots = max(peak_slots, len(srv.active))
        peak_bytes = max(peak_bytes, srv.used)
        return slot

    srv.admit = admit
    run = srv.run(reqs)
    srv.close()
    assert len(run["results"]) == len(reqs) and run["refused"] == 0
    assert peak_slots <= 2 and peak_bytes <= budget


def test_request_larger_than_budget_is_refused():
    reqs = _requests()
    smallest = min(serving.request_bytes(r.problem, "f32") for r in reqs)
    srv = serving.Server(hbm_budget=smallest, max_slots=4, tol=1e-6, check_every=500, cap=500)
    run = srv.run(reqs)
    srv.close()
    assert run["refused"] == sum(serving.request_bytes(r.problem, "f32") > smallest for r in reqs)
    assert len(run["results"]) == len(reqs) - run["refused"]


def test_requests_retire_on_the_residual_and_free_slots_are_reused():
    """Solves that reach the steady-state residual (max |du|, |dT| over 1000
    steps below 1e-7) retire at different steps while another stays
    resident, and a queued request is admitted into the freed slot; every
    result is bitwise the solve alone (same stopping step, fields and Nu)."""
    specs = [("cavity", W.cavity(16, 1e3)), ("cavity", W.cavity(24, 1e4)),
             ("rb", W.rayleigh_benard(32, 16, 1e3)), ("cavity", W.cavity(32, 3e3)),
             ("cavity", W.cavity(48, 1e3))]
    reqs = [W.Request(rid=k, arrival=0.0, problem=pb, kind=kind) for k, (kind, pb) in enumerate(specs)]
    srv = serving.Server(hbm_budget=1 << 30, max_slots=2, tol=1e-7, check_every=1000, cap=60000,
                         keep_fields=True)
    events = []
    admit0, retire0 = srv.admit, srv.retire

    def admit(req, now):
        slot = admit0(req, now)
        events.append(("admit", req.rid, slot, len(srv.active)))
        return slot

    def retire(slot, now, status):
        res = retire0(slot, now, status)
        events.append(("retire", res.rid, slot, len(srv.active), status, res.steps))
        return res

    srv.admit, srv.retire = admit, retire
    run = srv.run(reqs)
    srv.close()
    res = {r.rid: r for r in run["results"]}
    assert sorted(res) == list(range(len(reqs)))
    assert all(r.status == "converged" for r in res.values()), {k: r.status for k, r in res.items()}
    assert len({r.steps for r in res.values()}) >= 3
    # a slot freed by a converged solve goes to a queued request while
    # another solve stays resident
    reused = [k for k in range(1, len(events))
              if events[k][0] == "admit" and events[k - 1][0] == "retire" and events[k - 1][4] == "converged"
              and events[k][2] == events[k - 1][2] and events[k - 1][3] >= 1]
    assert len(reused) >= 2, events
    for req in reqs:
        alone = serving.solve_alone(req, 1e-7, 1000, 60000, keep_fields=True)
        r = res[req.rid]
        assert (r.steps, r.status) == (alone.steps, alone.status), req.rid
        for a, b in zip(r.fields, alone.fields):
            assert np.array_equal(a, b), req.rid
        assert r.nu == alone.nu


def test_fp64_server_counts_fp64_bytes():
    pb = W.cavity(256, 1e4)
    assert serving.request_bytes(pb, "f64") > serving.request_bytes(pb, "f32") > serving.request_bytes(pb, "f16")
    srv = serving.Server(hbm_budget=serving.request_bytes(pb, "f32"), max_slots=4, storage="f64")
    req = W.Request(rid=0, arrival=0.0, problem=pb, kind="cavity")
    assert not srv.fits(req)
    srv.close()
