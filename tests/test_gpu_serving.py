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
