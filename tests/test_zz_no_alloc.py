"""lbm_residual_static, the residual for callers that cannot allocate: its
partial results live in a static device array instead of buffers the
handle allocates.  It must give bitwise lbm_residual's results on twin
solvers (same problem, same steps), on consecutive calls whose second has
a smaller lattice (fewer partials than the array's last contents), refuse
a handle without a residual snapshot and lattices beyond the array, and
report non-finite values like lbm_residual."""
import numpy as np
import pytest

from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W

pytestmark = pytest.mark.gpu


def _twins(pb, storage, T=None):
    out = []
    for _ in range(2):
        S = lbm.Solver(pb.nx, pb.ny, storage)
        S.set_params(pb)
        if T is not None:
            S.init_temperature(T)
        out.append(S)
    return out


def test_static_residual_equals_the_allocating_one():
    big = _twins(W.cavity(96, 1e5, ny=80), "f64")
    small_pb = W.rayleigh_benard(40, 24, 3e4)
    small = _twins(small_pb, "f32", W.rb_initial_temperature(40, 24, amp=1e-2, seed=5))
    for A, B in (big, small):
        ra, ba = A.residual()          # allocates the snapshots; first call: +inf
        rb, bb = B.residual()
        assert ra == rb == float("inf") and ba == bb == 0
    for rep in range(2):
        for A, B in (big, small):      # second call of each round: the smaller lattice
            A.step(300)
            B.step(300)
        got = [A.residual_static() for A, _ in (big, small)]
        want = [B.residual() for _, B in (big, small)]
        for (r1, b1), (r2, b2) in zip(got, want):
            assert np.float64(r1).tobytes() == np.float64(r2).tobytes() and b1 == b2, (rep, r1, r2)
            assert 0 < r1 < 1
    # a fresh call order: the small lattice right after the big one, alone
    A, B = big
    A.step(10); B.step(10)
    S, T = small
    S.step(10); T.step(10)
    assert A.residual_static() == B.residual()
    assert S.residual_static() == T.residual()
    for X in big + small:
        X.close()


def test_static_residual_reports_nonfinite_like_lbm_residual():
    pb = W.cavity(64, 1e4, ny=48)
    A, B = _twins(pb, "f64")
    for S in (A, B):
        S.residual()
        S.step(20)
        f, g = S.get_populations()
        f[3, 10, 17] = np.nan
        g[0, 30, 5] = np.inf
        S.set_populations(f, g)       # resets the snapshot: the next call only takes it
        S.residual(raise_unstable=False)
    with pytest.raises(lbm.LbmError) as e:
        A.residual_static()
    assert e.value.code == lbm.LBM_ERR_UNSTABLE
    assert A.residual_static(raise_unstable=False)[1] == B.residual(raise_unstable=False)[1] == 2
    A.close(); B.close()


def test_static_residual_needs_a_snapshot_and_a_fitting_lattice():
    pb = W.cavity(32, 1e4)
    S = lbm.Solver(32, 32, "f64")
    S.set_params(pb)
    with pytest.raises(lbm.LbmError) as e:
        S.residual_static()
    assert e.value.code == lbm.LBM_ERR_STATE
    S.close()
    # 4096^2 nodes is the largest lattice the static partials serve; one
    # more column is refused
    for nx, ok in ((4096, True), (4097, False)):
        pb = W.cavity(nx, 1e5, ny=4096)
        S = lbm.Solver(nx, 4096, "f16")
        S.set_params(pb)
        S.residual()
        S.step(2)
        if ok:
            r, bad = S.residual_static()
            assert 0 < r < 1 and bad == 0
        else:
            with pytest.raises(lbm.LbmError) as e:
                S.residual_static()
            assert e.value.code == lbm.LBM_ERR_ARG and "16777216" in str(e.value)
        S.close()
