"""Three time steps per launch (LBM_POLICY_FUSE3): the kernel steps a tile
grown by two nodes from HBM into LDS, the tile grown by one node in place in
LDS, and the tile again into HBM.  It must give bitwise the populations of
three single steps for FP64 and FP32 storage, the D2Q5 model and the flow
alone, every collision operator and wall family, ragged, periodic and open
tiles, graph replay, and remainders run as pairs or single steps.  Where no
three-step kernel exists (FP16 storage, the D2Q9 thermal model) or NEE
walls leave a one-node edge tile, lbm_step falls back to the pair (or
single steps) and says so through lbm_steps_per_launch."""
import numpy as np
import pytest

from gpu_util import max_rel_pop_error, run_pair
from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W
from test_gpu_fuse2 import CASES, _lid, _run, _sides

pytestmark = pytest.mark.gpu
F2, F3 = lbm.LBM_POLICY_FUSE2, lbm.LBM_POLICY_FUSE3
BANDS, STRIPS, KEEP = lbm.LBM_POLICY_XCD_BANDS, lbm.LBM_POLICY_XCD_STRIPS, lbm.LBM_POLICY_KEEP_STORES

# built for FP64 and FP32 storage with D2Q5 or no temperature field; 64 x 8
# tiles (NEE with nx % 64 == 1 or ny % 8 == 1 falls back)
FALLBACK3 = {"nee_last_column_one_wide", "nee_top_row_one_high"}


def _built(model, storage):
    return model in ("d2q5", "isothermal") and storage in ("f64", "f32")


def _triple(case, storage):
    model, mk, _ = CASES[case]
    return _built(model, storage) and case not in FALLBACK3


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("case", list(CASES))
def test_three_steps_equal_single_steps(case, storage):
    model, mk, _ = CASES[case]
    pb = mk()
    T = W.random_temperature(pb.nx, pb.ny, 0.0, 1.0, seed=22)
    # 3 and 6 run as triples only; 7 and 11 leave one and two steps over
    steps = [1, 3, 2, 6, 7, 11]
    (fa, ga), ta = _run(model, pb, storage, steps, 0, 0, T, spl=1)
    k = 3 if _triple(case, storage) else 1
    for pol in (F3, F3 | BANDS | KEEP, F3 | STRIPS):
        (fb, gb), tb = _run(model, pb, storage, steps, pol, 0, T, spl=k)
        assert ta == tb == sum(steps)
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), pol
    # with pairs allowed too: remainders of two run as a pair, and lattices
    # without a three-step kernel take pairs
    pair = 1 if case in ("nee_last_column_one_wide", "nee_top_row_one_high") else 2
    (fb, gb), tb = _run(model, pb, storage, steps, F3 | F2 | BANDS, 0, T, spl=3 if k == 3 else pair)
    assert ta == tb
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_three_steps_graph_replay(storage):
    pb = W.cavity(130, 1e5, ny=70)
    T = W.random_temperature(130, 70, 0.0, 1.0, seed=6)
    ref = _run("d2q5", pb, storage, [9, 9, 5, 18], 0, 0, T, spl=1)
    # graphs hold an even number of steps: 12 is four triples, 10 three
    # triples and a single step, 8 two triples and a pair (an odd launch
    # count swaps the buffers), 6 two triples
    for graph, pol in ((12, F3), (10, F3), (8, F3 | F2), (6, F3 | F2)):
        got = _run("d2q5", pb, storage, [9, 9, 5, 18], pol, graph, T)
        assert got[1] == ref[1]
        assert np.array_equal(got[0][0], ref[0][0]) and np.array_equal(got[0][1], ref[0][1]), graph


@pytest.mark.parametrize("model", ["d2q5", "isothermal"])
def test_three_steps_match_oracle(model):
    pb = W.with_nee_walls(W.cavity(100, 1e5, ny=44)) if model != "isothermal" else _lid(100).replace(ny=44)
    S, L = run_pair(pb, 42, launch=(0, 0, 0, F3 | BANDS), model=model)
    assert S.steps_per_launch == 3
    fa, ga = S.get_populations()
    fo, go = L.get_state()
    ef, eg = max_rel_pop_error(pb, fa, ga, fo, go)
    assert ef < 1e-12 and eg < 1e-12
    S.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_three_steps_full_size(storage):
    """The 2048^2 heated cavity of the benchmark, in the launch it times:
    three steps per launch equal three single steps bitwise."""
    pb = W.workload_cavity2048()
    runs = []
    for pol in (0, F3 | BANDS):
        S = lbm.Solver(2048, 2048, storage)
        S.set_params(pb)
        S.set_launch(policy=pol)
        S.step(7)
        runs.append(S.get_populations())
        assert S.steps_per_launch == (3 if pol else 1)
        S.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


# lattices narrower or shorter than the tile and its two-node margin, one
# node wide, and sizes one past a tile edge: every step's region must still
# visit each node once (periodic axes wrap the margins several times)
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 6), (7, 1), (2, 2), (3, 7), (2, 11), (65, 3), (64, 8), (66, 9),
                                   (129, 17), (70, 5)])
def test_three_steps_degenerate_sizes(storage, nx, ny):
    T = W.random_temperature(nx, ny, 0.0, 1.0, seed=nx * 100 + ny + 7)
    for px in (False, True):
        for py in (False, True):
            pb = _sides(W.cavity(max(nx, ny), 1e4).replace(nx=nx, ny=ny, wall_u=((0.0, 0.01), (0.0, -0.02),
                                                                                   (0.03, 0.0), (0.05, 0.0))),
                        px, py)
            (fa, ga), _ = _run("d2q5", pb, storage, [1, 3, 2, 6], 0, 0, T, spl=1)
            (fb, gb), _ = _run("d2q5", pb, storage, [1, 3, 2, 6], F3, 0, T, spl=3)
            assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (px, py)


# ---------------------------------------------------------------------------
# Three steps per launch for a whole batch (lbm_batch_set_policy).
# ---------------------------------------------------------------------------
from test_gpu_batch import _alone, _batch  # noqa: E402
from test_gpu_batch import _fused_mix  # noqa: E402


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_three_step_batch_matches_alone_bitwise(storage):
    mix = _fused_mix()
    B, sols = _batch(storage, mix)
    B.set_policy(F3 | F2)
    assert B.steps_per_launch == (3 if storage != "f16" else 2)
    B.step(37)            # 12 three-step launches and one single step
    B.step(26)            # 8 three-step launches and a pair
    B.residual()          # first call: snapshot only
    B.step(1)
    r, bad = B.residual()
    for k, ((pb, mkT), S) in enumerate(zip(mix, sols)):
        A = lbm.Solver(pb.nx, pb.ny, storage)
        A.set_params(pb)
        A.set_launch(policy=0)
        if mkT:
            A.init_temperature(mkT())
        A.step(63)
        A.residual()
        A.step(1)
        ra, _ = A.residual()
        fa, ga = A.get_populations()
        A.close()
        fb, gb = S.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), pb.name
        assert S.time == 64 and bad[k] == 0
        assert r[k] == ra, pb.name
    B.close()


def test_three_step_batch_graphs_and_membership():
    # graphs of 6 steps hold 2 three-step launches (an even count); of 8,
    # two three-step launches and a pair (an odd count swaps the buffers)
    for graph in (6, 8):
        mix = _fused_mix()
        B, sols = _batch("f32", mix, graph=graph)
        B.set_policy(F3 | F2)
        B.step(13)
        B.remove(3)
        B.step(12)
        sols[0].step(1)       # a member stepped on its own
        B.step(7)
        expect = {0: 33, 3: 13}
        for k, S in enumerate(sols):
            pb, mkT = mix[k]
            fa, ga = _alone(pb, mkT() if mkT else None, "f32", expect.get(k, 32), launch=(64, 4, 1, 0))
            fb, gb = S.get_populations()
            assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (graph, k)
            assert S.time == expect.get(k, 32)
        B.close()


def test_three_step_batch_policy_rules():
    B = lbm.Batch("f32")
    S = B.new_solver(64, 64)
    S.set_params(W.cavity(64, 1e4))
    B.add(S)
    assert B.steps_per_launch == 2            # a small batch within the last-level cache: pairs
    B.set_policy(F3)
    assert B.steps_per_launch == 3
    B.set_policy(F3 | F2)
    assert B.steps_per_launch == 3
    # a wall rebuilt by extrapolation on a one-row edge tile of the 8-row
    # three-step tiles (41 rows; the FP32 pair's 12-row tiles leave 5): pairs
    S2 = B.new_solver(100, 41)
    pb2 = W.with_nee_walls(W.cavity(100, 1e4, ny=41))
    S2.set_params(pb2)
    slot2 = B.add(S2)
    assert B.steps_per_launch == 2
    B.set_policy(F3)
    assert B.steps_per_launch == 1
    B.step(9)
    fa, ga = _alone(pb2, None, "f32", 9)
    assert np.array_equal(fa, S2.get_populations()[0])
    B.remove(slot2)
    assert B.steps_per_launch == 3
    for bad in (1, 4, 32, F3 | 1, -3):
        with pytest.raises(lbm.LbmError):
            B.set_policy(bad)
    B.close()
