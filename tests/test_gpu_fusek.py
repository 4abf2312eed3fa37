"""K time steps per launch (LBM_POLICY_FUSEK): the kernel steps a tile grown
by K - 1 nodes from HBM into LDS, the tile grown by K - 2 .. 1 nodes within
LDS, and the tile again into HBM (K = 4 on 32 x 16 tiles for FP64 and FP32
storage with the D2Q5 model or the flow alone; K = 3 on 32 x 8 tiles for
FP64 storage with the D2Q9 thermal model).  It must give bitwise the
populations of K single steps for every collision operator and wall family,
ragged, periodic and open tiles, graph replay, and remainders run as pairs
or single steps.  Where no multi-step kernel exists (FP16 storage, FP32 with
the D2Q9 thermal model) or NEE walls leave a one-node edge tile, lbm_step
falls back to the pair (or single steps) and says so through
lbm_steps_per_launch."""
import numpy as np
import pytest

from gpu_util import max_rel_pop_error, run_pair
from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W
from test_gpu_fuse2 import CASES, _lid, _run, _sides

pytestmark = pytest.mark.gpu
F2, FK = lbm.LBM_POLICY_FUSE2, lbm.LBM_POLICY_FUSEK
K = 4        # D2Q5 and the flow alone
K9 = 3       # the D2Q9 thermal model (FP64)
BANDS, STRIPS, KEEP = lbm.LBM_POLICY_XCD_BANDS, lbm.LBM_POLICY_XCD_STRIPS, lbm.LBM_POLICY_KEEP_STORES

# built for FP64 and FP32 storage with D2Q5 or no temperature field; 32 x 16
# tiles (NEE with nx % 32 == 1 or ny % 16 == 1 falls back: 129 columns, 49
# rows)
FALLBACKK = {"nee_last_column_one_wide", "nee_top_row_one_high"}


def _built(model, storage):
    return (model in ("d2q5", "isothermal") and storage in ("f64", "f32")) or (model == "d2q9t" and storage == "f64")


def _k(model):
    return K9 if model == "d2q9t" else K


def _multi(case, storage):
    model, mk, _ = CASES[case]
    return _built(model, storage) and case not in FALLBACKK


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("case", list(CASES))
def test_k_steps_equal_single_steps(case, storage):
    model, mk, _ = CASES[case]
    pb = mk()
    T = W.random_temperature(pb.nx, pb.ny, 0.0, 1.0, seed=22)
    # 4 and 8 run as K-step launches only; 9, 10 and 11 leave one, two and
    # three steps over
    steps = [1, 4, 2, 8, 9, 10, 11]
    (fa, ga), ta = _run(model, pb, storage, steps, 0, 0, T, spl=1)
    k = _k(model) if _multi(case, storage) else 1
    for pol in (FK, FK | BANDS | KEEP, FK | STRIPS):
        (fb, gb), tb = _run(model, pb, storage, steps, pol, 0, T, spl=k)
        assert ta == tb == sum(steps)
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), pol
    # with pairs allowed too: remainders of two run as a pair, and lattices
    # without a multi-step kernel take pairs
    pair = 1 if case in ("nee_last_column_one_wide", "nee_top_row_one_high") else 2
    (fb, gb), tb = _run(model, pb, storage, steps, FK | F2 | BANDS, 0, T, spl=k if k > 1 else pair)
    assert ta == tb
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_k_steps_graph_replay(storage):
    pb = W.cavity(130, 1e5, ny=70)
    T = W.random_temperature(130, 70, 0.0, 1.0, seed=6)
    ref = _run("d2q5", pb, storage, [9, 9, 5, 18], 0, 0, T, spl=1)
    # graphs hold an even number of steps: 12 is three K-step launches (an
    # odd launch count swaps the buffers), 10 two and a pair, 6 one K-step
    # launch and two single steps, 14 three and a pair
    for graph, pol in ((12, FK), (10, FK | F2), (6, FK), (14, FK | F2)):
        got = _run("d2q5", pb, storage, [9, 9, 5, 18], pol, graph, T)
        assert got[1] == ref[1]
        assert np.array_equal(got[0][0], ref[0][0]) and np.array_equal(got[0][1], ref[0][1]), graph


@pytest.mark.parametrize("model", ["d2q5", "isothermal", "d2q9t"])
def test_k_steps_match_oracle(model):
    pb = W.with_nee_walls(W.cavity(100, 1e5, ny=44)) if model != "isothermal" else _lid(100).replace(ny=44)
    S, L = run_pair(pb, 42, launch=(0, 0, 0, FK | BANDS), model=model)
    assert S.steps_per_launch == _k(model)
    fa, ga = S.get_populations()
    fo, go = L.get_state()
    ef, eg = max_rel_pop_error(pb, fa, ga, fo, go)
    assert ef < 1e-12 and eg < 1e-12
    S.close()


@pytest.mark.parametrize("storage,model", [("f64", "d2q5"), ("f32", "d2q5"), ("f64", "d2q9t")])
def test_k_steps_full_size(storage, model):
    """The 2048^2 heated cavity of the benchmark, in the launch it times:
    K steps per launch equal K single steps bitwise."""
    pb = W.workload_cavity2048()
    runs = []
    for pol in (0, FK | BANDS):
        S = lbm.Solver(2048, 2048, storage, model=model)
        S.set_params(pb)
        S.set_launch(policy=pol)
        S.step(9)
        runs.append(S.get_populations())
        assert S.steps_per_launch == (_k(model) if pol else 1)
        S.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


# lattices narrower or shorter than the tile and its three-node margin, one
# node wide, and sizes one past a tile edge: every step's region must still
# visit each node once (periodic axes wrap the margins several times)
@pytest.mark.parametrize("storage,model", [("f64", "d2q5"), ("f32", "d2q5"), ("f64", "d2q9t")])
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 6), (7, 1), (2, 2), (3, 7), (2, 11), (33, 3), (32, 16), (34, 17),
                                   (65, 3), (66, 9), (129, 17), (70, 5)])
def test_k_steps_degenerate_sizes(storage, model, nx, ny):
    T = W.random_temperature(nx, ny, 0.0, 1.0, seed=nx * 100 + ny + 7)
    for px in (False, True):
        for py in (False, True):
            pb = _sides(W.cavity(max(nx, ny), 1e4).replace(nx=nx, ny=ny, wall_u=((0.0, 0.01), (0.0, -0.02),
                                                                                   (0.03, 0.0), (0.05, 0.0))),
                        px, py)
            (fa, ga), _ = _run(model, pb, storage, [1, 4, 3, 8], 0, 0, T, spl=1)
            (fb, gb), _ = _run(model, pb, storage, [1, 4, 3, 8], FK, 0, T, spl=_k(model))
            assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (px, py)


# ---------------------------------------------------------------------------
# K steps per launch for a whole batch (lbm_batch_set_policy).
# ---------------------------------------------------------------------------
from test_gpu_batch import _alone, _batch  # noqa: E402
from test_gpu_batch import _fused_mix  # noqa: E402


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_k_step_batch_matches_alone_bitwise(storage):
    mix = _fused_mix()
    B, sols = _batch(storage, mix)
    B.set_policy(FK | F2)
    assert B.steps_per_launch == (K if storage != "f16" else 2)
    B.step(37)            # 9 K-step launches and one single step
    B.step(26)            # 6 K-step launches and a pair
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


def test_k_step_batch_graphs_and_membership():
    # graphs of 8 steps hold 2 K-step launches (an even count); of 6, one
    # K-step launch and a pair; of 4, one K-step launch (an odd count swaps
    # the buffers)
    for graph in (8, 6, 4):
        mix = _fused_mix()
        B, sols = _batch("f32", mix, graph=graph)
        B.set_policy(FK | F2)
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


def test_k_step_batch_policy_rules():
    B = lbm.Batch("f32")
    S = B.new_solver(64, 64)
    S.set_params(W.cavity(64, 1e4))
    B.add(S)
    assert B.steps_per_launch == 2            # a small batch within the last-level cache: pairs
    B.set_policy(FK)
    assert B.steps_per_launch == K
    B.set_policy(FK | F2)
    assert B.steps_per_launch == K
    # a wall rebuilt by extrapolation on a one-row edge tile of the 16-row
    # K-step tiles (33 rows; the FP32 pair's 12-row tiles leave 9): pairs
    S2 = B.new_solver(100, 33)
    pb2 = W.with_nee_walls(W.cavity(100, 1e4, ny=33))
    S2.set_params(pb2)
    slot2 = B.add(S2)
    assert B.steps_per_launch == 2
    B.set_policy(FK)
    assert B.steps_per_launch == 1
    B.step(9)
    fa, ga = _alone(pb2, None, "f32", 9)
    assert np.array_equal(fa, S2.get_populations()[0])
    B.remove(slot2)
    assert B.steps_per_launch == K
    for bad in (1, 4, 32, FK | 1, -3):
        with pytest.raises(lbm.LbmError):
            B.set_policy(bad)
    B.close()


def test_d2q9t_k_step_batch_matches_alone_bitwise():
    """FP64 batches of D2Q9 thermal members take three steps per launch by
    default; every member equals its single steps alone."""
    mix = [W.cavity(70, 1e5, ny=45), W.with_nee_walls(W.cavity(96, 2e5, ny=70)), W.rayleigh_benard(130, 37, 2e4),
           W.cavity(33, 1e4, ny=17)]
    B = lbm.Batch("f64")
    sols = []
    for pb in mix:
        S = B.new_solver(pb.nx, pb.ny, model="d2q9t")
        S.set_params(pb)
        B.add(S)
        sols.append(S)
    assert B.steps_per_launch == K9
    B.step(37)            # 12 three-step launches and one single step
    B.step(26)            # 8 three-step launches and a pair
    for pb, S in zip(mix, sols):
        A = lbm.Solver(pb.nx, pb.ny, "f64", model="d2q9t")
        A.set_params(pb)
        A.set_launch(policy=0)
        A.step(63)
        fa, ga = A.get_populations()
        A.close()
        fb, gb = S.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), pb.name
        assert S.time == 63
    B.close()


# walls rebuilt by extrapolation with a one-node last tile: K-step tiles are
# 32 wide and 16 (D2Q5, no temperature) or 8 (D2Q9 thermal) high, pair tiles
# 64 wide and 8 high (12 for FP32 D2Q5); each launch kind falls back on its
# own, so a lattice may lose the K-step launch and keep the pair
@pytest.mark.parametrize("model,storage,nx,ny,spl", [
    ("d2q5", "f64", 97, 40, 2),      # 97 % 32 == 1: pairs
    ("d2q5", "f64", 100, 49, 1),     # 49 % 16 == 1 and 49 % 8 == 1: single steps
    ("d2q5", "f64", 100, 41, 4),     # 41 % 16 == 9: K steps
    ("d2q5", "f32", 97, 40, 2),      # FP32 pair tiles are 12 high: 40 % 12 == 4
    ("d2q9t", "f64", 100, 41, 1),    # 41 % 8 == 1 for both tiles
    ("d2q9t", "f64", 97, 44, 2),     # 97 % 32 == 1, 97 % 64 == 33: pairs
    ("d2q9t", "f64", 100, 44, 3),
])
def test_nee_one_node_edge_tiles_fall_back_per_launch_kind(model, storage, nx, ny, spl):
    pb = W.with_nee_walls(W.cavity(nx, 1e5, ny=ny))
    T = W.random_temperature(nx, ny, 0.0, 1.0, seed=nx + ny)
    (fa, ga), ta = _run(model, pb, storage, [5, 6], 0, 0, T, spl=1)
    (fb, gb), tb = _run(model, pb, storage, [5, 6], FK | F2 | BANDS, 0, T, spl=spl)
    assert ta == tb == 11
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
