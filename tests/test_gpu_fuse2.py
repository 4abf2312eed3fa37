"""Two time steps per launch (LBM_POLICY_FUSE2): the fused kernel steps a
tile and its halo from HBM into LDS and the tile again from LDS, and must
give bitwise the populations of two single steps, for every storage,
temperature model and wall family, on ragged and periodic lattices, with
and without graph replay, including the cases where lbm_step falls back to
single steps (NEE walls with a one-node edge tile).  The comparison
collision operators (BGK, orthogonal MRT) fuse too.  Tiles whose halo is
clear of the lattice's edges ("open" tiles: every 130-wide case has some)
take a path without per-slot tests and must match as well."""
import numpy as np
import pytest

import oracle
from gpu_util import max_rel_pop_error, run_pair
from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W

pytestmark = pytest.mark.gpu
FUSE = lbm.LBM_POLICY_FUSE2


def _lid(n, re=100.0, u0=0.1):
    return W.lid_cavity(n, oracle.rate_for_reynolds(re, n, u0), u0)


CASES = {
    "cavity150x70": ("d2q5", lambda: W.cavity(150, 1e5, ny=70), 8),
    # open tiles (tile and halo clear of the lattice's edges) take a path
    # without per-slot tests; a lattice with many of them, every operator
    "open_cavity330x90": ("d2q5", lambda: W.cavity(330, 1e5, ny=90), 8),
    "open_bgk_cavity330x90": ("d2q5", lambda: W.cavity(330, 1e5, ny=90).replace(collision=W.COLL_BGK), 8),
    "open_ortho_cavity330x90": ("d2q5", lambda: W.cavity(330, 1e5, ny=90).replace(collision=W.COLL_ORTHO), 8),
    "rb130x37": ("d2q5", lambda: W.rayleigh_benard(130, 37, 2e4), 8),
    "periodic70x45": ("d2q5", lambda: W.periodic_box(70, 45, s_nu=1.1, zeta_alpha=1.3, ax=2e-4, ay=1e-4,
                                                     u_c=0.05), 8),
    "small20x9": ("d2q5", lambda: W.cavity(20, 1e4, ny=9), 8),
    "injection13x20": ("d2q5", lambda: W.channel(13, 20, s_nu=0.8, zeta_alpha=0.9, u_top=(0.02, 0.01),
                                                 u_bottom=(0.0, 0.01)), 8),
    "moving_walls130x40": ("d2q5", lambda: W.cavity(130, 1e5, ny=40).replace(
        wall_u=((0.0, 0.003), (0.0, -0.01), (0.01, 0.0), (0.05, 0.0))), 8),
    "nee_cavity130x70": ("d2q5", lambda: W.with_nee_walls(W.cavity(130, 3e5, ny=70)), 8),
    "nee_rb140x34": ("d2q5", lambda: W.with_nee_walls(W.rayleigh_benard(140, 34, 2e4)), 8),
    "nee_top_row_one_high": ("d2q5", lambda: W.with_nee_walls(W.cavity(130, 1e4, ny=49)), 8),
    "nee_last_column_one_wide": ("d2q5", lambda: W.with_nee_walls(W.cavity(129, 1e4, ny=40)), 8),
    "d2q9t_cavity130x50": ("d2q9t", lambda: W.cavity(130, 1e5, ny=50), 8),
    "d2q9t_nee_cavity70x42": ("d2q9t", lambda: W.with_nee_walls(W.cavity(70, 1e5, ny=42)), 8),
    "iso_lid130x61": ("isothermal", lambda: _lid(130).replace(ny=61), 8),
    "iso_nee_lid66x35": ("isothermal", lambda: W.with_nee_walls(_lid(66).replace(ny=35)), 8),
    "bgk_cavity90x30": ("d2q5", lambda: W.cavity(90, 1e5, ny=30).replace(collision=W.COLL_BGK), 8),
    "ortho_nee_cavity130x70": ("d2q5", lambda: W.with_nee_walls(W.cavity(130, 1e5, ny=70)).replace(
        collision=W.COLL_ORTHO), 8),
    "bgk_iso_lid130x61": ("isothermal", lambda: _lid(130).replace(ny=61, collision=W.COLL_BGK), 8),
    "ortho_d2q9t_rb130x42": ("d2q9t", lambda: W.rayleigh_benard(130, 42, 2e4).replace(collision=W.COLL_ORTHO), 8),
}


# cases where lbm_step must fall back to single steps: walls rebuilt by
# extrapolation with a one-node edge tile (64-wide tiles of 8 rows, 12 for
# FP32/FP16 D2Q5: 49 rows leave one in the last tile for both)
FALLBACK = {"nee_last_column_one_wide", "nee_top_row_one_high"}


def _run(model, pb, storage, steps, policy, graph, T=None, spl=None):
    S = lbm.Solver(pb.nx, pb.ny, storage, model=model)
    S.set_params(pb)
    S.set_graph_steps(graph)
    if policy is not None:
        S.set_launch(policy=policy)
    if T is not None and model != "isothermal":
        S.init_temperature(T)
    if spl is not None:
        assert S.steps_per_launch == spl
    for k in steps:
        S.step(k)
    out = S.get_populations(), S.time
    S.close()
    return out


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("case", list(CASES))
def test_fused_pairs_equal_single_steps(case, storage):
    model, mk, _ = CASES[case]
    pb = mk()
    T = W.random_temperature(pb.nx, pb.ny, 0.0, 1.0, seed=21)
    steps = [1, 2, 3, 7, 11]
    (fa, ga), ta = _run(model, pb, storage, steps, 0, 0, T, spl=1)
    for pol in (FUSE, FUSE | lbm.LBM_POLICY_XCD_BANDS | lbm.LBM_POLICY_KEEP_STORES,
                FUSE | lbm.LBM_POLICY_XCD_STRIPS):
        (fb, gb), tb = _run(model, pb, storage, steps, pol, 0, T, spl=1 if case in FALLBACK else 2)
        assert ta == tb == sum(steps)
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), pol


def test_fused_graph_replay():
    pb = W.cavity(130, 1e5, ny=70)
    T = W.random_temperature(130, 70, 0.0, 1.0, seed=5)
    ref = _run("d2q5", pb, "f64", [8, 8, 5, 16], 0, 0, T, spl=1)
    for graph in (8, 6):   # 4 and 3 fused launches per graph: odd launch counts swap the buffers
        got = _run("d2q5", pb, "f64", [8, 8, 5, 16], FUSE, graph, T)
        assert got[1] == ref[1]
        assert np.array_equal(got[0][0], ref[0][0]) and np.array_equal(got[0][1], ref[0][1])


@pytest.mark.parametrize("model", ["d2q5", "d2q9t", "isothermal"])
def test_fused_matches_oracle(model):
    pb = W.with_nee_walls(W.cavity(100, 1e5, ny=44)) if model != "isothermal" else _lid(100).replace(ny=44)
    S, L = run_pair(pb, 40, launch=(0, 0, 0, FUSE | lbm.LBM_POLICY_XCD_BANDS), model=model)
    assert S.get_launch()[3] & FUSE
    fa, ga = S.get_populations()
    fb, gb = L.get_state()
    ef, eg = max_rel_pop_error(pb, fa, ga, fb, gb)
    assert ef < 1e-12 and eg < 1e-12, (ef, eg)
    S.close()


def test_fused_full_size_cavity2048():
    pb = W.workload_cavity2048()
    T = W.random_temperature(2048, 2048, 0.0, 1.0, seed=3)
    ref = _run("d2q5", pb, "f64", [4], 0, 0, T, spl=1)
    got = _run("d2q5", pb, "f64", [4], FUSE, 0, T, spl=2)
    assert np.array_equal(got[0][0], ref[0][0]) and np.array_equal(got[0][1], ref[0][1])


def _sides(pb, px, py):
    """The cavity's walls with the x and/or y sides made periodic."""
    flow = ((W.FLOW_PERIODIC,) * 2 if px else (W.FLOW_WALL,) * 2) + \
           ((W.FLOW_PERIODIC,) * 2 if py else (W.FLOW_WALL,) * 2)
    temp = ((W.TEMP_PERIODIC,) * 2 if px else (W.TEMP_DIRICHLET,) * 2) + \
           ((W.TEMP_PERIODIC,) * 2 if py else (W.TEMP_ADIABATIC,) * 2)
    return pb.replace(bc_flow=flow, bc_temp=temp)


# lattices narrower or shorter than a tile, one node wide, and sizes one
# past a tile edge: the first fused step's slot order must still visit each
# node of the tile and halo once
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 6), (7, 1), (2, 2), (3, 7), (65, 3), (64, 4), (66, 5), (129, 9)])
def test_fused_degenerate_sizes(storage, nx, ny):
    T = W.random_temperature(nx, ny, 0.0, 1.0, seed=nx * 100 + ny)
    for px in (False, True):
        for py in (False, True):
            pb = _sides(W.cavity(max(nx, ny), 1e4).replace(nx=nx, ny=ny), px, py)
            (fa, ga), _ = _run("d2q5", pb, storage, [1, 2, 3], 0, 0, T, spl=1)
            (fb, gb), _ = _run("d2q5", pb, storage, [1, 2, 3], FUSE, 0, T, spl=2)
            assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (px, py)


@pytest.mark.parametrize("nx,ny", [(1, 6), (7, 1), (2, 2), (3, 7), (65, 3)])
def test_degenerate_sizes_match_oracle(nx, ny):
    # a node that is a wall on both sides of an axis, in both step kernels
    T = W.random_temperature(nx, ny, 0.0, 1.0, seed=nx * 10 + ny)
    for px in (False, True):
        for py in (False, True):
            pb = _sides(W.cavity(max(nx, ny), 1e4).replace(nx=nx, ny=ny, wall_u=((0.0, 0.01), (0.0, -0.02),
                                                                                   (0.03, 0.0), (0.05, 0.0))),
                        px, py)
            for pol in (0, FUSE):
                S, L = run_pair(pb, 9, T_init=T, launch=(0, 0, 0, pol))
                fa, ga = S.get_populations()
                fb, gb = L.get_state()
                ef, eg = max_rel_pop_error(pb, fa, ga, fb, gb)
                assert ef < 1e-12 and eg < 1e-12, (px, py, pol, ef, eg)
                S.close()
