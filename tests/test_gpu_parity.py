"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle
on the same seeded inputs, element by element.

Bar (FP64 storage): every pre-collision population within 1e-12 of the
oracle relative to max(|p_oracle|, p_ref), p_ref the rest weight of the
population (w_i for fbar, the D2Q5 rest equilibrium at the largest
temperature for g); moments within 1e-12 of the field scale; Nusselt
numbers within 1e-11 relative.  The oracle multiplies dense matrices without
FMA while the kernels use the sparse, fused form, so the two agree to
rounding, not bitwise.
"""
import numpy as np
import pytest

import oracle
from gpu_util import field_scale, max_rel_pop_error, run_pair
from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _check(pb, S, L, tol=TOL, nusselt=True):
    fa, ga = S.get_populations()
    fb, gb = L.get_state()
    ef, eg = max_rel_pop_error(pb, fa, ga, fb, gb)
    assert ef < tol and eg < tol, (ef, eg)
    us, ts = field_scale(pb)
    mg, mo = S.moments(), L.moments()
    assert np.max(np.abs(mg[0] - mo[0])) < tol
    assert np.max(np.abs(mg[1] - mo[1])) < tol * us and np.max(np.abs(mg[2] - mo[2])) < tol * us
    assert np.max(np.abs(mg[3] - mo[3])) < tol * ts
    if nusselt:
        for side in range(4):
            if pb.bc_temp[side] not in (W.TEMP_DIRICHLET, W.TEMP_NEE_DIRICHLET):
                continue
            depth = pb.nx if side in (W.LEFT, W.RIGHT) else pb.ny
            if depth < 3 or pb.t_hot == pb.t_cold:
                continue
            a = S.nusselt(side)
            b = L.nusselt(side)
            assert abs(a[0] - b[0]) <= 1e-11 * max(1.0, abs(b[0]))
            assert abs(a[1] - b[1]) <= 1e-11 * max(1.0, abs(b[1]))
            loc_a = S.nusselt_local(side)
            loc_b = L.nusselt(side, local=True)[3]
            assert np.max(np.abs(loc_a - loc_b)) <= 1e-11 * max(1.0, np.max(np.abs(loc_b)))
    return ef, eg


def test_single_node_periodic_is_pure_collision():
    # 1 x 1 fully periodic lattice: streaming maps every link onto the node
    # itself, so one step is one collision.
    for seed in range(4):
        rng = np.random.default_rng(seed)
        pb = W.periodic_box(1, 1, s_nu=float(rng.uniform(0.5, 1.9)), zeta_alpha=float(rng.uniform(0.5, 1.9)),
                            ax=1e-3, ay=-2e-3, u_c=0.05, s_e=1.4, s_q=0.9, s_eps=1.7, zeta_e=1.3, zeta_nu=0.7)
        pops = W.random_populations(1, 1, seed=seed, spread=0.5)
        S, L = run_pair(pb, 1, pops=pops)
        fa, ga = S.get_populations()
        fb, gb = L.get_state()
        assert np.max(np.abs(fa - fb)) < 1e-15 and np.max(np.abs(ga - gb)) < 1e-15
        S.close()


CASES = {
    "cavity64_ra1e4": (lambda: W.cavity(64, 1e4), None, None),
    "cavity37x23_ra1e5_randT": (lambda: W.cavity(37, 1e5, ny=23),
                                lambda pb: W.random_temperature(37, 23, 0.0, 1.0, seed=11), None),
    "rb50x17_noise": (lambda: W.rayleigh_benard(50, 17, 2e4),
                      lambda pb: W.rb_initial_temperature(50, 17, amp=1e-2, seed=1510), None),
    "injection_channel13x20": (lambda: W.channel(13, 20, s_nu=0.8, zeta_alpha=0.9, u_top=(0.02, 0.01),
                                                 u_bottom=(0.0, 0.01), t_bottom=0.0, t_top=1.0), None, None),
    "periodic_box19x11_random": (lambda: W.periodic_box(19, 11, s_nu=1.1, zeta_alpha=1.3, ax=2e-4, ay=1e-4,
                                                        u_c=0.05), None, lambda pb: W.random_populations(19, 11, 3)),
    "adiabatic_box16x9_random": (lambda: W.cavity(16, 1e4, ny=9).replace(bc_temp=(W.TEMP_ADIABATIC,) * 4),
                                 None, lambda pb: W.random_populations(16, 9, 4)),
    "y_periodic_21x14": (lambda: W.cavity(21, 1e4, ny=14).replace(
        bc_flow=(W.FLOW_WALL, W.FLOW_WALL, W.FLOW_PERIODIC, W.FLOW_PERIODIC),
        bc_temp=(W.TEMP_DIRICHLET, W.TEMP_DIRICHLET, W.TEMP_PERIODIC, W.TEMP_PERIODIC),
        wall_u=((0.0, 0.01), (0.0, -0.02), (0.0, 0.0), (0.0, 0.0))), None, lambda pb: W.random_populations(21, 14, 5)),
    "lid_cavity_moving_walls_30x30": (lambda: W.cavity(30, 1e5).replace(
        wall_u=((0.0, 0.003), (0.0, 0.0), (0.01, 0.0), (0.05, 0.0))), None, None),
    "cavity_paper_temperatures_24": (lambda: W.cavity(24, 1e4, t_hot=21.0, t_cold=1.0), None, None),
    # non-equilibrium extrapolation walls (walls through the edge nodes)
    "nee_cavity40x30_randT": (lambda: W.with_nee_walls(W.cavity(40, 1e5, ny=30)),
                              lambda pb: W.random_temperature(40, 30, 0.0, 1.0, seed=13), None),
    "nee_cavity130x70_fastpath": (lambda: W.with_nee_walls(W.cavity(130, 3e5, ny=70)), None, None),
    "nee_rb70x17_noise": (lambda: W.with_nee_walls(W.rayleigh_benard(70, 17, 2e4)),
                          lambda pb: W.rb_initial_temperature(70, 17, amp=1e-2, seed=7), None),
    "nee_injection_channel13x21": (lambda: W.with_nee_walls(W.channel(13, 21, s_nu=0.8, zeta_alpha=0.9,
                                   u_top=(0.02, 0.01), u_bottom=(0.0, 0.01))), None, None),
    "nee_cavity_random_pops_24x20": (lambda: W.with_nee_walls(W.cavity(24, 1e4, ny=20)), None,
                                     lambda pb: W.random_populations(24, 20, 17)),
}


@pytest.mark.parametrize("steps", [1, 10, 100])
@pytest.mark.parametrize("case", list(CASES))
def test_parity_short_runs(case, steps):
    mk, mkT, mkP = CASES[case]
    pb = mk()
    T = mkT(pb) if mkT else None
    P = mkP(pb) if mkP else None
    S, L = run_pair(pb, steps, T_init=T, pops=P)
    _check(pb, S, L)
    S.close()


def test_parity_cavity64_20000_steps():
    """The 64 x 64 cavity, Ra = 1e4, Pr = 0.71, u_c = 0.1, from rest at
    T = 0.5, 20000 steps: every population, u, v, T and both wall Nusselt
    numbers."""
    pb = W.workload_cavity64()
    S, L = run_pair(pb, 20000)
    ef, eg = _check(pb, S, L)
    print(f"cavity64 20000 steps: max rel population error f {ef:.3e} g {eg:.3e}")
    nu_g, nu_o = S.nusselt(W.LEFT)[0], L.nusselt(W.LEFT)[0]
    assert abs(nu_g - 2.2447) < 0.02          # near-steady Nu of this workload
    S.close()


@pytest.mark.parametrize("launch", [(64, 4, 1, 0), (128, 2, 2, 3), (256, 1, 2, 1), (64, 1, 2, 2),
                                    (128, 1, 1, lbm.LBM_POLICY_DEFAULT), (64, 4, 1, 4), (64, 2, 2, 6)])
def test_launch_shape_and_policy_do_not_change_results(launch):
    pb = W.cavity(150, 1e5, ny=70)
    T = W.random_temperature(150, 70, 0.0, 1.0, seed=8)
    ref = lbm.Solver(150, 70, "f64")
    ref.set_params(pb)
    ref.init_temperature(T)
    ref.step(60)
    fa, ga = ref.get_populations()
    S = lbm.Solver(150, 70, "f64")
    S.set_params(pb)
    S.set_launch(*launch)
    S.init_temperature(T)
    S.step(60)
    fb, gb = S.get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    ref.close(); S.close()


@pytest.mark.parametrize("launch", [(64, 4, 1, 4), (64, 2, 2, 6), (128, 2, 1, 4)])
def test_xcd_strips_order_does_not_change_results(launch):
    # 512 columns: 8 tiles of 64 per row (strips active) or 4 of 128 (bands)
    pb = W.rayleigh_benard(512, 37, 3e4)
    T = W.rb_initial_temperature(512, 37, amp=1e-2, seed=4)
    runs = []
    for shape in (None, launch):
        S = lbm.Solver(512, 37, "f64")
        S.set_params(pb)
        if shape:
            S.set_launch(*shape)
        S.init_temperature(T)
        S.step(25)
        runs.append(S.get_populations())
        S.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("n,storage,model,policy", [
    # FP64 with D2Q5 or no temperature: K steps per launch with bands at
    # every size (pairs allowed for remainders), kept stores within the
    # last-level cache
    (64, "f64", "d2q5", 27), (1024, "f64", "d2q5", 27), (2048, "f64", "d2q5", 25), (4096, "f64", "d2q5", 25),
    (3072, "f64", "isothermal", 25), (2048, "f64", "isothermal", 25), (512, "f64", "isothermal", 27),
    # FP32: K steps beyond the last-level cache and up to 96 MiB (kept
    # stores), fused pairs between
    (1024, "f32", "d2q5", 11), (2048, "f32", "d2q5", 25), (3072, "f32", "d2q5", 25), (2048, "f32", "isothermal", 25),
    (1024, "f32", "isothermal", 27), (512, "f32", "d2q5", 27), (64, "f32", "d2q5", 27), (1200, "f32", "isothermal", 11),
    # D2Q9 thermal: K steps for FP64 too; FP32 (no multi-step kernel) fused pairs
    (3072, "f64", "d2q9t", 25), (2048, "f64", "d2q9t", 25), (512, "f64", "d2q9t", 27), (2048, "f32", "d2q9t", 9),
    # FP16: fused pairs with bands for every model and size
    (1024, "f16", "d2q5", 11), (2048, "f16", "d2q5", 11), (2048, "f16", "d2q9t", 9), (3072, "f16", "d2q5", 9),
    (4096, "f16", "d2q5", 9), (1024, "f16", "isothermal", 11), (4096, "f16", "isothermal", 9)])
def test_default_policy_follows_footprint(n, storage, model, policy):
    S = lbm.Solver(n, n, storage, model=model)
    assert S.get_launch()[3] == policy
    S.set_launch(policy=lbm.LBM_POLICY_XCD_BANDS)
    assert S.get_launch()[3] == lbm.LBM_POLICY_XCD_BANDS
    S.set_launch(policy=lbm.LBM_POLICY_DEFAULT)
    assert S.get_launch()[3] == policy
    with pytest.raises(lbm.LbmError):
        S.set_launch(policy=lbm.LBM_POLICY_XCD_BANDS | lbm.LBM_POLICY_XCD_STRIPS)
    with pytest.raises(lbm.LbmError):
        S.set_launch(policy=32)
    S.set_launch(policy=lbm.LBM_POLICY_XCD_STRIPS | lbm.LBM_POLICY_KEEP_STORES)
    assert S.get_launch()[3] == lbm.LBM_POLICY_XCD_STRIPS | lbm.LBM_POLICY_KEEP_STORES
    with pytest.raises(lbm.LbmError):
        S.set_launch(rows=4)
    S.close()


def test_autotune_keeps_state_and_results():
    from paper_1510_08224_amd import tuning
    pb = W.cavity(150, 1e5, ny=70)
    T = W.random_temperature(150, 70, 0.0, 1.0, seed=8)
    runs = []
    for tune in (False, True):
        S = lbm.Solver(150, 70, "f64")
        S.set_params(pb)
        S.init_temperature(T)
        S.step(7)
        if tune:
            bx, pol, gbs = tuning.autotune(S, steps=4)
            assert S.get_launch()[0] == bx and S.get_launch()[3] == pol and gbs > 0
            assert S.time == 7
        S.step(30)
        runs.append(S.get_populations())
        S.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_set_get_roundtrip_and_checkpoint():
    pb = W.rayleigh_benard(40, 20, 5e4)
    f0, g0 = W.random_populations(40, 20, seed=12)
    S = lbm.Solver(40, 20, "f64")
    S.set_params(pb)
    S.set_populations(f0, g0)
    f1, g1 = S.get_populations()
    assert np.max(np.abs(f1 - f0)) < 1e-16 and np.max(np.abs(g1 - g0)) < 4e-16
    S.step(37)
    blob = S.save_state()
    S.step(41)
    fa, ga = S.get_populations()
    S.load_state(blob)
    assert S.time == 37
    S.step(41)
    fb, gb = S.get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    S.close()


def test_residual_matches_oracle_and_flags_nonfinite():
    pb = W.cavity(48, 1e4)
    S = lbm.Solver(48, 48, "f64")
    S.set_params(pb)
    L = oracle.Lattice(pb)
    r0, bad0 = S.residual()
    assert r0 == float("inf") and bad0 == 0
    prev = L.moments()[1:]
    S.step(300); L.step(300)
    r, bad = S.residual()
    ro = oracle.residual(prev, L.moments()[1:])
    assert bad == 0 and abs(r - ro) <= 1e-12 * max(ro, 1e-300) + 1e-17
    # a non-finite population is reported, and only as an error code
    f, g = S.get_populations()
    f[3, 10, 7] = np.nan
    S.set_populations(f, g)
    S.residual(raise_unstable=False)
    r, bad = S.residual(raise_unstable=False)
    assert bad >= 1
    with pytest.raises(lbm.LbmError) as e:
        S.residual()
    assert e.value.code == lbm.LBM_ERR_UNSTABLE
    S.close()


def test_torch_memory_and_stream_path():
    import torch
    pb = W.cavity(33, 1e5)
    a = lbm.Solver(33, 33, "f64")
    a.set_params(pb)
    a.step(50)
    b = lbm.Solver(33, 33, "f64", torch_memory=True)
    b.set_params(pb)
    b.step(50)
    fa, ga = a.get_populations()
    fb, gb = b.get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    rho = torch.empty(33 * 33, dtype=torch.float64, device="cuda")
    T = torch.empty(33 * 33, dtype=torch.float64, device="cuda")
    b.moments_device(rho=rho, T=T)
    b.synchronize()
    m = b.moments()
    assert np.array_equal(rho.cpu().numpy().reshape(33, 33), m[0])
    assert np.array_equal(T.cpu().numpy().reshape(33, 33), m[3])
    a.close(); b.close()


def test_error_paths():
    S = lbm.Solver(8, 8, "f64")
    with pytest.raises(lbm.LbmError) as e:
        S.step(1)
    assert e.value.code == lbm.LBM_ERR_STATE
    with pytest.raises(lbm.LbmError) as e:
        S.set_params(W.cavity(8, 1e4).replace(s_e=2.5))
    assert e.value.code == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LbmError) as e:
        S.set_params(W.cavity(8, 1e4).replace(varpi=1.0))
    assert e.value.code == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LbmError) as e:
        S.set_params(W.cavity(8, 1e4).replace(bc_flow=(0, 1, 1, 1)))
    assert e.value.code == lbm.LBM_ERR_ARG
    S.set_params(W.cavity(8, 1e4))
    with pytest.raises(lbm.LbmError) as e:
        S.nusselt(W.TOP)
    assert e.value.code == lbm.LBM_ERR_ARG
    d = S.derived()
    o = oracle.derive(W.cavity(8, 1e4))
    assert np.allclose(d["s"], o["s"], rtol=1e-15) and np.allclose(d["q"], o["q"], rtol=1e-15)
    assert abs(d["gbeta"] - o["gbeta"]) < 1e-18
    S.close()


@pytest.mark.parametrize("which", ["cavity2048", "rb4096x1024"])
def test_parity_full_size_in_bench_launch(which):
    """Full-size lattices in the default launch shape that the benchmark
    times: two steps from a non-uniform temperature, every population."""
    if which == "cavity2048":
        pb = W.workload_cavity2048()
        T = W.random_temperature(pb.nx, pb.ny, 0.0, 1.0, seed=21)
    else:
        pb = W.workload_rb4096x1024()
        T = W.rb_initial_temperature(pb.nx, pb.ny)
    S, L = run_pair(pb, 2, T_init=T)
    fa, ga = S.get_populations()
    fb, gb = L.get_state()
    ef, eg = max_rel_pop_error(pb, fa, ga, fb, gb)
    assert ef < TOL and eg < TOL, (ef, eg)
    S.close()


def test_graph_replays_match_eager_launches():
    """lbm_step in captured graphs of 8 sweeps: every replay, with eager
    work and synchronizations between replays, matches the one-launch-per-
    step path bitwise (and an odd tail of plain launches is handled)."""
    pb = W.cavity(48, 1e5, ny=40)
    T = W.random_temperature(48, 40, 0.0, 1.0, seed=31)
    eager = lbm.Solver(48, 40, "f64")
    eager.set_params(pb)
    eager.set_graph_steps(0)
    eager.init_temperature(T)
    graph = lbm.Solver(48, 40, "f64")
    graph.set_params(pb)
    graph.set_graph_steps(8)
    graph.init_temperature(T)
    assert graph.get_graph_steps() == 8
    for rep in range(5):
        n = 8 * (rep + 1) + (rep % 2) * 3        # graphs plus a plain tail
        eager.step(n)
        graph.step(n)
        graph.moments()                           # eager work between replays
        fa, ga = eager.get_populations()
        fb, gb = graph.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), rep
        assert graph.time == eager.time
    # parameters change: the graph must be rebuilt, not replayed stale
    pb2 = pb.replace(ra=3e4)
    eager.set_params(pb2); graph.set_params(pb2)
    eager.step(16); graph.step(16)
    assert np.array_equal(eager.get_populations()[0], graph.get_populations()[0])
    with pytest.raises(lbm.LbmError):
        graph.set_graph_steps(7)
    eager.close(); graph.close()


def test_buffers_above_4gib_match_the_buffer_path():
    """A population buffer of 4 GiB or more is addressed with 64-bit
    pointers and steps singly; a buffer below 4 GiB uses buffer descriptors
    and, for FP64, four steps per launch.  An x-periodic Rayleigh-Benard cell 6208
    wide (4.3 GB per buffer) whose initial temperature repeats every 64
    columns must equal, column for column and bitwise, the 64-wide cell."""
    ny, nx_big, reps = 6208, 6208, 97
    assert lbm.lbm_required_bytes(nx_big, ny, lbm.LBM_F64, lbm.LBM_MODEL_D2Q5) // 2 >= 1 << 32
    rng = np.random.default_rng(1510)
    T = 0.5 + 0.1 * rng.uniform(-1, 1, (ny, 64))
    out = []
    for nx in (64, nx_big):
        pb = W.rayleigh_benard(nx, ny, 1e5)
        S = lbm.Solver(nx, ny, "f64")
        S.set_params(pb)
        S.init_temperature(np.tile(T, (1, nx // 64)))
        assert S.steps_per_launch == (4 if nx == 64 else 1)
        S.step(5)
        out.append(S.get_populations())
        S.close()
    (fs, gs), (fb, gb) = out
    for k in range(reps):
        sl = slice(64 * k, 64 * (k + 1))
        assert np.array_equal(fb[:, :, sl], fs) and np.array_equal(gb[:, :, sl], gs), k


def test_profile_trace(capfd, monkeypatch):
    """LBM_PROFILE set at create: lbm_destroy reports the traced calls."""
    import json
    pb = W.cavity(64, 1e4)
    monkeypatch.setenv("LBM_PROFILE", "1")
    S = lbm.Solver(64, 64, "f64")
    monkeypatch.delenv("LBM_PROFILE")
    S.set_params(pb)
    S.step(100)          # a captured graph of 64 steps and a tail of 36
    S.step(7)
    # four steps per launch (FP64): the graph holds 16, the tail 9, the
    # call of 7 one, a pair and a single step
    S.step(0)
    S.close()
    lines = [l for l in capfd.readouterr().err.splitlines() if l.startswith('{"lbm_profile"')]
    assert len(lines) == 1
    rec = json.loads(lines[0])["lbm_profile"]
    assert rec["nx"] == 64 and rec["ny"] == 64 and rec["storage"] == "f64"
    assert rec["calls"] == 2 and rec["steps"] == 107
    assert rec["launches"] == 16 + 9 + 3 and rec["gpu_ms"] > 0 and rec["mlups"] > 0
    S2 = lbm.Solver(64, 64, "f64")     # not traced
    S2.set_params(pb)
    S2.step(10)
    S2.close()
    assert '"lbm_profile"' not in capfd.readouterr().err
