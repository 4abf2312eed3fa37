"""Batched stepping: many independent lattices advanced by one launch per
step must give every member bitwise the result it has alone, whatever the
mix, the order of members, graph replay, or members joining and leaving;
and a non-finite member must not disturb the others."""
import numpy as np
import pytest

import oracle
from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W

pytestmark = pytest.mark.gpu


def _mix():
    return [
        (W.cavity(64, 1e4), None),
        (W.cavity(96, 3e5, pr=7.0), None),
        (W.cavity(70, 1e5, ny=33), lambda: W.random_temperature(70, 33, 0.0, 1.0, seed=2)),
        (W.rayleigh_benard(128, 40, 5e4), lambda: W.rb_initial_temperature(128, 40, amp=1e-2, seed=1510)),
        (W.channel(65, 24, s_nu=0.9, zeta_alpha=1.1, u_top=(0.03, 0.0)), None),
        (W.cavity(200, 1e6, ny=130), None),
    ]


def _alone(pb, T, storage, steps, launch=None):
    S = lbm.Solver(pb.nx, pb.ny, storage)
    S.set_params(pb)
    if launch:
        S.set_launch(*launch)
    if T is not None:
        S.init_temperature(T)
    S.step(steps)
    out = S.get_populations()
    S.close()
    return out


def _batch(storage, mix, graph=0):
    B = lbm.Batch(storage)
    if graph:
        B.set_graph_steps(graph)
    sols = []
    for pb, mkT in mix:
        S = B.new_solver(pb.nx, pb.ny)
        S.set_params(pb)
        if mkT:
            S.init_temperature(mkT())
        B.add(S)
        sols.append(S)
    return B, sols


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_batch_members_match_alone_bitwise(storage):
    mix = _mix()
    B, sols = _batch(storage, mix)
    B.step(37)
    B.step(26)
    for (pb, mkT), S in zip(mix, sols):
        fa, ga = _alone(pb, mkT() if mkT else None, storage, 63)
        fb, gb = S.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), pb.name
        assert S.time == 63
    B.close()


def test_batch_f64_matches_oracle():
    mix = _mix()[:4]
    B, sols = _batch("f64", mix)
    B.step(120)
    for (pb, mkT), S in zip(mix, sols):
        L = oracle.Lattice(pb, T_init=mkT() if mkT else None)
        L.step(120)
        fo, go = L.get_state()
        fb, gb = S.get_populations()
        assert np.max(np.abs(fb - fo)) < 1e-14 and np.max(np.abs(gb - go)) < 1e-14, pb.name
    B.close()


def test_batch_graph_replay_and_membership_changes():
    mix = _mix()
    B, sols = _batch("f32", mix, graph=16)
    B.step(32)            # two graph replays
    B.step(5)             # plain tail
    slot = 2
    B.remove(slot)        # member 2 leaves after 37 steps
    B.step(20)            # the others go on
    newpb = W.cavity(80, 2e4)
    S_new = B.new_solver(80, 80)
    S_new.set_params(newpb)
    assert B.add(S_new) == slot        # takes the free slot
    B.step(40)
    sols[0].step(3)       # a member stepped on its own
    B.step(16)
    expect = {0: 37 + 20 + 40 + 3 + 16, 1: 113, 3: 113, 4: 113, 5: 113}
    for k, S in enumerate(sols):
        if k == slot:
            continue
        pb, mkT = mix[k]
        fa, ga = _alone(pb, mkT() if mkT else None, "f32", expect[k])
        fb, gb = S.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), k
    fa, ga = _alone(mix[slot][0], mix[slot][1](), "f32", 37)
    fb, gb = sols[slot].get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    fa, ga = _alone(newpb, None, "f32", 56)
    fb, gb = S_new.get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    B.close()


def test_batch_launch_shapes_per_member():
    mix = _mix()
    B, sols = _batch("f32", mix)
    sols[1].set_launch(64, 4, 1)
    sols[5].set_launch(128, 2, 1)
    B.step(30)
    for (pb, mkT), S in zip(mix, sols):
        fa, ga = _alone(pb, mkT() if mkT else None, "f32", 30)
        fb, _ = S.get_populations()
        assert np.array_equal(fa, fb)
    B.close()


def test_nonfinite_member_is_isolated():
    mix = _mix()[:3]
    B, sols = _batch("f32", mix)
    B.step(10)
    f, g = sols[1].get_populations()
    f[0, 5, 5] = np.nan
    sols[1].set_populations(f, g)
    B.step(50)
    r, bad = B.residual()
    assert bad[1] >= 1 and bad[0] == 0 and bad[2] == 0
    for k in (0, 2):
        pb, mkT = mix[k]
        fa, _ = _alone(pb, mkT() if mkT else None, "f32", 60)
        assert np.array_equal(fa, sols[k].get_populations()[0])
    B.close()
