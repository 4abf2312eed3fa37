"""Pins for the oracle's single-node collision.

* Exact rational reference (tests/exact_ref.py): the velocity-space update
  of Eq. 7 / Eq. 23 with Lambda~ = M^-1 Lambda M built from the basis
  definitions, f^eq of Eq. 22, g^eq of Eq. 30 and the Guo source S whose
  moments Eq. 10 defines.  The oracle instead relaxes in moment space with
  the printed Eqs. 8, 16, 17, 24, 28 and the printed M, M^-1, N, N^-1.
* BGK special case: with every rate equal the MRT collision is the
  textbook BGK update with Guo forcing (Eq. 7 with Lambda~ = omega I).
* The printed S~_8 (Eq. 17) differs from M S for the Guo source; the
  reading that replaces it is checked here and its switch is exercised.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import exact_ref as X


def _params(s, q, varpi=0.5, gbeta=0.0, T0=0.5, ax=0.0, ay=0.0, s8_literal=False):
    p = oracle.OrcParams()
    p.nx = p.ny = 1
    for k in range(9):
        p.s[k] = s[k]
    for k in range(5):
        p.q[k] = q[k]
    p.varpi, p.rho0, p.gbeta, p.T0, p.ax, p.ay = varpi, 1.0, gbeta, T0, ax, ay
    for k in range(4):
        p.bc_flow[k] = 0
        p.bc_temp[k] = 0
    p.s8_literal = 1 if s8_literal else 0
    return p


def _rand_state(rng, far=False):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    spread = 0.5 if far else 0.05
    f = w * (1 + spread * rng.uniform(-1, 1, 9))
    T = rng.uniform(0.2, 1.5)
    g = np.array([0.5 * T] + [0.125 * T] * 4) * (1 + spread * rng.uniform(-1, 1, 5))
    return f, g


def _exact(p, f, g):
    s = [Fr(v) for v in p.s]
    q = [Fr(v) for v in p.q[:5]]
    fo, go = X.collide([Fr(v) for v in f], [Fr(v) for v in g], s, q, Fr(p.varpi),
                       Fr(p.gbeta), Fr(p.T0), Fr(p.ax), Fr(p.ay))
    return np.array([float(v) for v in fo]), np.array([float(v) for v in go])


@pytest.mark.parametrize("seed", range(12))
def test_collision_matches_exact_eq7(seed):
    rng = np.random.default_rng(seed)
    s_nu, s_e, s_q, s_eps = rng.uniform(0.3, 1.95, 4)
    z_a, z_e, z_nu = rng.uniform(0.3, 1.95, 3)
    p = _params([1, 1, 1, s_e, s_nu, s_nu, s_q, s_q, s_eps], [1, z_a, z_a, z_e, z_nu],
                varpi=rng.uniform(0.2, 0.8), gbeta=rng.uniform(-0.05, 0.05),
                T0=rng.uniform(0.2, 1.0), ax=rng.uniform(-1e-2, 1e-2), ay=rng.uniform(-1e-2, 1e-2))
    f, g = _rand_state(rng, far=bool(seed % 2))
    fo, go = oracle.collide_node(p, f, g)
    fe, ge = _exact(p, f, g)
    assert np.max(np.abs(fo - fe)) <= 1e-15 * 8
    assert np.max(np.abs(go - ge)) <= 1e-15 * 8


def test_bgk_special_case():
    # All rates omega: fbar* = fbar - omega (fbar - f^eq) + (1 - omega/2) S (textbook BGK, Guo forcing)
    rng = np.random.default_rng(7)
    om = 1.37
    p = _params([om] * 9, [om] * 5, gbeta=0.02, T0=0.4, ax=3e-3, ay=-2e-3)
    f, g = _rand_state(rng, far=True)
    fo, go = oracle.collide_node(p, f, g)
    e = np.array(X.E9, dtype=float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    T = g.sum()
    F = np.array([3e-3, -2e-3 + 0.02 * (T - 0.4)])
    rho = f.sum()
    u = (e.T @ f + F / 2)
    eu = e @ u
    feq = w * (rho + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u @ u))
    S = w * (3 * (e @ F) - 3 * (u @ F) + 9 * eu * (e @ F))
    ref = f - om * (f - feq) + (1 - om / 2) * S
    assert np.max(np.abs(fo - ref)) < 1e-15 * 8
    geq = np.concatenate([[0.5 * T], 0.125 * T + 0.5 * (e[1:5] @ u) * T])
    gref = g - om * (g - geq)
    assert np.max(np.abs(go - gref)) < 1e-15 * 8


def test_printed_s8_is_not_guo_moment_but_reading_is():
    # M S_Guo row 8 = (2/3) rho0 (ux Fx + uy Fy); the printed form pairs ux with Fy.
    ux, uy, Fx, Fy = Fr(3, 100), Fr(-1, 70), Fr(2, 1000), Fr(5, 1000)
    ms = X.guo_moments(ux, uy, Fx, Fy)
    assert ms[8] == Fr(2, 3) * (ux * Fx + uy * Fy)
    assert ms[8] != Fr(2, 3) * (ux * Fy + uy * Fx)
    # rows 0..7 agree with the printed Eq. 17
    assert ms[:8] == [0, Fx, Fy, 2 * (ux * Fx + uy * Fy), 2 * (ux * Fx - uy * Fy),
                      ux * Fy + uy * Fx, Fy / 3, Fx / 3]


def test_literal_s8_switch_changes_only_through_s8():
    rng = np.random.default_rng(3)
    s = [1, 1, 1, 1.6, 1.3, 1.3, 1.2, 1.2, 1.8]
    q = [1, 1.1, 1.1, 1.9, 1.9]
    p0 = _params(s, q, gbeta=0.03, T0=0.5, ax=1e-2)
    p1 = _params(s, q, gbeta=0.03, T0=0.5, ax=1e-2, s8_literal=True)
    f, g = _rand_state(rng, far=True)
    fa, ga = oracle.collide_node(p0, f, g)
    fb, gb = oracle.collide_node(p1, f, g)
    assert np.array_equal(ga, gb)
    d = fb - fa
    assert np.max(np.abs(d)) > 1e-8
    # the difference lies along the last column of M^-1 (the epsilon moment)
    col = np.array([1, -0.5, -0.5, -0.5, -0.5, 0.25, 0.25, 0.25, 0.25])
    k = d[0] / col[0]
    assert np.allclose(d, k * col, atol=1e-16)


def test_momentum_update_is_rho0_F():
    # m_bar_1* - m_bar_1 = rho0 F_x whatever the state (Eqs. 8, 15, 19)
    rng = np.random.default_rng(11)
    p = _params([1, 1, 1, 1.6, 0.9, 0.9, 1.2, 1.2, 1.8], [1, 0.8, 0.8, 1.9, 1.9],
                gbeta=0.01, T0=0.3, ax=4e-3, ay=1e-3)
    for _ in range(5):
        f, g = _rand_state(rng, far=True)
        fo, _ = oracle.collide_node(p, f, g)
        e = np.array(X.E9, dtype=float)
        dj = e.T @ fo - e.T @ f
        Fy = 1e-3 + 0.01 * (g.sum() - 0.3)
        assert np.allclose(dj, [4e-3, Fy], atol=1e-16, rtol=0)
        assert abs(fo.sum() - f.sum()) < 4e-16
