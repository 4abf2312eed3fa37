"""Pins for the oracle's comparison operators of Sec. 3.2: the single-
relaxation-time (BGK) collision and the classical MRT with an orthogonal
basis.

* Exact rational references (tests/exact_ref.py): Eq. 7 in velocity space
  with Lambda~ = omega I (BGK) or Lambda~ = M_o^-1 diag(s) M_o with M_o
  built by exact Gram-Schmidt; the oracle instead uses the velocity-space
  BGK formula and a floating-point Gram-Schmidt basis with dense products.
* Special cases: every rate equal makes all three operators the same
  update; the BGK temperature update is the textbook one.
* Invariants: mass, and momentum growing by exactly rho0 F per collision.
* Lattice pins: plane Couette flow is exact with both operators; the body
  force channel converges at second order.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import exact_ref as X
from paper_1510_08224_amd import workloads as W

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
E = np.array(X.E9, dtype=float)


def _params(coll, model=0, s=(1, 1, 1, 1.6, 1.3, 1.3, 1.2, 1.2, 1.8), q=(1, 1.1, 1.1, 1.9, 1.7, 1.7, 1.4, 1.4, 0.9),
            gbeta=0.02, T0=0.4, ax=2e-3, ay=-1e-3, theta=1.0):
    p = oracle.OrcParams()
    p.nx = p.ny = 1
    p.model, p.collision = model, coll
    for k in range(9):
        p.s[k] = s[k]
        p.q[k] = q[k]
    p.varpi, p.theta, p.rho0, p.gbeta, p.T0, p.ax, p.ay = 0.5, theta, 1.0, gbeta, T0, ax, ay
    return p


def _state(rng, ng=5):
    f = W9 * (1 + 0.5 * rng.uniform(-1, 1, 9))
    T = rng.uniform(0.2, 1.5)
    base = np.array([0.5 * T] + [0.125 * T] * 4) if ng == 5 else W9 * T
    return f, base * (1 + 0.5 * rng.uniform(-1, 1, ng))


def _force(p, g):
    T = g.sum() if len(g) else p.T0
    return p.ax, p.ay + p.gbeta * (T - p.T0)


@pytest.mark.parametrize("seed", range(6))
def test_bgk_flow_matches_exact(seed):
    rng = np.random.default_rng(300 + seed)
    w = float(rng.uniform(0.3, 1.95))
    p = _params(oracle.COLL_BGK, s=(1, 1, 1, 1.6, w, w, 1.2, 1.2, 1.8))
    f, g = _state(rng)
    fo, _ = oracle.collide_node(p, f, g)
    Fx, Fy = _force(p, g)
    fe = X.collide_bgk_flow([Fr(v) for v in f], Fr(w), Fr(Fx), Fr(Fy))
    assert np.max(np.abs(fo - np.array([float(v) for v in fe]))) < 8e-16


@pytest.mark.parametrize("model", [0, 1])
def test_bgk_temperature_is_textbook(model):
    rng = np.random.default_rng(7)
    z = 1.17
    p = _params(oracle.COLL_BGK, model=model, q=(1, z, z, 1.9, 1.7, 1.7, 1.4, 1.4, 0.9), theta=1.0)
    ng = 5 if model == 0 else 9
    f, g = _state(rng, ng)
    _, go = oracle.collide_node(p, f, g)
    T = g.sum()
    Fx, Fy = _force(p, g)
    u = E.T @ f + np.array([Fx, Fy]) / 2
    eu = E[:ng] @ u
    if ng == 5:
        geq = np.concatenate([[0.5 * T], 0.125 * T + 0.5 * eu[1:] * T])          # Eq. 30
    else:
        geq = W9 * T * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u @ u))            # Eq. 31
    assert np.max(np.abs(go - (g - z * (g - geq)))) < 8e-16


@pytest.mark.parametrize("seed", range(6))
def test_orthogonal_mrt_matches_exact(seed):
    rng = np.random.default_rng(400 + seed)
    s_e, s_nu, s_q, s_eps = rng.uniform(0.3, 1.95, 4)
    p = _params(oracle.COLL_ORTHO, s=(1, 1, 1, s_e, s_nu, s_nu, s_q, s_q, s_eps))
    f, g = _state(rng)
    fo, go = oracle.collide_node(p, f, g)
    Fx, Fy = _force(p, g)
    # rates along the orthogonal basis: rho, e, eps, jx, qx, jy, qy, pxx, pxy
    so = [Fr(1), Fr(s_e), Fr(s_eps), Fr(1), Fr(s_q), Fr(1), Fr(s_q), Fr(s_nu), Fr(s_nu)]
    fe = X.collide_ortho_flow([Fr(v) for v in f], so, Fr(Fx), Fr(Fy))
    assert np.max(np.abs(fo - np.array([float(v) for v in fe]))) < 2e-15
    # the temperature keeps the model's own MRT
    _, gm = oracle.collide_node(_params(oracle.COLL_MRT, s=(1, 1, 1, s_e, s_nu, s_nu, s_q, s_q, s_eps)), f, g)
    assert np.array_equal(go, gm)


def test_orthogonal_basis_rows_are_the_classical_integer_rows():
    M = np.array([[float(v) for v in r] for r in X.MO9])
    ints = np.array([[1] * 9, [-4, -1, -1, -1, -1, 2, 2, 2, 2], [4, -2, -2, -2, -2, 1, 1, 1, 1],
                     [0, 1, 0, -1, 0, 1, -1, -1, 1], [0, -2, 0, 2, 0, 1, -1, -1, 1],
                     [0, 0, 1, 0, -1, 1, 1, -1, -1], [0, 0, -2, 0, 2, 1, 1, -1, -1],
                     [0, 1, -1, 1, -1, 0, 0, 0, 0], [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=float)
    for a, b in zip(M, ints):
        k = b[np.argmax(np.abs(b))] / a[np.argmax(np.abs(b))]
        assert np.allclose(a * k, b, atol=1e-14)
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)), atol=1e-14)


def test_equal_rates_make_all_operators_one():
    rng = np.random.default_rng(11)
    om = 1.37
    outs = []
    for coll in (oracle.COLL_MRT, oracle.COLL_BGK, oracle.COLL_ORTHO):
        p = _params(coll, s=[om] * 9, q=[om] * 9)
        f, g = _state(np.random.default_rng(11))
        outs.append(oracle.collide_node(p, f, g))
    for fo, go in outs[1:]:
        assert np.max(np.abs(fo - outs[0][0])) < 4e-16
        assert np.max(np.abs(go - outs[0][1])) < 4e-16


@pytest.mark.parametrize("coll", [1, 2])
def test_mass_and_momentum_update(coll):
    rng = np.random.default_rng(13)
    p = _params(coll, s=(1, 1, 1, 1.4, 0.9, 0.9, 1.1, 1.1, 1.6))
    for _ in range(4):
        f, g = _state(rng)
        fo, _ = oracle.collide_node(p, f, g)
        Fx, Fy = _force(p, g)
        assert abs(fo.sum() - f.sum()) < 1e-15
        assert np.allclose(E.T @ fo - E.T @ f, [Fx, Fy], atol=2e-16, rtol=0)


@pytest.mark.parametrize("coll", [1, 2])
def test_couette_exact(coll):
    n = 16
    pb = W.channel(3, n, s_nu=1.3, zeta_alpha=1.1, u_top=(0.05, 0.0)).replace(collision=coll)
    L = oracle.Lattice(pb)
    L.step(12000)
    _, ux, uy, T = L.moments()
    y = (np.arange(n) + 0.5) / n
    assert np.max(np.abs(ux - 0.05 * y[:, None])) < 1e-13
    assert np.max(np.abs(T - y[:, None])) < 1e-13


def _poiseuille_error(H, coll, s_nu=1.6, re=20.0):
    nu = (1 / s_nu - 0.5) / 3
    lc = (H - 1) / 2
    ax = 2 * re * nu ** 2 / lc ** 3          # Re = u0 lc / nu, u0 = ax lc^2 / (2 nu)
    u0 = ax * lc ** 2 / (2 * nu)
    pb = W.with_nee_walls(W.channel(1, H, s_nu=s_nu, zeta_alpha=1.0, ax=ax, rates_one=True)).replace(collision=coll)
    L = oracle.Lattice(pb, model="isothermal")
    prev = None
    for _ in range(400):
        L.step(2000)
        ux = L.moments()[1][:, 0]
        if prev is not None and np.max(np.abs(ux - prev)) < 1e-11 * u0:
            break
        prev = ux
    # NEE walls pass through the first and last node: half-width (H - 1)/2
    y = np.arange(H) - (H - 1) / 2
    ua = oracle.poiseuille_profile(y, ax * ((H - 1) / 2) ** 2 / (2 * nu), (H - 1) / 2)
    return oracle.error_u(ua, np.zeros(H), ux, np.zeros(H))


@pytest.mark.parametrize("coll", [1, 2])
def test_poiseuille_second_order(coll):
    e = [_poiseuille_error(H, coll) for H in (16, 32)]
    slope = np.log(e[0] / e[1]) / np.log(2)
    assert 1.8 < slope < 2.3, (e, slope)
