"""Pins of the oracle against the paper's closed forms and printed results.

* Channel with a moving, injecting wall (Sec. 3.3): the steady profiles of
  Eqs. 36-37 are reached with second-order global errors (Eqs. 35, 38) at
  Re = 10, s_nu = 0.8, Pr = 0.71 (the paper states slopes 1.9670 and
  1.9948 for its wall scheme).
* Body-force channel (Sec. 3.1): the parabola of Eq. 34 with second-order
  error (stated slopes 1.9889-1.9912).
* Natural convection in the square cavity (Sec. 3.4, Table 3): mean and
  maximum wall Nusselt numbers and the velocity extrema at steady state.
  The paper's walls use non-equilibrium extrapolation and Ma = 0.1 on finer
  lattices, so these are loose physics checks (Table 3 itself spreads by
  about 1% across its sources).
"""
import math

import numpy as np
import pytest

import oracle
from golden_io import paper_tables
from paper_1510_08224_amd import workloads as W

CS2 = 1.0 / 3.0


def _steady(L, chunk, tol, cap):
    prev, n = None, 0
    while n < cap:
        L.step(chunk)
        n += chunk
        cur = L.moments()[1:]
        if prev is not None and oracle.residual(prev, cur) < tol:
            return n
        prev = cur
    raise AssertionError("no steady state")


def _slope(h, e):
    return float(np.polyfit(np.log(h), np.log(e), 1)[0])


def _injection_errors(H):
    s_nu, re, pr = 0.8, 10.0, 0.71
    nu = CS2 * (1 / s_nu - 0.5)
    v0 = re * nu / H
    u0 = v0
    za = 1 / (0.5 + CS2 * (1 / s_nu - 0.5) / (0.25 * pr))   # Sec. 3.3 rate map, c_sT^2 = 1/4
    pb = W.channel(1, H, s_nu=s_nu, zeta_alpha=za, u_top=(u0, v0), u_bottom=(0.0, v0),
                   t_bottom=0.0, t_top=1.0, rates_one=True)
    L = oracle.Lattice(pb)
    _steady(L, 2000, 1e-13, 400000)
    _, ux, uy, T = L.moments()
    y = np.arange(H) + 0.5
    ua = oracle.porous_plate_u(y, u0, re, H)
    ta = oracle.porous_plate_T(y, 0.0, 1.0, pr, re, H)
    return (oracle.error_u(ua, np.full(H, v0), ux[:, 0], uy[:, 0]),
            oracle.error_T(ta, T[:, 0]))


def test_injection_channel_second_order():
    hs = [30, 60, 90]
    errs = [_injection_errors(H) for H in hs]
    su = _slope(1 / np.array(hs), [e[0] for e in errs])
    st = _slope(1 / np.array(hs), [e[1] for e in errs])
    stated = {r[0]: float(r[1]) for r in paper_tables()["slopes"]}
    assert 1.8 < su < 2.2 and 1.8 < st < 2.2
    assert abs(su - stated["injection_u"]) < 0.1 and abs(st - stated["injection_T"]) < 0.1
    assert errs[0][0] < 2e-3 and errs[0][1] < 1e-2


def _poiseuille_error(H, s_nu, re=49.4146):
    nu = CS2 * (1 / s_nu - 0.5)
    lc = H / 2
    ax = 2 * re * nu ** 2 / lc ** 3          # Re = u0 lc / nu, u0 = ax lc^2 / (2 nu)
    u0 = ax * lc ** 2 / (2 * nu)
    L = oracle.Lattice(W.channel(1, H, s_nu=s_nu, zeta_alpha=1.0, ax=ax, rates_one=True))
    _steady(L, 5000, 1e-10 * u0, 2000000)
    _, ux, uy, _ = L.moments()
    y = np.arange(H) + 0.5 - H / 2
    return oracle.error_u(oracle.poiseuille_profile(y, u0, lc), np.zeros(H), ux[:, 0], uy[:, 0])


def test_body_force_channel_second_order():
    hs = [20, 40, 60]
    e = [_poiseuille_error(H, 1.6) for H in hs]
    s = _slope(1 / np.array(hs), e)
    stated = {r[0]: float(r[1]) for r in paper_tables()["slopes"]}
    assert abs(s - stated["channel_1.60"]) < 0.1


def _table3_row(ra):
    for r in paper_tables()["table3"]:
        if float(r[0]) == ra:
            return [float(v) for v in r]
    raise KeyError(ra)


def _cavity_steady(n, ra, u_c=0.1):
    pb = W.cavity(n, ra, 0.71, u_c)
    L = oracle.Lattice(pb)
    _steady(L, 1000, 1e-9, 200000)
    return L


def _extrema(L):
    """u_x,max on the vertical midplane and u_y,max on the horizontal one,
    scaled by alpha/L, with positions scaled by L (Table 3 conventions)."""
    n = L.nx
    _, ux, uy, _ = L.moments()
    a = L.derived["alpha"]
    col = 0.5 * (ux[:, n // 2 - 1] + ux[:, n // 2]) if n % 2 == 0 else ux[:, n // 2]
    row = 0.5 * (uy[n // 2 - 1, :] + uy[n // 2, :]) if n % 2 == 0 else uy[n // 2, :]
    j, i = int(np.argmax(col)), int(np.argmax(row))
    return col[j] * n / a, (j + 0.5) / n, row[i] * n / a, (i + 0.5) / n


def test_table3_ra1e3_coarse():
    ra, _, uxm, ym, uym, xm, numax, ynu, numean = _table3_row(1e3)
    L = _cavity_steady(32, ra)
    mean, mx, imax = L.nusselt(W.RIGHT)
    assert abs(mean / numean - 1) < 0.005
    assert abs(mx / numax - 1) < 0.01
    u, yu, v, xv = _extrema(L)
    assert abs(u / uxm - 1) < 0.02 and abs(v / uym - 1) < 0.02


def test_table3_ra1e4():
    ra, _, uxm, ym, uym, xm, numax, ynu, numean = _table3_row(1e4)
    L = _cavity_steady(64, ra)
    mean, mx, imax = L.nusselt(W.RIGHT)
    assert abs(mean / numean - 1) < 0.002
    assert abs(mx / numax - 1) < 0.005
    assert abs((imax + 0.5) / 64 - ynu) < 1.5 / 64
    # both walls carry the same heat at steady state
    assert abs(L.nusselt(W.LEFT)[0] / mean - 1) < 1e-4
    u, yu, v, xv = _extrema(L)
    assert abs(u / uxm - 1) < 0.02 and abs(v / uym - 1) < 0.02
    assert abs(yu - ym) < 1.5 / 64 and abs(xv - xm) < 1.5 / 64
