"""Pins for the oracle's parameter map (Eq. 40 and the definitions of
viscosity and diffusivity after Eqs. 20 and 29) and its Nusselt stencil
(Eq. 39 and the local definition before it)."""
import math

import numpy as np
import pytest

import oracle
from paper_1510_08224_amd import workloads as W


@pytest.mark.parametrize("ra,pr,n", [(1e3, 0.71, 64), (1e4, 0.71, 64), (1e6, 0.71, 2048),
                                     (1e5, 7.0, 128), (1e5, 0.71, 1024)])
def test_eq40_reproduces_ra_and_pr(ra, pr, n):
    d = oracle.derive(W.cavity(n, ra, pr, 0.1))
    nu, alpha = d["nu"], d["alpha"]
    # Pr = nu/alpha and Ra = g beta dT L^3/(nu alpha), with u_c^2 = g beta dT L
    assert abs(nu / alpha / pr - 1) < 1e-13
    assert abs(d["gbeta"] * d["dT"] * d["length"] ** 3 / (nu * alpha) / ra - 1) < 1e-12
    assert abs(math.sqrt(d["gbeta"] * d["dT"] * d["length"]) - 0.1) < 1e-15
    assert 0 < d["s_nu"] < 2 and 0 < d["zeta_alpha"] < 2


def test_eq40_uses_varpi_through_csT2():
    pb = W.cavity(64, 1e4)
    for varpi in (0.3, 0.5, 0.7):
        d = oracle.derive(pb.replace(varpi=varpi))
        assert abs(d["nu"] / d["alpha"] / 0.71 - 1) < 1e-13


@pytest.mark.parametrize("side", [W.LEFT, W.RIGHT, W.BOTTOM, W.TOP])
def test_nusselt_stencil_exact_for_quadratic_profile(side):
    # T = Tw + a d + b d^2, d the distance from the wall: the half-cell
    # one-sided stencil recovers dT/dn = a exactly.
    nx, ny = 7, 9
    pb = W.cavity(nx, 1e4, ny=ny).replace(
        bc_temp=(W.TEMP_DIRICHLET,) * 4, wall_T=(0.9, 0.1, 0.7, 0.2), t_hot=0.9, t_cold=0.1)
    tw, a, b = pb.wall_T[side], 0.013, -0.0021
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    d = {W.LEFT: xx + 0.5, W.RIGHT: nx - 0.5 - xx, W.BOTTOM: yy + 0.5, W.TOP: ny - 0.5 - yy}[side]
    T = tw + a * d + b * d * d
    L = oracle.Lattice(pb, T_init=T)
    mean, mx, imax, loc = L.nusselt(side, local=True)
    length, dT = L.derived["length"], L.derived["dT"]
    sign = 1.0 if side in (W.LEFT, W.BOTTOM) else -1.0
    expect = -length * sign * a / dT
    assert np.allclose(loc, expect, rtol=1e-12, atol=0)
    assert abs(mean - expect) < 1e-12 * abs(expect)
