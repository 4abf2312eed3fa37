"""Pins for the oracle's time stepping: conservation laws, exact solutions
that link-wise walls reproduce to round-off, and symmetries.

* Mass: collision conserves m_0 (Eq. 8 with m_0^eq = rho); streaming and
  bounce-back permute populations, so sum(rho) is constant.
* Heat: T = n_0 is conserved by Eq. 24; with adiabatic walls the sum of T
  is constant, and with Dirichlet walls it changes by exactly the
  anti-bounce-back link fluxes.
* Momentum: in a periodic box under a constant force the total momentum
  grows by N rho0 F per step (Eqs. 8, 15, 19).
* Rest state, plane Couette flow and pure conduction are exact.
* Centro-symmetry of the heated cavity (with T0 = 0); x-mirror symmetry of a
  Rayleigh-Benard cell (which the printed S~_8 breaks).
"""
import numpy as np
import pytest

import oracle
from paper_1510_08224_amd import workloads as W


def test_mass_conserved_in_cavity():
    L = oracle.Lattice(W.cavity(24, 1e4))
    r0 = L.moments()[0].sum()
    L.step(1500)
    r1 = L.moments()[0].sum()
    assert abs(r1 - r0) / r0 < 1e-13


def test_heat_conserved_with_adiabatic_walls():
    pb = W.cavity(20, 1e4).replace(bc_temp=(W.TEMP_ADIABATIC,) * 4)
    T0 = W.random_temperature(20, 20, 0.0, 1.0, seed=5)
    L = oracle.Lattice(pb, T_init=T0)
    s0 = L.moments()[3].sum()
    L.step(800)
    s1 = L.moments()[3].sum()
    assert abs(s1 - s0) / abs(s0) < 1e-13


def test_heat_balance_with_dirichlet_walls():
    # One step: sum T(t+1) - sum T(t) = sum over Dirichlet wall links of
    # (varpi T_w / 2 - 2 g*_i), the anti-bounce-back exchange.
    pb = W.cavity(12, 1e4)
    L = oracle.Lattice(pb, T_init=W.random_temperature(12, 12, 0.0, 1.0, seed=2))
    L.step(3)
    s0 = L.moments()[3].sum()
    _, gp = L.post_collision()
    # left wall: links leaving through x = -1/2 carry direction 3; right: direction 1
    flux = (0.5 * 0.5 * 1.0 - 2 * gp[3, :, 0]).sum() + (0.5 * 0.5 * 0.0 - 2 * gp[1, :, -1]).sum()
    L.step(1)
    s1 = L.moments()[3].sum()
    assert abs((s1 - s0) - flux) < 1e-13


def test_momentum_growth_in_periodic_box():
    pb = W.periodic_box(6, 5, s_nu=1.2, zeta_alpha=1.0, ax=1e-4, ay=-3e-5)
    L = oracle.Lattice(pb, T_init=W.random_temperature(6, 5, 0.0, 1.0, seed=1))
    _, ux0, uy0, _ = L.moments()
    L.step(10)
    _, ux1, uy1, _ = L.moments()
    n = 30
    assert abs((ux1.sum() - ux0.sum()) - 10 * n * 1e-4) < 1e-14
    assert abs((uy1.sum() - uy0.sum()) + 10 * n * 3e-5) < 1e-14


def test_rest_state_is_fixed_point():
    pb = W.cavity(10, 1e4, t_hot=0.5, t_cold=0.5)
    L = oracle.Lattice(pb)
    f0, g0 = L.get_state()
    L.step(200)
    f1, g1 = L.get_state()
    assert np.max(np.abs(f1 - f0)) < 1e-15
    assert np.max(np.abs(g1 - g0)) < 1e-15


def test_plane_couette_is_exact():
    n = 16
    pb = W.channel(3, n, s_nu=1.3, zeta_alpha=1.1, u_top=(0.05, 0.0), t_bottom=0.0, t_top=1.0)
    L = oracle.Lattice(pb)
    L.step(12000)
    _, ux, uy, T = L.moments()
    y = (np.arange(n) + 0.5) / n
    assert np.max(np.abs(ux - 0.05 * y[:, None])) < 1e-13
    assert np.max(np.abs(uy)) < 1e-13
    assert np.max(np.abs(T - y[:, None])) < 1e-13


def test_conduction_is_exact_and_nusselt_is_one():
    n = 16
    pb = W.cavity(n, 1e4).replace(u_c=0.0, s_nu=1.2, zeta_alpha=1.3)
    L = oracle.Lattice(pb)
    L.step(12000)
    _, ux, uy, T = L.moments()
    x = (np.arange(n) + 0.5) / n
    assert np.max(np.abs(T - (1 - x)[None, :])) < 1e-13
    assert np.max(np.abs(ux)) == 0.0 and np.max(np.abs(uy)) == 0.0
    for side in (W.LEFT, W.RIGHT):
        mean, mx, _ = L.nusselt(side)
        assert abs(mean - 1) < 1e-12 and abs(mx - 1) < 1e-12


def test_cavity_centro_symmetry():
    # The map (i, j) -> (N-1-i, N-1-j), u -> -u, T -> -T is a symmetry of the
    # discrete scheme when T0 = 0 (then every equilibrium and the force are
    # odd or even as needed).  With T0 != 0 the map is affine in T and the
    # n_1^eq = u_x T flux makes it hold only as far as the lattice velocity
    # is divergence-free, so T_h = -T_c here.
    pb = W.cavity(18, 1e5, t_hot=0.5, t_cold=-0.5)
    L = oracle.Lattice(pb)
    L.step(400)
    _, ux, uy, T = L.moments()
    r = lambda a: a[::-1, ::-1]
    assert np.max(np.abs(ux)) > 1e-3
    assert np.max(np.abs(ux + r(ux))) < 1e-14
    assert np.max(np.abs(uy + r(uy))) < 1e-14
    assert np.max(np.abs(T + r(T))) < 1e-14


@pytest.mark.parametrize("literal", [False, True])
def test_rb_mirror_symmetry_and_printed_s8(literal):
    nx, ny = 16, 8
    pb = W.rayleigh_benard(nx, ny, 5e4)
    T = W.rb_initial_temperature(nx, ny, amp=1e-2, seed=9)
    T = 0.5 * (T + T[:, ::-1])              # mirror-symmetric start
    L = oracle.Lattice(pb, s8_literal=literal, T_init=T)
    L.step(300)
    _, ux, uy, T1 = L.moments()
    asym = max(np.max(np.abs(ux + ux[:, ::-1])), np.max(np.abs(uy - uy[:, ::-1])),
               np.max(np.abs(T1 - T1[:, ::-1])))
    if literal:
        assert asym > 1e-12       # the printed S~_8 is odd under the mirror
    else:
        assert asym < 1e-14
