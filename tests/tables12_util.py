"""The body-force channel of Sec. 3.1 (Eq. 34, Tables 1-2) with walls by
non-equilibrium extrapolation through the first and last node rows: Ny
spacings between the plates (Ny + 1 node rows), l_c = Ny / 2, s_nu as
given, every other rate 1, a_x from Re = u0 l_c / nu with u0 = a_x l_c^2 /
(2 nu).  Shared by the oracle test and the GPU test (no method arithmetic
beyond the problem statement and the error norms)."""
import numpy as np

CS2 = 1.0 / 3.0
RE = 49.4146
NEE_Y = dict(bc_flow=(0, 0, 2, 2), bc_temp=(0, 0, 3, 3))


def channel_case(Ny, s_nu, ax=None):
    """(problem, u0, l_c, analytic profile at the node rows)."""
    from paper_1510_08224_amd import workloads as W
    nu = CS2 * (1.0 / s_nu - 0.5)
    lc = Ny / 2.0
    if ax is None:
        ax = 2.0 * RE * nu ** 2 / lc ** 3
    u0 = ax * lc ** 2 / (2.0 * nu)
    pb = W.channel(1, Ny + 1, s_nu=s_nu, zeta_alpha=1.0, ax=ax, rates_one=True).replace(**NEE_Y)
    y = np.arange(Ny + 1) - Ny / 2.0
    ua = u0 * (1.0 - (y / lc) ** 2)          # Eq. 34
    return pb, u0, lc, ua


def start_state(ua):
    """Populations at rest density with the analytic velocity (Eq. 22 at
    rho0 = 1), [i][y][x] for one column: a start near the steady state."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    eu = ex[:, None] * ua[None, :]
    feq = w[:, None] * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * ua[None, :] ** 2)
    return feq[:, :, None].copy()


def errors(ua, ux, uy):
    """Eq. 35 as printed (sum of node-wise 2-norms over the sum of the
    analytic ones) and the global L2 form sqrt(sum |du|^2 / sum |u_A|^2)."""
    e35 = float(np.sum(np.hypot(ua - ux, uy)) / np.sum(np.abs(ua)))
    el2 = float(np.sqrt(np.sum((ua - ux) ** 2 + uy ** 2) / np.sum(ua ** 2)))
    return e35, el2
