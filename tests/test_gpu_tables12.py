"""The body-force channel of Tables 1-2 (Sec. 3.1) on the GPU, FP64.

* At steady state the GPU channel (delta_x = 1/60, s_nu = 1.754, walls by
  non-equilibrium extrapolation) equals the oracle's, population by
  population.
* The Table 2 entries at delta_x = 1/120 and 1/150, too slow for the
  oracle in the CPU suite, come from the GPU path (whose FP64 parity with
  the oracle the other tests pin) and sit in the same bands as the oracle's
  at coarser spacings (tests/test_oracle_tables12.py): a factor 1.05-1.16
  over the printed value in the form of Eq. 35, 1.00-1.06 in the global
  L2 form, the same at both spacings, second order between them."""
import numpy as np
import pytest

import oracle
from golden_io import paper_tables
from paper_1510_08224_amd import lbm
from tables12_util import channel_case, errors, start_state

pytestmark = pytest.mark.gpu


def _gpu_steady(Ny, s_nu, ax=None, tol=1e-12):
    pb, u0, lc, ua = channel_case(Ny, s_nu, ax)
    S = lbm.Solver(pb.nx, pb.ny, "f64")
    S.set_params(pb)
    _, g0 = S.get_populations()
    S.set_populations(start_state(ua), g0)
    prev, n = None, 0
    while n < 20_000_000:
        S.step(5000)
        n += 5000
        cur = S.moments()[1][:, 0].copy()
        if prev is not None and np.max(np.abs(cur - prev)) < tol * u0:
            break
        prev = cur
    return S, ua, n


def test_steady_channel_equals_the_oracle():
    S, ua, n = _gpu_steady(60, 1.754)
    f, _ = S.get_populations()
    S.close()
    pb, u0, _, _ = channel_case(60, 1.754)
    L = oracle.Lattice(pb)
    _, g0 = L.get_state()
    L.set_state(start_state(ua), g0)
    L.step(n)
    fo, _ = L.get_state()
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    assert np.max(np.abs(f - fo) / w) < 1e-11


def test_table2_finest_spacings():
    table2 = {float(r[0]): [float(v) for v in r[1:]] for r in paper_tables()["table2"]}
    for s in (1.60, 1.754, 1.90):
        e = {}
        for k, N in ((3, 120), (4, 150)):
            S, ua, _ = _gpu_steady(N, s, tol=1e-11)
            _, ux, uy, _ = S.moments()
            S.close()
            e35, el2 = errors(ua, ux[:, 0], uy[:, 0])
            ref = table2[s][k]
            assert 1.05 < e35 / ref < 1.16 and 1.0 < el2 / ref < 1.06, (s, N, e35 / ref, el2 / ref)
            e[N] = (e35, ref)
        r120, r150 = e[120][0] / e[120][1], e[150][0] / e[150][1]
        assert max(r120, r150) / min(r120, r150) < 1.015, (s, r120, r150)
        slope = np.log(e[120][0] / e[150][0]) / np.log(150 / 120)
        ref_slope = np.log(e[120][1] / e[150][1]) / np.log(150 / 120)
        assert abs(slope - ref_slope) < 0.05, (s, slope, ref_slope)
