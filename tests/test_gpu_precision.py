"""FP32 and FP16 deviation storage against the FP64 oracle.

Populations are stored as deviations from the rest equilibrium (w_i rho0
for fbar, g_i^eq(T0, 0) for g) and collided in FP32; conserved sums are
accumulated in FP64.  The bounds below are the stated error bounds of the
two storage modes on the 64 x 64 cavity (Ra = 1e4, Pr = 0.71, u_c = 0.1),
relative to u_c for velocity, to dT for temperature and to Nu itself."""
import numpy as np
import pytest

import oracle
from gpu_util import run_pair
from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W

pytestmark = pytest.mark.gpu

BOUNDS = {  # storage: (velocity / u_c, temperature / dT, relative Nu)
    "f32": (2e-6, 2e-6, 2e-6),
    "f16": (2e-2, 1e-2, 2e-2),
}


def _errors(S, L, pb):
    mg, mo = S.moments(), L.moments()
    du = np.max(np.hypot(mg[1] - mo[1], mg[2] - mo[2])) / pb.u_c
    dT = np.max(np.abs(mg[3] - mo[3])) / (pb.t_hot - pb.t_cold)
    nu_g, nu_o = S.nusselt(W.LEFT)[0], L.nusselt(W.LEFT)[0]
    return du, dT, abs(nu_g - nu_o) / abs(nu_o)


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("steps", [1000, 20000])
def test_deviation_storage_error_bounds(storage, steps):
    pb = W.workload_cavity64()
    S, L = run_pair(pb, steps, storage=storage)
    du, dT, dnu = _errors(S, L, pb)
    print(f"{storage} {steps} steps: max|du|/u_c {du:.3e}  max|dT|/dT {dT:.3e}  |dNu|/Nu {dnu:.3e}")
    bu, bt, bn = BOUNDS[storage]
    assert du < bu and dT < bt and dnu < bn
    S.close()


@pytest.mark.parametrize("storage,tol", [("f32", 1e-7), ("f16", 2e-3)])
def test_deviation_storage_roundtrip(storage, tol):
    # populations near rest: the stored deviation keeps about 24 (FP32) or
    # 11 (FP16) significant bits of the deviation, not of the population.
    # FP32 deviations are from the rest state at T0; FP16 ones from the rest
    # state at the conduction profile between the Dirichlet walls (here
    # left T = 1, right T = 0: T_ref = 1 - (x + 1/2) / nx).
    pb = W.cavity(20, 1e4, ny=12)
    S = lbm.Solver(20, 12, storage)
    S.set_params(pb)
    L = oracle.Lattice(pb, T_init=W.random_temperature(20, 12, 0.2, 0.8, seed=3))
    L.step(30)
    f, g = L.get_state()
    S.set_populations(f, g)
    fb, gb = S.get_populations()
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    tref = 0.5 if storage == "f32" else (1.0 - (np.arange(20) + 0.5) / 20)[None, None, :]
    grest = np.array([0.5] + [0.125] * 4)[:, None, None] * tref
    assert np.max(np.abs(fb - f) / np.maximum(np.abs(f - w), 1e-6)) < tol * 4
    assert np.max(np.abs(gb - g) / np.maximum(np.abs(g - grest), 1e-6)) < tol * 4
    S.close()


def test_fp16_scale_keeps_small_deviations_normal():
    # a deviation of 1e-6 in a population is far below FP16's normal range
    # (6.1e-5) unscaled; the power-of-two scale keeps it representable
    pb = W.cavity(16, 1e4, ny=8)
    L = oracle.Lattice(pb)
    f, g = L.get_state()
    f = f.copy()
    f[1] += 1e-6
    S = lbm.Solver(16, 8, "f16")
    S.set_params(pb)
    S.set_populations(f, g)
    fb, _ = S.get_populations()
    assert abs((fb[1] - 1 / 9).mean() - 1e-6) < 2e-8
    S.close()
