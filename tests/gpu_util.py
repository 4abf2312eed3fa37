"""Helpers shared by the GPU tests: run the same seeded problem through the
HIP library (via the C ABI binding) and through the CPU oracle, and compare
element by element."""
import numpy as np

import oracle
from paper_1510_08224_amd import lbm
from paper_1510_08224_amd import workloads as W

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def population_scale(pb, ng=5):
    """Reference magnitudes for the relative comparison of populations:
    max(|p_oracle|, p_ref) with p_ref = w_i for fbar and the rest
    equilibrium of the temperature model (D2Q5: (1 - varpi) T, varpi T / 4;
    D2Q9: w_i T) at the largest wall/reference temperature for g."""
    tmax = max(abs(pb.t_hot), abs(pb.t_cold), *(abs(t) for t in pb.wall_T), 1e-300)
    if ng == 9:
        gref = W9 * tmax
    else:
        gref = np.array([(1 - pb.varpi) * tmax] + [pb.varpi * tmax / 4] * 4)[:ng]
    return W9[:, None, None], gref[:, None, None]


def max_rel_pop_error(pb, fa, ga, fb, gb):
    ng = ga.shape[0]
    fr, gr = population_scale(pb, ng)
    ef = np.max(np.abs(fa - fb) / np.maximum(np.abs(fb), fr))
    eg = float(np.max(np.abs(ga - gb) / np.maximum(np.abs(gb), gr))) if ng else 0.0
    return float(ef), eg


def run_pair(pb, steps, storage="f64", T_init=None, pops=None, launch=None, s8_literal=False,
             model="d2q5"):
    """Advance the GPU solver and the oracle from the same initial state.
    Returns (solver, oracle lattice) after `steps` steps."""
    S = lbm.Solver(pb.nx, pb.ny, storage, model=model)
    S.set_params(pb)
    if launch:
        S.set_launch(*launch)
    L = oracle.Lattice(pb, s8_literal=s8_literal, T_init=T_init, model=model)
    if T_init is not None:
        S.init_temperature(T_init)
    if pops is not None:
        S.set_populations(*pops)
        L.set_state(*pops)
    S.step(steps)
    L.step(steps)
    return S, L


def field_scale(pb):
    """Scales for velocity and temperature comparisons."""
    u = max(pb.u_c, *(abs(v) for w in pb.wall_u for v in w), 1e-3)
    t = max(abs(pb.t_hot - pb.t_cold), 1e-3)
    return u, t
