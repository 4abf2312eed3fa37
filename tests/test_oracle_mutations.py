"""The pins must catch plausible mistakes in the oracle.  Each case copies
oracle/orc_lbm.c to a temporary directory, plants one mistake by text
substitution (a dropped term, a wrong sign, a transposed operand, a wrong
index), builds it with the same flags, and runs a quick battery of the
pins from the other oracle tests against the copy.  At least one pin must
fail for every planted mistake; the unmodified copy must pass them all."""
import ctypes
import os
import shutil
import subprocess
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import exact_ref as X
from paper_1510_08224_amd import workloads as W

MUTANTS = {
    "none": None,
    "dropped_half_force": ("jx += 0.5 * p->rho0 * fx;", "jx += 0.0 * p->rho0 * fx;"),
    "minv_sign": ("{1, 0, 0, -1, 0, 0, 0, 0, 1},", "{1, 0, 0, 1, 0, 0, 0, 0, 1},"),
    "m_transposed": ("acc += M9[k][i] * f[i];", "acc += M9[i][k] * f[i];"),
    "s7_wrong_component": ("S[7] = 1.0 / 3.0 * r0 * Fx;", "S[7] = 1.0 / 3.0 * r0 * Fy;"),
    "s8_printed": ("S[8] = p->s8_literal ?", "S[8] = !p->s8_literal ?"),
    "meq3_coefficient": ("meq[3] = 2.0 / 3.0 * rho + r0 * usq;", "meq[3] = 1.0 / 3.0 * rho + r0 * usq;"),
    "neq3_no_varpi": ("neq[3] = p->varpi * T;", "neq[3] = T;"),
    "neq1_wrong_u": ("neq[1] = ux * T;", "neq[1] = uy * T;"),
    "opposite_table": ("{0, 3, 4, 1, 2, 7, 8, 5, 6}", "{0, 3, 4, 1, 2, 8, 7, 6, 5}"),
    "antibounce_sign": ("= -L->gp[c * ng + i] + 2.0 * even;", "= L->gp[c * ng + i] + 2.0 * even;"),
    "moving_wall_sign": ("L->fp[c * 9 + i] - 6.0 * W9[i]", "L->fp[c * 9 + i] + 6.0 * W9[i]"),
    "buoyancy_sign": ("p->ay + p->gbeta * (t - p->T0)", "p->ay - p->gbeta * (t - p->T0)"),
    "nusselt_first_order": ("(9.0 * t[0] - t[1] - 8.0 * tw) / 3.0", "2.0 * (t[0] - tw)"),
    "nee_neq_sign": ("fb[i] = feq_i(p, i, rho, uwx, uwy) + (ff[i] - feq_i(p, i, rho, ux, uy));",
                     "fb[i] = feq_i(p, i, rho, uwx, uwy) - (ff[i] - feq_i(p, i, rho, ux, uy));"),
    "nee_wall_temperature": ("double Tb = tside >= 0 ? p->wall_T[tside] : T;", "double Tb = T;"),
    "nee_wall_velocity": ("double uwx = p->wall_u[vside][0], uwy = p->wall_u[vside][1];",
                          "double uwx = ux, uwy = uy;"),
    "d2q9t_theta_term_sign": ("p->theta * (4.5 * eu * eu - 1.5 * usq));\n    }\n    if (i == 0)",
                              "p->theta * (4.5 * eu * eu + 1.5 * usq));\n    }\n    if (i == 0)"),
    "d2q9t_advection_coefficient": ("(1.0 + 3.0 * eu + p->theta", "(1.0 + 2.0 * eu + p->theta"),
    "d2q9t_rates_reversed": ("ns9[k] = n9[k] - p->q[k] * (n9[k] - ne9[k]);",
                             "ns9[k] = n9[k] - p->q[8 - k] * (n9[k] - ne9[k]);"),
    "d2q9t_antibounce_weight": ("even = W9[i] * p->wall_T[side]", "even = 0.25 * p->wall_T[side]"),
    "d2q9t_antibounce_no_velocity": ("(1.0 + p->theta * (4.5 * eu * eu - 1.5 * usq));\n                    } else",
                                     "(1.0 + 0.0 * (4.5 * eu * eu - 1.5 * usq));\n                    } else"),
    "bgk_source_factor": ("+ (1.0 - 0.5 * w) * guo_i(", "+ (1.0 - w) * guo_i("),
    "guo_velocity_sign": ("(3.0 * (eF - uF) + 9.0 * eu * eF)", "(3.0 * (eF + uF) + 9.0 * eu * eF)"),
    "bgk_thermal_rate": ("const double z = p->q[1];", "const double z = p->q[3];"),
    "ortho_rates_swapped": ("{1.0, p->s[3], p->s[8], 1.0,", "{1.0, p->s[8], p->s[3], 1.0,"),
    "gram_schmidt_sign": ("v[k][i] -= num / den * MO9[j][i];", "v[k][i] += num / den * MO9[j][i];"),
    "stream_index": ("L->fn[((size_t)ty * nx + tx) * 9 + i]", "L->fn[((size_t)ty * nx + tx) * 9 + OPP9[i]]"),
    "nee_nusselt_first_order": ("(-3.0 * t[0] + 4.0 * t[1] - t[2]) / 2.0", "(t[1] - t[0])"),
    "nee_nusselt_midpoint_mean": [("(nee && (k == 0 || k == count - 1)) ? 0.5 * nu : nu", "nu"),
                                  ("nee ? sum / (count - 1) : sum / count", "sum / count")],
    "nee_nusselt_full_end_weights": ("(nee && (k == 0 || k == count - 1)) ? 0.5 * nu : nu",
                                     "(nee && (k == 0 || k == count - 1)) ? 1.0 * nu : nu"),
    "nee_nusselt_one_end_weight": ("(nee && (k == 0 || k == count - 1)) ? 0.5 * nu : nu",
                                   "(nee && k == 0) ? 0.5 * nu : nu"),
    "nee_nusselt_divisor": ("nee ? sum / (count - 1) : sum / count", "sum / count"),
}


def _build(tmp, name, mut):
    src = open(oracle._SRC).read()
    for old, new in ([] if mut is None else ([mut] if isinstance(mut, tuple) else mut)):
        assert src.count(old) >= 1, name
        src = src.replace(old, new, 1)
    c = os.path.join(tmp, f"{name}.c")
    so = os.path.join(tmp, f"lib{name}.so")
    open(c, "w").write(src)
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, c, "-lm"],
                   check=True)
    return oracle.load(so)


def _p(lib_s, s, q, **kw):
    p = oracle.OrcParams()
    p.nx = p.ny = 1
    for k in range(9):
        p.s[k] = s[k]
    for k in range(len(q)):
        p.q[k] = q[k]
    p.varpi, p.rho0 = kw.get("varpi", 0.5), 1.0
    p.gbeta, p.T0, p.ax, p.ay = kw.get("gbeta", 0.0), kw.get("T0", 0.5), kw.get("ax", 0.0), kw.get("ay", 0.0)
    return p


def _battery(lib):
    """Return the names of the pins that fail for this oracle build."""
    failed = []
    # exact single-node collision (Eq. 7 in rationals)
    rng = np.random.default_rng(0)
    for seed in range(3):
        s = [1, 1, 1, 1.6, 1.3, 1.3, 1.1, 1.1, 1.8]
        q = [1, 1.2, 1.2, 1.9, 1.7]
        p = _p(lib, s, q, gbeta=0.03, T0=0.4, ax=2e-3, ay=-1e-3, varpi=0.45)
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
        f = w * (1 + 0.4 * rng.uniform(-1, 1, 9))
        g = np.array([0.5] + [0.125] * 4) * (1 + 0.4 * rng.uniform(-1, 1, 5))
        fo, go = oracle.collide_node(p, f, g, library=lib)
        fe, ge = X.collide([Fr(v) for v in f], [Fr(v) for v in g], [Fr(v) for v in p.s],
                           [Fr(v) for v in p.q][:5], Fr(p.varpi), Fr(p.gbeta), Fr(p.T0), Fr(p.ax), Fr(p.ay))
        if (np.max(np.abs(fo - np.array([float(v) for v in fe]))) > 1e-14
                or np.max(np.abs(go - np.array([float(v) for v in ge]))) > 1e-14):
            failed.append("collision_exact")
            break
    # exact single-node collision of the D2Q9 thermal model (Eqs. 31-32)
    p = _p(lib, [1, 1, 1, 1.6, 1.3, 1.3, 1.1, 1.1, 1.8], [1, 1.2, 1.2, 1.9, 1.7, 1.7, 1.4, 1.4, 0.8],
           gbeta=0.03, T0=0.4, ax=2e-3, ay=-1e-3)
    p.model, p.theta = oracle.MODEL_D2Q9T, 1.0
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = w * (1 + 0.4 * rng.uniform(-1, 1, 9))
    g = w * 0.7 * (1 + 0.4 * rng.uniform(-1, 1, 9))
    fo, go = oracle.collide_node(p, f, g, library=lib)
    fe, ge = X.collide_d2q9t([Fr(v) for v in f], [Fr(v) for v in g], [Fr(v) for v in p.s],
                             [Fr(v) for v in p.q], Fr(1), Fr(p.gbeta), Fr(p.T0), Fr(p.ax), Fr(p.ay))
    if (np.max(np.abs(fo - np.array([float(v) for v in fe]))) > 1e-14
            or np.max(np.abs(go - np.array([float(v) for v in ge]))) > 1e-14):
        failed.append("collision_exact_d2q9t")
    # Couette exact, D2Q9 thermal model (moving wall, Dirichlet walls)
    L = oracle.Lattice(W.channel(3, 16, s_nu=1.3, zeta_alpha=1.1, u_top=(0.05, 0.0)), library=lib,
                       model="d2q9t")
    L.step(12000)
    _, ux, uy, T = L.moments()
    y = (np.arange(16) + 0.5) / 16
    if not (np.max(np.abs(ux - 0.05 * y[:, None])) < 1e-13 and np.max(np.abs(T - y[:, None])) < 1e-13):
        failed.append("couette_exact_d2q9t")
    # BGK (velocity-space flow update, textbook temperature update) and the
    # orthogonal MRT, each against its exact reference
    s = [1, 1, 1, 1.5, 1.2, 1.2, 1.1, 1.1, 1.7]
    f = w * (1 + 0.4 * rng.uniform(-1, 1, 9))
    g = np.array([0.5] + [0.125] * 4) * (1 + 0.4 * rng.uniform(-1, 1, 5))
    Fx, Fy = 2e-3, -1e-3 + 0.03 * (g.sum() - 0.4)
    for coll in (oracle.COLL_BGK, oracle.COLL_ORTHO):
        p = _p(lib, s, [1, 1.2, 1.2, 1.9, 1.7], gbeta=0.03, T0=0.4, ax=2e-3, ay=-1e-3)
        p.collision = coll
        fo, go = oracle.collide_node(p, f, g, library=lib)
        if coll == oracle.COLL_BGK:
            fe = X.collide_bgk_flow([Fr(v) for v in f], Fr(1.2), Fr(Fx), Fr(Fy))
            e = np.array(X.E9, dtype=float)
            u = e.T @ f + np.array([Fx, Fy]) / 2
            T = g.sum()
            geq = np.concatenate([[0.5 * T], 0.125 * T + 0.5 * (e[1:5] @ u) * T])
            if np.max(np.abs(go - (g - 1.2 * (g - geq)))) > 1e-14:
                failed.append("bgk_thermal")
        else:
            so = [Fr(1), Fr(1.5), Fr(1.7), Fr(1), Fr(1.1), Fr(1), Fr(1.1), Fr(1.2), Fr(1.2)]
            fe = X.collide_ortho_flow([Fr(v) for v in f], so, Fr(Fx), Fr(Fy))
        if np.max(np.abs(fo - np.array([float(v) for v in fe]))) > 1e-14:
            failed.append(f"collision_exact_{coll}")
    # uniformly moving equilibrium between moving Dirichlet plates is a fixed point
    u = np.array([0.05, 0.02])
    e = np.array(X.E9, dtype=float)
    eu = e @ u
    feq = w * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u @ u))
    pb = W.channel(3, 8, s_nu=1.3, zeta_alpha=1.1, u_top=(0.05, 0.02), u_bottom=(0.05, 0.02),
                   t_bottom=1.0, t_top=1.0).replace(t_hot=1.0, t_cold=0.0)
    L = oracle.Lattice(pb, library=lib, model="d2q9t")
    L.set_state(np.broadcast_to(feq[:, None, None], (9, 8, 3)).copy(),
                np.broadcast_to(feq[:, None, None], (9, 8, 3)).copy())
    L.step(200)
    if np.max(np.abs(L.moments()[3] - 1)) > 1e-14:
        failed.append("moving_equilibrium_d2q9t")
    # Couette exact (moving wall, Dirichlet walls)
    L = oracle.Lattice(W.channel(3, 16, s_nu=1.3, zeta_alpha=1.1, u_top=(0.05, 0.0)), library=lib)
    L.step(12000)
    _, ux, uy, T = L.moments()
    y = (np.arange(16) + 0.5) / 16
    if not (np.max(np.abs(ux - 0.05 * y[:, None])) < 1e-13 and np.max(np.abs(T - y[:, None])) < 1e-13):
        failed.append("couette_exact")
    # mass conservation and the centro-symmetry of the heated cavity
    L = oracle.Lattice(W.cavity(12, 1e5, t_hot=0.5, t_cold=-0.5), library=lib)
    r0 = L.moments()[0].sum()
    L.step(300)
    rho, ux, uy, T = L.moments()
    if abs(rho.sum() - r0) / r0 > 1e-13 or not np.all(np.isfinite(rho)):
        failed.append("mass")
    if np.max(np.abs(ux + ux[::-1, ::-1])) > 1e-14 or np.max(np.abs(T + T[::-1, ::-1])) > 1e-14:
        failed.append("centro_symmetry")
    # the hot wall must drive an upward flow next to it (buoyancy sign, Eq. 4)
    if not uy[6, 0] > 0:
        failed.append("buoyancy_direction")
    # Nusselt stencil on a quadratic profile
    pb = W.cavity(6, 1e4).replace(u_c=0.0, s_nu=1.0, zeta_alpha=1.0)
    xx = np.arange(6) + 0.5
    Tq = 1.0 - 0.1 * xx + 0.004 * xx ** 2
    L = oracle.Lattice(pb, T_init=np.tile(Tq, (6, 1)), library=lib)
    if abs(L.nusselt(W.LEFT)[0] - 6 * 0.1) > 1e-12:
        failed.append("nusselt_quadratic")
    # non-equilibrium extrapolation walls: Couette exact with the walls on the nodes
    pb = W.channel(3, 12, s_nu=1.2, zeta_alpha=0.9, u_top=(0.04, 0.0)).replace(
        bc_flow=(0, 0, 2, 2), bc_temp=(0, 0, 3, 3))
    L = oracle.Lattice(pb, library=lib)
    L.step(8000)
    _, ux, uy, T = L.moments()
    yy = np.arange(12) / 11.0
    if not (np.max(np.abs(ux - 0.04 * yy[:, None])) < 1e-12 and np.max(np.abs(T - yy[:, None])) < 1e-12):
        failed.append("nee_couette_exact")
    # NEE Nusselt number: quadratic in the wall distance, slope quadratic
    # along the wall (local values and the trapezoidal mean in closed form)
    pb = W.cavity(7, 1e4, ny=9).replace(bc_flow=(2, 2, 0, 0), bc_temp=(3, 3, 0, 0), length=6.0)
    yy, xx = np.mgrid[0:9, 0:7].astype(float)
    a = 0.013 - 0.0011 * yy + 0.00031 * yy ** 2
    L = oracle.Lattice(pb, T_init=1.0 + a * xx - 0.0021 * xx ** 2, library=lib)
    mean, _, _, loc = L.nusselt(W.LEFT, local=True)
    k = np.arange(9.0)
    if (np.max(np.abs(loc + 6.0 * (0.013 - 0.0011 * k + 0.00031 * k * k))) > 1e-12
            or abs(mean + 6.0 * (0.013 - 0.0011 * 4 + 0.00031 * (64 / 3 + 1 / 6))) > 1e-12):
        failed.append("nee_nusselt_quadratic")
    # mirror symmetry of a Rayleigh-Benard cell with a symmetric start
    T = W.rb_initial_temperature(12, 6, amp=1e-2, seed=9)
    T = 0.5 * (T + T[:, ::-1])
    L = oracle.Lattice(W.rayleigh_benard(12, 6, 5e4), T_init=T, library=lib)
    L.step(200)
    _, ux, uy, T1 = L.moments()
    if np.max(np.abs(ux + ux[:, ::-1])) > 1e-14 or np.max(np.abs(T1 - T1[:, ::-1])) > 1e-14:
        failed.append("rb_mirror")
    return failed


@pytest.fixture(scope="module")
def tmpdir_mod(tmp_path_factory):
    return str(tmp_path_factory.mktemp("mutants"))


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_is_caught(name, tmpdir_mod):
    lib = _build(tmpdir_mod, name, MUTANTS[name])
    failed = _battery(lib)
    if name == "none":
        assert failed == []
    else:
        assert failed, f"mutant {name} passed every pin"
