"""CPU FP64 oracle for the non-orthogonal MRT lattice Boltzmann method
(Liu, He, Li & Li, arXiv:1510.08224).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_1510_08224_amd``) never imports it, and this package imports
nothing from the product.

The arithmetic of a time step lives in ``orc_lbm.c`` (plain C, dense matrix
products, push streaming, ``-ffp-contract=off``).  This module adds, in
plain Python:

* the parameter map of Eq. 40 and the rate diagonals of Eqs. 20, 29 and 32;
* the closed-form profiles of Eqs. 34, 36 and 37 and the error norms of
  Eqs. 35 and 38, used to pin the oracle against the paper;
* a ``Lattice`` wrapper around the C oracle.

Problems are passed as any object with the attributes of
``paper_1510_08224_amd.workloads.Problem`` (duck typing: nothing is
imported from the product package).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc_lbm.c")
_LIB = os.path.join(_HERE, "liborc_lbm.so")
_LIB_OMP = os.path.join(_HERE, "liborc_lbm_omp.so")

# Interface constants (the same values the C library header uses).
LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3
FLOW_PERIODIC, FLOW_WALL, FLOW_NEE = 0, 1, 2
TEMP_PERIODIC, TEMP_DIRICHLET, TEMP_ADIABATIC, TEMP_NEE_DIRICHLET, TEMP_NEE_ADIABATIC = 0, 1, 2, 3, 4
MODEL_D2Q5, MODEL_D2Q9T, MODEL_ISOTHERMAL = 0, 1, 2
MODELS = {"d2q5": MODEL_D2Q5, "d2q9t": MODEL_D2Q9T, "isothermal": MODEL_ISOTHERMAL}
MODEL_NG = {MODEL_D2Q5: 5, MODEL_D2Q9T: 9, MODEL_ISOTHERMAL: 0}
COLL_MRT, COLL_BGK, COLL_ORTHO = 0, 1, 2

CS2 = 1.0 / 3.0  # D2Q9 lattice sound speed squared (Sec. 2.1, after Eq. 19)


_CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction; also its
    OpenMP build (the same source and flags plus -fopenmp), which only the
    CPU timing uses."""
    if force or not os.path.exists(_LIB):
        subprocess.run(["gcc", *_CFLAGS, "-Wno-unknown-pragmas", "-o", _LIB, _SRC, "-lm"], check=True)
    if force or not os.path.exists(_LIB_OMP):
        subprocess.run(["gcc", *_CFLAGS, "-fopenmp", "-o", _LIB_OMP, _SRC, "-lm"], check=True)
    return _LIB


def lib_openmp():
    """The OpenMP build of the oracle (built if missing or stale): loops
    over nodes and rows split across the OpenMP team; results bitwise those
    of the serial build."""
    if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
        build()
    return load(_LIB_OMP)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("model", ctypes.c_int32),
        ("s", ctypes.c_double * 9), ("q", ctypes.c_double * 9),
        ("varpi", ctypes.c_double), ("theta", ctypes.c_double), ("rho0", ctypes.c_double),
        ("gbeta", ctypes.c_double), ("T0", ctypes.c_double),
        ("ax", ctypes.c_double), ("ay", ctypes.c_double),
        ("bc_flow", ctypes.c_int32 * 4), ("bc_temp", ctypes.c_int32 * 4),
        ("wall_T", ctypes.c_double * 4), ("wall_u", (ctypes.c_double * 2) * 4),
        ("s8_literal", ctypes.c_int32), ("collision", ctypes.c_int32),
    ]


_lib = None


def lib():
    """The oracle library (built on first use if missing or stale)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = load(_LIB)
    return _lib


def load(path: str):
    """Load an oracle build from ``path`` and declare its C signatures."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER(OrcParams)
    L.orc_create.argtypes = [P]
    L.orc_create.restype = ctypes.c_void_p
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    L.orc_check_params.argtypes = [P]
    L.orc_check_params.restype = ctypes.c_int
    L.orc_init_equilibrium.argtypes = [ctypes.c_void_p, dp]
    L.orc_set_state.argtypes = [ctypes.c_void_p, dp, dp]
    L.orc_get_state.argtypes = [ctypes.c_void_p, dp, dp]
    L.orc_threads.argtypes = []
    L.orc_threads.restype = ctypes.c_int
    L.orc_time.argtypes = [ctypes.c_void_p]
    L.orc_time.restype = ctypes.c_int64
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    L.orc_post_collision.argtypes = [ctypes.c_void_p, dp, dp]
    L.orc_moments.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
    L.orc_nusselt.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              dp, dp, dp, ctypes.POINTER(ctypes.c_int32)]
    L.orc_nusselt.restype = ctypes.c_int
    L.orc_collide_node.argtypes = [P, dp, dp, dp, dp]
    L.orc_tables.argtypes = [dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32)]
    L.orc_params_size.restype = ctypes.c_size_t
    assert L.orc_params_size() == ctypes.sizeof(OrcParams)
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tables(library=None) -> dict:
    """The oracle's own M, M^-1, N, N^-1, weights and velocities."""
    m9 = np.zeros((9, 9)); mi9 = np.zeros((9, 9))
    n5 = np.zeros((5, 5)); ni5 = np.zeros((5, 5)); w9 = np.zeros(9)
    ex = np.zeros(9, dtype=np.int32); ey = np.zeros(9, dtype=np.int32)
    (library or lib()).orc_tables(_dp(m9), _dp(mi9), _dp(n5), _dp(ni5), _dp(w9),
                                  ex.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  ey.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return {"M": m9, "Minv": mi9, "N": n5, "Ninv": ni5, "w": w9, "ex": ex, "ey": ey}


# ---------------------------------------------------------------------------
# Parameter map (Eqs. 20, 29, 40; Sec. 3 global settings)
# ---------------------------------------------------------------------------
def _model(model) -> int:
    return MODELS[model] if isinstance(model, str) else int(model)


def derive(pb, model=MODEL_D2Q5) -> dict:
    """Relaxation diagonals and forcing constants for a problem.

    s_nu and zeta_alpha come from Eq. 40 unless given explicitly (> 0):
        1/s_nu = 1/2 + Ma L sqrt(3 Pr) / sqrt(Ra),  Ma = sqrt(3) u_c,
        1/zeta_alpha = 1/2 + c_s^2 (1/s_nu - 1/2) / (c_sT^2 Pr),
    with c_s^2 = 1/3 and c_sT^2 = varpi/2 for the D2Q5 model (Sec. 2.2),
    c_sT^2 = c_s^2 for the D2Q9 thermal model (the diffusivity stated after
    Eq. 32).  g*beta follows from u_c = sqrt(g beta dT L) (text after
    Eq. 40), and is 0 without a temperature field; T0 = (T_h + T_c)/2.
    L defaults to the distance between the bottom and top walls: ny for
    link-wise walls (half a spacing outside the nodes), ny - 1 for NEE walls.
    The thermal diagonal is Eq. 29 (D2Q5, 5 entries) or Eq. 32 (D2Q9, 9).
    """
    model = _model(model)
    length = pb.length if pb.length > 0 else (float(pb.ny - 1) if pb.bc_flow[BOTTOM] == FLOW_NEE
                                               else float(pb.ny))
    dT = pb.t_hot - pb.t_cold
    csT2 = CS2 if model == MODEL_D2Q9T else pb.varpi / 2.0
    if pb.s_nu > 0:
        s_nu = pb.s_nu
    else:
        if not (pb.u_c > 0 and pb.ra > 0 and pb.pr > 0):
            raise ValueError("s_nu needs either an explicit value or Ra, Pr, u_c")
        ma = math.sqrt(3.0) * pb.u_c
        s_nu = 1.0 / (0.5 + ma * length * math.sqrt(3.0 * pb.pr) / math.sqrt(pb.ra))
    if pb.zeta_alpha > 0:
        z_a = pb.zeta_alpha
    else:
        if not pb.pr > 0:
            raise ValueError("zeta_alpha needs either an explicit value or Pr")
        z_a = 1.0 / (0.5 + CS2 * (1.0 / s_nu - 0.5) / (csT2 * pb.pr))
    gbeta = (pb.u_c ** 2 / (dT * length)
             if (model != MODEL_ISOTHERMAL and pb.u_c > 0 and dT != 0) else 0.0)
    s = [1.0, 1.0, 1.0, pb.s_e, s_nu, s_nu, pb.s_q, pb.s_q, pb.s_eps]       # Eq. 20
    if model == MODEL_D2Q9T:                                                # Eq. 32
        q = [1.0, z_a, z_a, pb.zeta_e, pb.zeta_nu, pb.zeta_nu, pb.zeta_q, pb.zeta_q, pb.zeta_eps]
    else:                                                                   # Eq. 29
        q = [1.0, z_a, z_a, pb.zeta_e, pb.zeta_nu]
    return {"model": model, "s": s, "q": q, "s_nu": s_nu, "zeta_alpha": z_a, "gbeta": gbeta,
            "T0": 0.5 * (pb.t_hot + pb.t_cold), "length": length, "dT": dT,
            "nu": CS2 * (1.0 / s_nu - 0.5), "alpha": csT2 * (1.0 / z_a - 0.5)}


def rate_for_reynolds(re: float, length: float, u: float) -> float:
    """s_nu for a Reynolds number Re = L u / nu (Sec. 3.2):
    1/s_nu = 1/2 + L u / (c_s^2 Re)."""
    return 1.0 / (0.5 + length * u / (CS2 * re))


def make_params(pb, s8_literal: bool = False, overrides: dict | None = None,
                model=MODEL_D2Q5) -> OrcParams:
    d = derive(pb, model)
    if overrides:
        d.update(overrides)
    p = OrcParams()
    p.nx, p.ny = int(pb.nx), int(pb.ny)
    p.model = d["model"]
    for k in range(9):
        p.s[k] = d["s"][k]
    for k in range(len(d["q"])):
        p.q[k] = d["q"][k]
    p.varpi = pb.varpi
    p.theta = getattr(pb, "theta", 1.0)
    p.rho0 = 1.0
    p.gbeta = d["gbeta"]
    p.T0 = d["T0"]
    p.ax, p.ay = pb.ax, pb.ay
    for k in range(4):
        p.bc_flow[k] = int(pb.bc_flow[k])
        p.bc_temp[k] = int(pb.bc_temp[k])
        p.wall_T[k] = float(pb.wall_T[k])
        p.wall_u[k][0] = float(pb.wall_u[k][0])
        p.wall_u[k][1] = float(pb.wall_u[k][1])
    p.s8_literal = 1 if s8_literal else 0
    p.collision = int(getattr(pb, "collision", COLL_MRT))
    return p


def collide_node(params: OrcParams, f, g, library=None):
    """One-node collision (Eqs. 8 and 24 followed by M^-1 and N^-1)."""
    ng = MODEL_NG[params.model]
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g if ng else np.zeros(1), dtype=np.float64)
    fo = np.zeros(9); go = np.zeros(max(ng, 1))
    (library or lib()).orc_collide_node(ctypes.byref(params), _dp(f), _dp(g), _dp(fo), _dp(go))
    return fo, go[:ng]


class Lattice:
    """An nx x ny lattice advanced by the C oracle.  State = pre-collision
    populations at time t, exchanged in plane order [i][y][x]."""

    def __init__(self, pb, s8_literal: bool = False, T_init=None, overrides=None, library=None,
                 model=MODEL_D2Q5):
        self._lib = library or lib()
        self.pb = pb
        self.model = _model(model)
        self.ng = MODEL_NG[self.model]
        self.params = make_params(pb, s8_literal, overrides, self.model)
        self.derived = derive(pb, self.model)
        if overrides:
            self.derived.update(overrides)
        self._h = self._lib.orc_create(ctypes.byref(self.params))
        if not self._h:
            raise ValueError("inconsistent oracle parameters")
        self.nx, self.ny = int(pb.nx), int(pb.ny)
        self.init(T_init)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def init(self, T=None):
        if T is None:
            self._lib.orc_init_equilibrium(self._h, None)
        else:
            T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.ny, self.nx)
            self._lib.orc_init_equilibrium(self._h, _dp(T))

    @property
    def t(self) -> int:
        return self._lib.orc_time(self._h)

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    def _gbuf(self):
        return np.zeros((max(self.ng, 1), self.ny, self.nx))

    def get_state(self):
        f = np.zeros((9, self.ny, self.nx)); g = self._gbuf()
        self._lib.orc_get_state(self._h, _dp(f), _dp(g))
        return f, g[:self.ng]

    def set_state(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        if self.ng:
            g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.ng, self.ny, self.nx)
        else:
            g = self._gbuf()
        self._lib.orc_set_state(self._h, _dp(f), _dp(g))

    def post_collision(self):
        f = np.zeros((9, self.ny, self.nx)); g = self._gbuf()
        self._lib.orc_post_collision(self._h, _dp(f), _dp(g))
        return f, g[:self.ng]

    def moments(self):
        shp = (self.ny, self.nx)
        rho, ux, uy, T = (np.zeros(shp) for _ in range(4))
        self._lib.orc_moments(self._h, _dp(rho), _dp(ux), _dp(uy), _dp(T))
        return rho, ux, uy, T

    def nusselt(self, side: int, local: bool = False):
        n = self.ny if side in (LEFT, RIGHT) else self.nx
        loc = np.zeros(n)
        mean = ctypes.c_double(); mx = ctypes.c_double(); imax = ctypes.c_int32()
        rc = self._lib.orc_nusselt(self._h, side, self.derived["length"], self.derived["dT"],
                               _dp(loc), ctypes.byref(mean), ctypes.byref(mx), ctypes.byref(imax))
        if rc != 0:
            raise ValueError("Nusselt number needs a Dirichlet wall")
        out = (mean.value, mx.value, imax.value)
        return (out + (loc,)) if local else out


def residual(prev, cur) -> float:
    """max over nodes of max(|dux|, |duy|, |dT|) between two (ux, uy, T)."""
    return float(max(np.max(np.abs(a - b)) for a, b in zip(prev, cur)))


# ---------------------------------------------------------------------------
# Closed forms and error norms used to pin the oracle (Sec. 3)
# ---------------------------------------------------------------------------
def poiseuille_profile(y, u0, lc):
    """Eq. 34: u_x(y) = u0 (1 - (y/lc)^2), -H/2 <= y <= H/2."""
    return u0 * (1.0 - (y / lc) ** 2)


def porous_plate_u(y, u0, re, H):
    """Eq. 36: u_x(y) = u0 (exp(Re y/H) - 1)/(exp(Re) - 1)."""
    return u0 * np.expm1(re * y / H) / math.expm1(re)


def porous_plate_T(y, t_c, dT, pr, re, H):
    """Eq. 37: T = T_c + dT (exp(Pr Re y/H) - 1)/(exp(Pr Re) - 1)."""
    return t_c + dT * np.expm1(pr * re * y / H) / math.expm1(pr * re)


def error_u(ua_x, ua_y, ux, uy) -> float:
    """Eq. 35: sum ||u_A - u_LB||_2 / sum ||u_A||_2 (node-wise vector norms)."""
    num = np.sum(np.sqrt((ua_x - ux) ** 2 + (ua_y - uy) ** 2))
    den = np.sum(np.sqrt(ua_x ** 2 + ua_y ** 2))
    return float(num / den)


def error_T(ta, t) -> float:
    """Eq. 38: sqrt(sum |T_A - T_LB|^2) / sqrt(sum |T_A|^2)."""
    return float(np.sqrt(np.sum((ta - t) ** 2)) / np.sqrt(np.sum(ta ** 2)))
