"""Problem descriptions and seeded synthetic inputs.

This module holds no arithmetic of the lattice Boltzmann method: it only
states problems (lattice size, dimensionless groups, wall types and wall
values) and draws seeded random inputs.  It is the one module that both the
GPU path and the CPU oracle are fed from.

Workloads follow the paper's problems (Sec. 3): the differentially heated
square cavity (Sec. 3.4), the channel with a moving, injecting wall
(Sec. 3.3), the body-force-driven channel (Sec. 3.1), plus the
lid-driven cavity (Sec. 3.2), the Rayleigh-Benard cell, the batched cavity mix and the Poisson request stream
used for precision, batching and serving measurements.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3
FLOW_PERIODIC, FLOW_WALL, FLOW_NEE = 0, 1, 2
TEMP_PERIODIC, TEMP_DIRICHLET, TEMP_ADIABATIC, TEMP_NEE_DIRICHLET, TEMP_NEE_ADIABATIC = 0, 1, 2, 3, 4
COLL_MRT, COLL_BGK, COLL_ORTHO = 0, 1, 2   # collision operator (the paper's MRT and its comparisons)


def with_nee_walls(pb: "Problem") -> "Problem":
    """The same problem with non-equilibrium-extrapolation walls in place of
    link-wise walls (walls through the first/last node row or column)."""
    tmap = {TEMP_DIRICHLET: TEMP_NEE_DIRICHLET, TEMP_ADIABATIC: TEMP_NEE_ADIABATIC}
    flow = tuple(FLOW_NEE if f == FLOW_WALL else f for f in pb.bc_flow)
    temp = tuple(tmap.get(t, t) for t in pb.bc_temp)
    return dataclasses.replace(pb, bc_flow=flow, bc_temp=temp, name=pb.name + "_nee")


@dataclass
class Problem:
    """One lattice problem.  Field meanings match ``lbm_params`` in
    ``include/lbm.h``; zero for ``s_nu``/``zeta_alpha``/``length`` means
    "derive"."""
    nx: int
    ny: int
    ra: float = 0.0
    pr: float = 0.71
    u_c: float = 0.0
    length: float = 0.0
    t_hot: float = 1.0
    t_cold: float = 0.0
    s_e: float = 1.6
    s_q: float = 1.2
    s_eps: float = 1.8
    zeta_e: float = 1.9
    zeta_nu: float = 1.9
    varpi: float = 0.5
    zeta_q: float = 1.9
    zeta_eps: float = 1.9
    theta: float = 1.0
    s_nu: float = 0.0
    zeta_alpha: float = 0.0
    ax: float = 0.0
    ay: float = 0.0
    bc_flow: tuple = (FLOW_WALL, FLOW_WALL, FLOW_WALL, FLOW_WALL)
    bc_temp: tuple = (TEMP_DIRICHLET, TEMP_DIRICHLET, TEMP_ADIABATIC, TEMP_ADIABATIC)
    wall_T: tuple = (1.0, 0.0, 0.0, 0.0)
    wall_u: tuple = ((0.0, 0.0), (0.0, 0.0), (0.0, 0.0), (0.0, 0.0))
    collision: int = COLL_MRT
    name: str = ""

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


def cavity(n: int, ra: float, pr: float = 0.71, u_c: float = 0.1,
           t_hot: float = 1.0, t_cold: float = 0.0, ny: int | None = None) -> Problem:
    """Differentially heated cavity (Sec. 3.4): hot left wall, cold right
    wall, adiabatic top and bottom, no-slip everywhere."""
    return Problem(nx=n, ny=ny or n, ra=ra, pr=pr, u_c=u_c, t_hot=t_hot, t_cold=t_cold,
                   bc_flow=(FLOW_WALL,) * 4,
                   bc_temp=(TEMP_DIRICHLET, TEMP_DIRICHLET, TEMP_ADIABATIC, TEMP_ADIABATIC),
                   wall_T=(t_hot, t_cold, 0.0, 0.0), name=f"cavity{n}_ra{ra:g}")


def rayleigh_benard(nx: int, ny: int, ra: float, pr: float = 0.71, u_c: float = 0.1,
                    t_hot: float = 1.0, t_cold: float = 0.0) -> Problem:
    """Rayleigh-Benard cell: periodic in x, hot bottom, cold top, no-slip."""
    return Problem(nx=nx, ny=ny, ra=ra, pr=pr, u_c=u_c, t_hot=t_hot, t_cold=t_cold,
                   bc_flow=(FLOW_PERIODIC, FLOW_PERIODIC, FLOW_WALL, FLOW_WALL),
                   bc_temp=(TEMP_PERIODIC, TEMP_PERIODIC, TEMP_DIRICHLET, TEMP_DIRICHLET),
                   wall_T=(0.0, 0.0, t_hot, t_cold), name=f"rb{nx}x{ny}_ra{ra:g}")


def channel(nx: int, ny: int, s_nu: float, zeta_alpha: float = 1.0, ax: float = 0.0,
            u_top=(0.0, 0.0), u_bottom=(0.0, 0.0), t_bottom: float = 0.0, t_top: float = 1.0,
            rates_one: bool = False) -> Problem:
    """x-periodic channel between two plates (Secs. 3.1 and 3.3): the plates
    may move (u_top, u_bottom) and carry Dirichlet temperatures.  With
    ``rates_one`` every free rate other than s_nu and zeta_alpha is 1 (the
    setting of Secs. 3.1 and 3.3)."""
    kw = dict(s_e=1.0, s_q=1.0, s_eps=1.0, zeta_e=1.0, zeta_nu=1.0) if rates_one else {}
    return Problem(nx=nx, ny=ny, s_nu=s_nu, zeta_alpha=zeta_alpha, ax=ax,
                   t_hot=t_top, t_cold=t_bottom,
                   bc_flow=(FLOW_PERIODIC, FLOW_PERIODIC, FLOW_WALL, FLOW_WALL),
                   bc_temp=(TEMP_PERIODIC, TEMP_PERIODIC, TEMP_DIRICHLET, TEMP_DIRICHLET),
                   wall_T=(0.0, 0.0, t_bottom, t_top),
                   wall_u=((0.0, 0.0), (0.0, 0.0), tuple(u_bottom), tuple(u_top)),
                   name=f"channel{nx}x{ny}", **kw)


def lid_cavity(n: int, s_nu: float, u0: float = 0.1) -> Problem:
    """Lid-driven cavity (Sec. 3.2): the top wall moves in +x with u0, the
    other walls are at rest; s_e, s_q, s_eps at the paper's 1.6, 1.2, 1.8.
    Meant for the model without a temperature field (walls adiabatic)."""
    return Problem(nx=n, ny=n, s_nu=s_nu, zeta_alpha=1.0,
                   bc_flow=(FLOW_WALL,) * 4, bc_temp=(TEMP_ADIABATIC,) * 4,
                   wall_T=(0.0, 0.0, 0.0, 0.0),
                   wall_u=((0.0, 0.0), (0.0, 0.0), (0.0, 0.0), (u0, 0.0)),
                   name=f"lid{n}_snu{s_nu:.4f}")


def periodic_box(nx: int, ny: int, s_nu: float, zeta_alpha: float, **kw) -> Problem:
    """Fully periodic lattice (no walls)."""
    return Problem(nx=nx, ny=ny, s_nu=s_nu, zeta_alpha=zeta_alpha,
                   bc_flow=(FLOW_PERIODIC,) * 4, bc_temp=(TEMP_PERIODIC,) * 4,
                   name=f"periodic{nx}x{ny}", **kw)


# ---------------------------------------------------------------------------
# Seeded inputs
# ---------------------------------------------------------------------------
def rb_initial_temperature(nx: int, ny: int, t_hot: float = 1.0, t_cold: float = 0.0,
                           amp: float = 1e-3, seed: int = 1510) -> np.ndarray:
    """Linear conduction profile between the plates (walls half a spacing
    outside the first and last rows) plus uniform noise in [-amp, amp],
    drawn with PCG64(seed) in [y][x] order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y = (np.arange(ny, dtype=np.float64) + 0.5) / ny
    base = t_hot - (t_hot - t_cold) * y
    noise = rng.uniform(-amp, amp, size=(ny, nx))
    return np.ascontiguousarray(base[:, None] + noise)


def random_temperature(nx: int, ny: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(ny, nx))


def random_populations(nx: int, ny: int, seed: int, f_scale: float = 0.1, g_scale: float = 0.2,
                       spread: float = 0.3, ng: int = 5):
    """Arbitrary positive population fields in plane order [i][y][x]:
    value = scale * (1 + spread * U(-1, 1)), 9 flow planes then ``ng``
    temperature planes (5, 9 or 0).  Used for collision parity on states
    far from equilibrium."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = f_scale * (1.0 + spread * rng.uniform(-1.0, 1.0, size=(9, ny, nx)))
    g = g_scale * (1.0 + spread * rng.uniform(-1.0, 1.0, size=(ng, ny, nx)))
    return np.ascontiguousarray(f), np.ascontiguousarray(g)


def batch_mix(count: int = 256, seed: int = 3, sides=(64, 96, 128, 192, 256),
              ra_range=(1e3, 1e6), prs=(0.71, 7.0), u_c: float = 0.1) -> list[Problem]:
    """Independent cavities: side uniform over ``sides``, Ra log-uniform,
    Pr uniform over ``prs``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        n = int(rng.choice(sides))
        ra = float(10.0 ** rng.uniform(math.log10(ra_range[0]), math.log10(ra_range[1])))
        pr = float(rng.choice(prs))
        pb = cavity(n, ra, pr, u_c)
        pb.name = f"b{k}_n{n}_ra{ra:.3g}_pr{pr}"
        out.append(pb)
    return out


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the stream
    problem: Problem
    kind: str               # "cavity" or "rb"


def request_stream(count: int, rate: float, seed: int = 4, n_range=(64, 1024), round_to: int = 16,
                   ra_range=(1e3, 1e6), pr: float = 0.71, u_c: float = 0.1,
                   rb_aspect: int = 2) -> list[Request]:
    """Poisson arrivals (exponential gaps, mean 1/rate) of cavity and
    Rayleigh-Benard solves, 50/50.  Side uniform in n_range, rounded to a
    multiple of ``round_to``; Ra log-uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(rng.uniform(*n_range) / round_to) * round_to)
        n = max(n_range[0], min(n_range[1], n))
        ra = float(10.0 ** rng.uniform(math.log10(ra_range[0]), math.log10(ra_range[1])))
        if rng.uniform() < 0.5:
            pb, kind = cavity(n, ra, pr, u_c), "cavity"
        else:
            ny = max(round_to, (n // rb_aspect) // round_to * round_to)
            pb, kind = rayleigh_benard(n, ny, ra, pr, u_c), "rb"
        pb.name = f"r{k}_{kind}_{pb.nx}x{pb.ny}_ra{ra:.3g}"
        out.append(Request(rid=k, arrival=t, problem=pb, kind=kind))
    return out


# Named workloads (sizes and groups of the measured configurations).
def workload_cavity64() -> Problem:
    """64x64 cavity, Ra=1e4, Pr=0.71, u_c=0.1, rest, T=0.5, 20000 steps."""
    return cavity(64, 1e4, 0.71, 0.1)


def workload_cavity2048() -> Problem:
    """2048x2048 cavity, Ra=1e6, Pr=0.71, u_c=0.1."""
    return cavity(2048, 1e6, 0.71, 0.1)


def workload_rb4096x1024() -> Problem:
    """4096x1024 Rayleigh-Benard cell, Ra=1e5, Pr=0.71, u_c=0.1."""
    return rayleigh_benard(4096, 1024, 1e5, 0.71, 0.1)
