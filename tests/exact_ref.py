"""Exact (rational) single-node reference for the collision, used to pin the
oracle.  It follows a route independent of the oracle's:

* velocities are evaluated from the trigonometric definition of Eq. 5;
* M and N are built from their basis definitions (Eq. 12: products
  e_x^p e_y^q; Eq. 26: 1, e_x, e_y, e_x^2+e_y^2, e_x^2-e_y^2) and inverted
  by exact Gauss-Jordan elimination, not taken from the printed tables;
* the update is the velocity-space form, Eq. 7,
      fbar* = fbar - Lt (fbar - f^eq) + (S - Lt S / 2),  Lt = M^-1 Lambda M,
  with f^eq from Eq. 22 and S the Guo forcing term in velocity space, whose
  moments Eq. 10 defines as S~ = M S;
* the thermal update is Eq. 23 with g^eq from Eq. 30 (D2Q5) or Eq. 31
  (D2Q9, with N the D2Q9 basis matrix and Q of Eq. 32).

All arithmetic is in Fractions, so the only rounding is the final
conversion.  The incompressible reading is the one the build uses: rho only
in the rest part of f^eq, rho0 on every velocity term and in the force.
"""
from fractions import Fraction as Fr
import math


def velocities_eq5():
    """Eq. 5 with c = 1, rounded to the integer lattice."""
    e = [(0, 0)]
    for i in range(1, 5):
        a = (i - 1) * math.pi / 2
        e.append((round(math.cos(a)), round(math.sin(a))))
    for i in range(5, 9):
        a = (2 * i - 9) * math.pi / 4
        e.append((round(math.sqrt(2) * math.cos(a)), round(math.sqrt(2) * math.sin(a))))
    return e


E9 = velocities_eq5()
E5 = E9[:5]
W9 = [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4   # weights stated after Eq. 22


def basis_m9():
    """Rows |M_0>..|M_8> of Eq. 12 from their definitions."""
    defs = [lambda x, y: 1, lambda x, y: x, lambda x, y: y,
            lambda x, y: x * x + y * y, lambda x, y: x * x - y * y, lambda x, y: x * y,
            lambda x, y: x * x * y, lambda x, y: x * y * y, lambda x, y: x * x * y * y]
    return [[Fr(d(ex, ey)) for (ex, ey) in E9] for d in defs]


def basis_n5():
    """Rows of N (Eq. 26) from their definitions."""
    defs = [lambda x, y: 1, lambda x, y: x, lambda x, y: y,
            lambda x, y: x * x + y * y, lambda x, y: x * x - y * y]
    return [[Fr(d(ex, ey)) for (ex, ey) in E5] for d in defs]


def inverse(a):
    n = len(a)
    m = [list(row) + [Fr(int(i == j)) for j in range(n)] for i, row in enumerate(a)]
    for c in range(n):
        p = next(r for r in range(c, n) if m[r][c] != 0)
        m[c], m[p] = m[p], m[c]
        piv = m[c][c]
        m[c] = [v / piv for v in m[c]]
        for r in range(n):
            if r != c and m[r][c] != 0:
                fac = m[r][c]
                m[r] = [vr - fac * vc for vr, vc in zip(m[r], m[c])]
    return [row[n:] for row in m]


def matmul(a, b):
    return [[sum(a[i][k] * b[k][j] for k in range(len(b))) for j in range(len(b[0]))]
            for i in range(len(a))]


def matvec(a, v):
    return [sum(a[i][k] * v[k] for k in range(len(v))) for i in range(len(a))]


def diag(d):
    n = len(d)
    return [[d[i] if i == j else Fr(0) for j in range(n)] for i in range(n)]


M9 = basis_m9()
M9I = inverse(M9)
N5 = basis_n5()
N5I = inverse(N5)


def gram_schmidt(rows):
    """Orthogonalize rows (lists of Fractions) in order, plain dot product."""
    out = []
    for v in rows:
        w = list(v)
        for u in out:
            c = sum(a * b for a, b in zip(w, u)) / sum(b * b for b in u)
            w = [a - c * b for a, b in zip(w, u)]
        out.append(w)
    return out


def basis_ortho9():
    """The orthogonal D2Q9 basis: Gram-Schmidt of 1, |e|^2, |e|^4, e_x,
    e_x|e|^2, e_y, e_y|e|^2, e_x^2 - e_y^2, e_x e_y."""
    defs = [lambda x, y: 1, lambda x, y: x * x + y * y, lambda x, y: (x * x + y * y) ** 2,
            lambda x, y: x, lambda x, y: x * (x * x + y * y), lambda x, y: y,
            lambda x, y: y * (x * x + y * y), lambda x, y: x * x - y * y, lambda x, y: x * y]
    return gram_schmidt([[Fr(d(ex, ey)) for (ex, ey) in E9] for d in defs])


MO9 = basis_ortho9()
MO9I = inverse(MO9)


def _flow(f, s, Fx, Fy, rho0, M=None, MI=None):
    """Exact fbar* of Eq. 7 for given force, Lambda~ = M^-1 diag(s) M
    (M of Eq. 12 unless given); returns (fbar*, ux, uy)."""
    M = M9 if M is None else M
    MI = M9I if MI is None else MI
    rho = sum(f)                                     # Eq. 18
    ux = (sum(e[0] * fi for e, fi in zip(E9, f)) + rho0 * Fx / 2) / rho0   # Eq. 19
    uy = (sum(e[1] * fi for e, fi in zip(E9, f)) + rho0 * Fy / 2) / rho0
    usq = ux * ux + uy * uy
    feq, S = [], []
    for (ex, ey), w in zip(E9, W9):
        eu = ex * ux + ey * uy
        eF = ex * Fx + ey * Fy
        uF = ux * Fx + uy * Fy
        feq.append(w * (rho + rho0 * (3 * eu + Fr(9, 2) * eu * eu - Fr(3, 2) * usq)))  # Eq. 22
        S.append(w * rho0 * (3 * eF - 3 * uF + 9 * eu * eF))       # Guo source
    Lt = matmul(MI, matmul(diag(s), M))              # Lambda~ = M^-1 Lambda M
    neq = [fi - fe for fi, fe in zip(f, feq)]
    c1 = matvec(Lt, neq)
    c2 = matvec(Lt, S)
    fo = [fi - a + si - b / 2 for fi, a, si, b in zip(f, c1, S, c2)]   # Eq. 7
    return fo, ux, uy


def collide(f, g, s, q, varpi, gbeta, T0, ax, ay, rho0=Fr(1)):
    """Exact post-collision (fbar*, g*) at one node, D2Q5 temperature model.
    Every argument is a Fraction (or a list of them); s and q are the full
    diagonals."""
    T = sum(g)                                       # Eq. 27
    Fx = ax
    Fy = ay + gbeta * (T - T0)                       # Eq. 4
    fo, ux, uy = _flow(f, s, Fx, Fy, rho0)
    geq = [(1 - varpi) * T] + [varpi * T / 4 + (ex * ux + ey * uy) * T / 2 for (ex, ey) in E5[1:]]  # Eq. 30
    Qt = matmul(N5I, matmul(diag(q), N5))
    d = matvec(Qt, [gi - ge for gi, ge in zip(g, geq)])
    go = [gi - di for gi, di in zip(g, d)]           # Eq. 23
    return fo, go


CS2 = Fr(1, 3)   # D2Q9 sound speed squared


def geq_d2q9(T, ux, uy, theta):
    """Eq. 31 written with c_s^2 = 1/3 kept symbolic."""
    usq = ux * ux + uy * uy
    out = []
    for (ex, ey), w in zip(E9, W9):
        eu = ex * ux + ey * uy
        out.append(w * T * (1 + eu / CS2 + theta * (eu * eu / (2 * CS2 * CS2) - usq / (2 * CS2))))
    return out


def collide_d2q9t(f, g, s, q, theta, gbeta, T0, ax, ay, rho0=Fr(1)):
    """Exact post-collision at one node, D2Q9 temperature model: the
    velocity-space update g* = g - N^-1 Q N (g - g^eq) with N the D2Q9
    basis matrix of Eq. 12, Q of Eq. 32 and g^eq of Eq. 31."""
    T = sum(g)
    Fx = ax
    Fy = ay + gbeta * (T - T0)
    fo, ux, uy = _flow(f, s, Fx, Fy, rho0)
    geq = geq_d2q9(T, ux, uy, theta)
    Qt = matmul(M9I, matmul(diag(q), M9))
    d = matvec(Qt, [gi - ge for gi, ge in zip(g, geq)])
    return fo, [gi - di for gi, di in zip(g, d)]


def collide_isothermal(f, s, ax, ay, rho0=Fr(1)):
    """Exact fbar* without a temperature field: the force is a alone."""
    return _flow(f, s, ax, ay, rho0)[0]


def collide_ortho_flow(f, s_ortho, Fx, Fy, rho0=Fr(1)):
    """Exact fbar* of the classical orthogonal MRT: Eq. 7 with
    Lambda~ = M_o^-1 diag(s_ortho) M_o."""
    return _flow(f, s_ortho, Fx, Fy, rho0, MO9, MO9I)[0]


def collide_bgk_flow(f, w, Fx, Fy, rho0=Fr(1)):
    """Exact single-relaxation-time update with the Guo source."""
    return _flow(f, [w] * 9, Fx, Fy, rho0)[0]


def guo_moments(ux, uy, Fx, Fy, rho0=Fr(1)):
    """M S for the Guo source: the moment-space source that Eq. 10 defines."""
    S = []
    for (ex, ey), w in zip(E9, W9):
        eu = ex * ux + ey * uy
        eF = ex * Fx + ey * Fy
        S.append(w * rho0 * (3 * eF - 3 * (ux * Fx + uy * Fy) + 9 * eu * eF))
    return matvec(M9, S)
