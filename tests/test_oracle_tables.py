"""Pins for the oracle's lattice tables: the velocities of Eq. 5, the
matrices M (Eq. 13), M^-1 (Eq. A1), N (Eq. 26), N^-1 (Eq. A2) and the
Appendix B matrices E_x, E_y.  Each table is checked against both the
printed values (tests/golden/matrices.txt) and an independent construction
from the basis definitions (Eqs. 5, 12, 26) with exact inversion."""
from fractions import Fraction

import numpy as np

import oracle
import exact_ref as X
from golden_io import matrices


def _f(a):
    return np.array([[float(v) for v in row] for row in a])


def test_velocities_follow_eq5():
    t = oracle.tables()
    assert [(int(a), int(b)) for a, b in zip(t["ex"], t["ey"])] == X.E9


def test_weights_sum_and_isotropy():
    # zeroth, second and fourth moments of the D2Q9 weights (c_s^2 = 1/3)
    w = oracle.tables()["w"]
    ex, ey = np.array(X.E9).T
    assert abs(w.sum() - 1) < 1e-15
    assert abs((w * ex * ex).sum() - 1 / 3) < 1e-15
    assert abs((w * ex * ex * ey * ey).sum() - 1 / 9) < 1e-15
    assert abs((w * ex ** 4).sum() - 1 / 3) < 1e-15


def test_M_printed_equals_basis_and_oracle():
    g = matrices()
    assert g["M"] == X.M9
    assert np.array_equal(oracle.tables()["M"], _f(g["M"]))


def test_Minv_printed_is_exact_inverse_and_oracle():
    g = matrices()
    assert g["Minv"] == X.M9I
    assert X.matmul(g["M"], g["Minv"]) == [[Fraction(int(i == j)) for j in range(9)] for i in range(9)]
    assert np.array_equal(oracle.tables()["Minv"], _f(g["Minv"]))


def test_N_and_Ninv():
    g = matrices()
    assert g["N"] == X.N5
    assert g["Ninv"] == X.N5I
    t = oracle.tables()
    assert np.array_equal(t["N"], _f(g["N"]))
    assert np.array_equal(t["Ninv"], _f(g["Ninv"]))


def test_appendix_b_Ex_Ey_from_oracle_tables():
    # E_j = N diag(e_j) N^-1 built from the oracle's N and N^-1 must give the
    # printed Appendix B matrices: this pins N^-1 column by column.
    g = matrices()
    t = oracle.tables()
    ex = np.diag(t["ex"][:5].astype(float))
    ey = np.diag(t["ey"][:5].astype(float))
    assert np.array_equal(t["N"] @ ex @ t["Ninv"], _f(g["Ex"]))
    assert np.array_equal(t["N"] @ ey @ t["Ninv"], _f(g["Ey"]))


def test_sparsity_counts():
    # The efficiency argument of the non-orthogonal basis: zeros in M, M^-1.
    t = oracle.tables()
    assert np.count_nonzero(t["M"]) == 49
    assert np.count_nonzero(t["Minv"]) == 39
    assert np.count_nonzero(t["N"]) == 17
    assert np.count_nonzero(t["Ninv"]) == 14
