"""The OpenMP build of the oracle, which only the CPU timing of the
benchmark uses, must give bitwise the results of the serial build: the
same source and flags, with the loops over nodes (collision) and rows
(streaming) split across threads, each target written by one thread."""
import numpy as np
import pytest

import oracle
from paper_1510_08224_amd import workloads as W


@pytest.mark.parametrize("case", ["cavity", "rb", "nee", "d2q9t", "lid"])
def test_openmp_build_matches_serial_bitwise(case):
    omp = oracle.lib_openmp()
    assert omp.orc_threads() >= 1
    model = "d2q5"
    T = None
    if case == "cavity":
        pb = W.cavity(67, 1e5, ny=41)
    elif case == "rb":
        pb = W.rayleigh_benard(64, 23, 5e4)
        T = W.rb_initial_temperature(64, 23, amp=1e-2, seed=3)
    elif case == "nee":
        pb = W.with_nee_walls(W.cavity(37, 1e5, ny=29).replace(length=28))
    elif case == "d2q9t":
        pb, model = W.cavity(33, 1e4, ny=35), "d2q9t"
    else:
        pb, model = W.lid_cavity(40, 1.3, 0.1), "isothermal"
    out = []
    for library in (oracle.lib(), omp):
        L = oracle.Lattice(pb, T_init=T, library=library, model=model)
        L.step(60)
        out.append(L.get_state())
    (f1, g1), (f2, g2) = out
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2)
