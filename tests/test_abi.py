"""CPU checks of the boundary: the HIP library loads, exports every entry
point declared in include/lbm.h, and its host-only entry points (defaults,
sizes, versions, argument checks) behave as declared.  No GPU is touched."""
import ctypes

import numpy as np
import pytest

from paper_1510_08224_amd import lbm


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    names = lbm.header_symbols()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []
    # the binding declares a signature for each of them
    assert sorted(lbm._SIGS) == names


def test_params_struct_layout_matches():
    p = lbm.lbm_params_default()
    assert p.struct_size == ctypes.sizeof(lbm.LbmParams)
    assert (p.s_e, p.s_q, p.s_eps, p.zeta_e, p.zeta_nu, p.varpi) == (1.6, 1.2, 1.8, 1.9, 1.9, 0.5)
    assert p.pr == 0.71 and p.t_hot == 1.0 and p.t_cold == 0.0
    assert list(p.bc_flow) == [lbm.LBM_BC_WALL] * 4
    assert list(p.bc_temp) == [lbm.LBM_T_DIRICHLET, lbm.LBM_T_DIRICHLET, lbm.LBM_T_ADIABATIC,
                               lbm.LBM_T_ADIABATIC]
    assert list(p.wall_T) == [1.0, 0.0, 0.0, 0.0]
    assert (p.zeta_q, p.zeta_eps, p.theta) == (1.9, 1.9, 1.0)
    assert p.collision == lbm.LBM_COLLISION_MRT


def test_abi_version_and_info():
    assert lbm.lib().lbm_abi_version() == 2
    assert b"gfx950" in lbm.lib().lbm_build_info()


@pytest.mark.parametrize("model,planes", [("d2q5", 14), ("d2q9t", 18), ("isothermal", 9)])
@pytest.mark.parametrize("storage,b", [(lbm.LBM_F64, 8), (lbm.LBM_F32, 4), (lbm.LBM_F16, 2)])
def test_required_bytes(storage, b, model, planes):
    # two buffers of ny rows; a row holds 9 + NG population rows, each
    # padded to 256 bytes; a buffer rounded up to 4 KiB
    for nx, ny in [(64, 64), (2048, 2048), (37, 23), (1, 1), (4096, 1024)]:
        seg = -(-nx * b // 256) * 256
        buf = -(-planes * seg * ny // 4096) * 4096
        assert lbm.lbm_required_bytes(nx, ny, storage, lbm.MODEL[model]) == 2 * buf


def test_required_bytes_rejects_bad_input():
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_required_bytes(0, 5, lbm.LBM_F64)
    assert e.value.code == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LbmError):
        lbm.lbm_required_bytes(5, 5, 7)
    assert b"lbm_required_bytes" in lbm.lib().lbm_last_error(None)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_required_bytes(5, 5, lbm.LBM_F64, 3)


def test_required_bytes_rejects_what_create_rejects():
    """Sizes lbm_create refuses get no byte count either: more than 2^31
    nodes, or a row of nodes of 2^31 elements or more (the kernels hold the
    row pitch in 32 bits)."""
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_required_bytes(65536, 32769, lbm.LBM_F64)
    assert e.value.code == lbm.LBM_ERR_ARG
    # D2Q5: 14 population rows of align(nx, 32) FP64 values
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_required_bytes(153391690, 1, lbm.LBM_F64)
    assert e.value.code == lbm.LBM_ERR_ARG
    assert b"2^31 elements" in lbm.lib().lbm_last_error(None)
    assert lbm.lbm_required_bytes(153391680, 1, lbm.LBM_F64) == 2 * (-(-14 * 153391680 * 8 // 4096) * 4096)
    # large lattices are limited by device memory only
    assert lbm.lbm_required_bytes(32768, 16384, lbm.LBM_F64) == 2 * 14 * 32768 * 16384 * 8


def test_create_rejects_bad_arguments_before_touching_a_device():
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(0, 4, lbm.LBM_F64)
    assert e.value.code == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(4, 4, 9)
    assert e.value.code == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(4, 4, lbm.LBM_F64, 5)
    assert e.value.code == lbm.LBM_ERR_ARG
    with pytest.raises(lbm.LbmError):
        lbm.lbm_create_ext(4, 4, lbm.LBM_F64, 0, 0, 0)


def test_null_handles_are_rejected():
    L = lbm.lib()
    assert L.lbm_step(None, 1) == lbm.LBM_ERR_ARG
    assert L.lbm_set_params(None, None) == lbm.LBM_ERR_ARG
    assert L.lbm_synchronize(None) == lbm.LBM_ERR_ARG
    L.lbm_destroy(None)


def test_problem_marshalling():
    from paper_1510_08224_amd import workloads as W
    pb = W.rayleigh_benard(64, 32, 1e5)
    p = lbm.lbm_params_from_problem(pb)
    assert p.ra == 1e5 and p.u_c == 0.1 and list(p.bc_flow) == [0, 0, 1, 1]
    assert list(p.bc_temp) == [0, 0, 1, 1] and list(p.wall_T) == [0.0, 0.0, 1.0, 0.0]


def test_rate_for_reynolds_matches_the_oracle():
    """The library's Reynolds-number rate map (Sec. 3.2) against the
    oracle's, which its own pin ties to Re = L u / nu."""
    import oracle
    for re, length, u in [(1000.0, 2048, 0.1), (1200.0, 79, 0.1), (100.0, 72, 0.1), (3.5, 10, 0.05)]:
        s = lbm.lbm_rate_for_reynolds(re, length, u)
        assert 0 < s < 2
        assert abs(s - oracle.rate_for_reynolds(re, length, u)) <= 1e-15 * s
    for bad in [(0.0, 10, 0.1), (100.0, 0, 0.1), (100.0, 10, 0.0), (float("nan"), 10, 0.1),
                (float("inf"), 10, 0.1), (-1.0, 10, 0.1)]:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_rate_for_reynolds(*bad)
        assert e.value.code == lbm.LBM_ERR_ARG
