"""CPU checks of the C ABI: the library loads, exports every declared entry point, and the
host-only entry points behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2403_08084_amd as P

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "irk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irk_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libirk.so not built")
    lib = ctypes.CDLL(P.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(P.SYMBOLS)


def test_options_default():
    o = P.default_options()
    assert o.precond == P.PC_GS_LOWER and o.restart == 30 and o.rtol == 1e-10
    assert o.orth == P.ORTH_DCGS2 and o.splitting == P.SPLIT_AI and o.stage_type == P.STAGE_COUPLED
    assert o.lookahead == P.LOOKAHEAD_ADAPTIVE
    assert o.cheb_degree == 2 and o.cheb_lo == 0.25 and o.cheb_hi == 1.1
    assert o.mg_precision == P.F64 and o.use_graphs == 1 and o.basis_f64 == 0
    with pytest.raises(TypeError):
        P.default_options(nonsense=1)


def test_revolve_schedule_host():
    from oracle import revolve

    acts, adv = P.revolve_schedule(40, 8)
    assert adv == 70 == revolve.min_advances_dp(40, 8)
    acts, adv = P.revolve_schedule(10, 10)
    assert adv == 9
    with pytest.raises(P.IrkError) as e:
        P.revolve_schedule(5, 0)
    assert e.value.code == P.IRK_EINVAL


def test_argument_validation_before_device_work():
    L = P.lib()
    h = ctypes.c_void_p()
    assert L.irk_problem_create(ctypes.byref(h), 1, ctypes.c_void_p(8), None) == P.IRK_EINVAL
    assert b"N must be" in L.irk_last_error()
    assert L.irk_problem_create(ctypes.byref(h), 16, None, None) == P.IRK_EINVAL
    assert L.irk_problem_create(None, 16, ctypes.c_void_p(8), None) == P.IRK_EINVAL
    assert L.irk_advance(None, None, None, 1, None, None) == P.IRK_EINVAL
    assert L.irk_stepper_sizes(None, None, None, None) == P.IRK_EINVAL
    assert L.irk_kernel_timer(None, 0, 1) == P.IRK_EINVAL
    # the copy reference: a negative length, NULL vectors and overlapping vectors are refused before any launch;
    # an empty copy does nothing
    assert L.irk_device_copy(ctypes.c_void_p(64), ctypes.c_void_p(4096), -1, None) == P.IRK_EINVAL
    assert L.irk_device_copy(None, ctypes.c_void_p(4096), 4, None) == P.IRK_EINVAL
    assert L.irk_device_copy(ctypes.c_void_p(64), ctypes.c_void_p(64 + 8 * 3), 4, None) == P.IRK_EINVAL
    assert b"overlap" in L.irk_last_error()
    assert L.irk_device_copy(None, None, 0, None) == P.IRK_OK


def test_product_tableaux_match_oracle_collocation():
    import numpy as np

    from oracle import tableaux as OT

    for s in (1, 2, 3, 4):
        for a, b in ((P.tableaux.radau_iia(s), OT.radau_iia(s)), (P.tableaux.gauss_legendre(s), OT.gauss_legendre(s))):
            for k in ("A", "b", "c"):
                assert np.abs(a[k] - b[k]).max() < 1e-13
    for a, b in ((P.tableaux.alexander(), OT.alexander()), (P.tableaux.wsodirk433(), OT.wsodirk433()),
                 (P.tableaux.lobatto_iiic2(), OT.lobatto_iiic2())):
        for k in ("A", "b", "c"):
            assert np.abs(a[k] - b[k]).max() < 1e-8
