"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol include/tdgrad.h declares, and rejects bad input before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from tests import molecules

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tdg():
    from paper_2407_16586_amd import build, tdgrad
    if not os.path.exists(tdgrad.LIB_PATH):
        build.build()
    return tdgrad


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "tdgrad.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdg_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(tdg):
    names = _declared_functions()
    assert len(names) >= 6
    L = C.CDLL(tdg.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(tdg.EXPORTED) == set(names)


def test_class_table():
    from paper_2407_16586_amd import tdgrad
    assert len(tdgrad.CLASSES) == 21
    for la, lb, lc, ld in tdgrad.CLASSES:
        assert la >= lb and lc >= ld and (la, lb) >= (lc, ld)
        assert la == max(la, lb, lc, ld)   # highest momentum on the centre skipped by TI


def test_unsupported_angular_momentum(tdg):
    m = molecules.make([[0, 0, 0], [1.5, 0, 0]], [(0, 0, [1.0], [1.0]), (1, 3, [0.5], [1.0])])
    with pytest.raises(tdg.TdgError) as e:
        tdg.Plan(m)
    assert e.value.status == tdg.TDG_EUNSUPPORTED
    assert "l=3" in str(e.value)


def test_too_many_primitives(tdg):
    m = molecules.make([[0, 0, 0]], [(0, 0, list(np.linspace(1, 20, 17)), [1.0] * 17)])
    with pytest.raises(tdg.TdgError) as e:
        tdg.Plan(m)
    assert e.value.status == tdg.TDG_EUNSUPPORTED


def test_bad_indices_and_exponents(tdg):
    m = molecules.make([[0, 0, 0]], [(0, 0, [1.0], [1.0])])
    m.shell_atom = np.array([3], dtype=np.int32)
    with pytest.raises(tdg.TdgError) as e:
        tdg.Plan(m)
    assert e.value.status == tdg.TDG_EINVAL
    m = molecules.make([[0, 0, 0]], [(0, 0, [-1.0], [1.0])])
    with pytest.raises(tdg.TdgError) as e:
        tdg.Plan(m)
    assert e.value.status == tdg.TDG_EINVAL


def test_spherical_flag_checked(tdg):
    m = molecules.make([[0, 0, 0]], [(0, 2, [1.0], [1.0])])
    m.spherical = 2
    with pytest.raises(tdg.TdgError) as e:
        tdg.Plan(m)
    assert e.value.status == tdg.TDG_EINVAL


def test_null_arguments(tdg):
    L = tdg.lib()
    assert L.tdg_plan_create(None, None, 0, None) == tdg.TDG_EINVAL
    assert L.tdg_grad_jk(None, None, None, None, 0, None, None, None) == tdg.TDG_EINVAL
    assert L.tdg_plan_destroy(None) == tdg.TDG_OK
    assert b"null" in L.tdg_last_error()
    assert L.tdg_fock(None, None, 0, None, 1.0, 0.0, 0.0, 0, None, None) == tdg.TDG_EINVAL
    assert L.tdg_last_error()


def test_long_range_needs_omega(tdg):
    m = molecules.make([[0, 0, 0], [1.5, 0, 0]], [(0, 0, [1.0], [1.0]), (1, 0, [0.5], [1.0])])
    with pytest.raises(tdg.TdgError) as e:
        tdg.Plan(m, omega=0.0)
    assert e.value.status == tdg.TDG_EINVAL


def test_rys_rule_argument_checks(tdg):
    u = np.zeros(6); w = np.zeros(6)
    assert tdg.lib().tdg_rys_rule(6, 1.0, u.ctypes.data, w.ctypes.data) == tdg.TDG_EINVAL
    assert tdg.lib().tdg_rys_rule(2, -1.0, u.ctypes.data, w.ctypes.data) == tdg.TDG_EINVAL
