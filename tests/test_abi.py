"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/frelbm.h declares, and validates parameters on the host (no GPU call)."""
import ctypes as C
import os
import re

import pytest

from paper_2212_01617_amd import frelbm as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "frelbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fre_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(F.LIB_PATH):
        from paper_2212_01617_amd import build
        build.build()
    return F.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in F._SIGS}
    assert set(names) <= bound


def _ok_params(**kw):
    base = dict(A=0.04, kappa=0.09)
    base.update(kw)
    return F.make_params(F.FRE_D3Q19, (16, 8, 8), **base)


def test_footprint_host_only(lib):
    n32 = F.footprint(_ok_params())
    n16 = F.footprint(_ok_params(storage=F.FRE_FP16))
    assert n32 > n16 > 16 * 8 * 8 * 19 * 2 * 2


@pytest.mark.parametrize("bad,msg", [
    (dict(tau_f=0.5), "tau"),
    (dict(tau_g=0.4), "tau"),
    (dict(M=0.0), "mobility"),
    (dict(A=-1.0), "A and kappa"),
    (dict(wall_u=[[[0.2, 0, 0], [0, 0, 0]], [[0] * 3] * 2, [[0] * 3] * 2]), "Mach"),
    (dict(storage=7), "storage"),
])
def test_validation_errors(lib, bad, msg):
    with pytest.raises(F.FreError) as ei:
        F.footprint(_ok_params(**bad))
    assert ei.value.status == F.FRE_EINVAL
    assert msg in str(ei.value)


@pytest.mark.parametrize("bad,msg", [
    (dict(ternary=(0.0, 0.05, 1.0)), "kappa3"),
    (dict(ternary=(0.1, -0.1, 1.0)), "M3"),
    (dict(ternary=(0.1, 0.05, 0.5)), "tau_h"),
    (dict(ternary=(0.1, 0.05, 1.0), storage=F.FRE_FP16), "FP32"),
])
def test_ternary_validation_errors(lib, bad, msg):
    with pytest.raises(F.FreError) as ei:
        F.footprint(_ok_params(**bad))
    assert ei.value.status == F.FRE_EINVAL
    assert msg in str(ei.value)


def test_ternary_flag_is_0_or_1(lib):
    p = _ok_params()
    p.ternary = 2
    with pytest.raises(F.FreError) as ei:
        F.footprint(p)
    assert ei.value.status == F.FRE_EINVAL


@pytest.mark.parametrize("bad", [
    dict(stochastic_rounding=True),                                                   # FP32 storage
    dict(stochastic_rounding=True, storage=F.FRE_FP16, ternary=(0.1, 0.05, 1.0)),     # ternary
])
def test_stochastic_rounding_needs_binary_fp16(lib, bad):
    with pytest.raises(F.FreError) as ei:
        F.footprint(_ok_params(**bad))
    assert ei.value.status == F.FRE_EINVAL
    assert "fp16_rounding" in str(ei.value) or "FP32" in str(ei.value)
    p = _ok_params(storage=F.FRE_FP16)
    p.fp16_rounding = 2
    with pytest.raises(F.FreError) as ei:
        F.footprint(p)
    assert ei.value.status == F.FRE_EINVAL
    # accepted with FP16 storage, and the counter adds to the footprint
    assert F.footprint(_ok_params(storage=F.FRE_FP16, stochastic_rounding=True)) > F.footprint(
        _ok_params(storage=F.FRE_FP16))


def test_ternary_footprint_holds_the_third_population(lib):
    q, n = 19, 16 * 8 * 8
    assert F.footprint(_ok_params(ternary=(0.1, 0.05, 1.0))) >= F.footprint(_ok_params()) + q * n * 4 - 64 * n
    p = _ok_params(ternary=(0.1, 0.05, 1.0))
    out = C.c_void_p(1)
    # the binary entry point refuses ternary parameters before touching memory
    assert lib.fre_lattice_init(C.byref(p), None, 0, None, None, None, None, None, C.byref(out)) == F.FRE_EINVAL
    assert out.value is None and b"fre_lattice_init3" in lib.fre_last_error()
    b = _ok_params()
    assert lib.fre_lattice_init3(C.byref(b), None, 0, None, None, None, None, None, None,
                                 C.byref(out)) == F.FRE_EINVAL
    assert out.value is None


def test_d2q9_shape_rules(lib):
    with pytest.raises(F.FreError):
        F.footprint(F.make_params(F.FRE_D2Q9, (8, 8, 2), A=0.04, kappa=0.09))
    assert F.footprint(F.make_params(F.FRE_D2Q9, (8, 8, 1), A=0.04, kappa=0.09)) > 0


def test_null_arguments(lib):
    assert lib.fre_step(None, 1) == F.FRE_EINVAL
    assert b"NULL" in lib.fre_last_error()
    lib.fre_lattice_destroy(None)
