"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, validates arguments, and its pure-host figures of merit match the
oracle.  No GPU is touched (every call here returns before any HIP call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "piezohom.h")
LIB = os.path.join(ROOT, "paper_2410_03148_amd", "libpiezohom.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(phz_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(LIB)
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_lists_every_symbol():
    import paper_2410_03148_amd as P
    assert sorted(P.EXPORTS) == declared_symbols()


def test_create_rejects_bad_sizes_and_materials():
    import synth
    import paper_2410_03148_amd as P
    m = P.make_material(synth.material_workload())
    h = C.c_void_p()
    for n in (0, 1, 3, 7, 2048):
        assert P._lib.phz_create(n, n, n, C.byref(m), None, None, None, C.byref(h)) == -1
    # halving must end at a side of at most 10 (dense coarsest inverse)
    for n in (22, 100, 120):
        assert P._lib.phz_create(n, n, n, C.byref(m), None, None, None, C.byref(h)) == -1
    o = P.default_options(mg_levels=2)
    assert P._lib.phz_create(64, 64, 64, C.byref(m), C.byref(o), None, None, C.byref(h)) == -1
    bad = P.make_material(synth.material_workload())
    bad.C[0] = float("nan")
    assert P._lib.phz_create(8, 8, 8, C.byref(bad), None, None, None, C.byref(h)) == -2
    bad2 = P.make_material(synth.material_workload())
    bad2.void_scale = 0.0
    assert P._lib.phz_create(8, 8, 8, C.byref(bad2), None, None, None, C.byref(h)) == -1
    assert P._lib.phz_create(8, 8, 8, C.byref(m), None, None, None, None) == -1
    # the cell must be cubic
    for dims in ((8, 8, 16), (8, 16, 8), (16, 8, 8)):
        assert P._lib.phz_create(*dims, C.byref(m), None, None, None, C.byref(h)) == -1
        assert not h.value
    # an allocator needs both callbacks
    half = P.phz_allocator()
    assert P._lib.phz_create(8, 8, 8, C.byref(m), None, None, C.byref(half), C.byref(h)) == -1


def test_strerror_and_defaults():
    import paper_2410_03148_amd as P
    assert P._lib.phz_strerror(0) == b"ok"
    assert P._lib.phz_strerror(-2) == b"NaN or Inf"
    o = P.default_options()
    assert o.restart == 30 and o.rtol == 1e-10 and o.batched == 1 and o.cheby_degree == 2
    assert list(o.block_kernel) == [-1] * 4 and list(o.block_tile) == [-1] * 4
    assert o.bf16_terms == 3 and o.bf16_terms_precond == 1


def test_options_rejected_before_device_use():
    """phz_create validates the options before it touches a device, so bad
    per-block pins fail on a host without a GPU."""
    import ctypes as C
    import synth
    import paper_2410_03148_amd as P
    m = P.make_material(synth.material_workload())
    h = C.c_void_p()
    for field, val in (("block_kernel", [0, 3, -1, -1]), ("block_kernel", [-2, 0, 0, 0]),
                       ("block_tile", [0, 0, 0, 3]), ("fine_kernel", 5), ("elem_tile", 7), ("solver", -1),
                       ("inner", 2), ("inner_eps", 0.0), ("inner_eps", 1.0), ("inner_maxit", 0),
                       ("warm_start", 2), ("solver", 3), ("smoothing", 2), ("bf16_terms_precond", 2),
                       ("bf16_terms_precond", 0), ("coarse_kernel", 3), ("coarse_kernel", -2)):
        o = P.default_options(**{field: val})
        assert P._lib.phz_create(16, 16, 16, C.byref(m), C.byref(o), None, None, C.byref(h)) == -1, field
        assert not h.value
    # TriCG runs in float64 only, and with element smoothing
    o = P.default_options(solver=P.PHZ_SOLVER_TRICG, precision=P.PHZ_FP32_IR)
    assert P._lib.phz_create(16, 16, 16, C.byref(m), C.byref(o), None, None, C.byref(h)) == -1
    o = P.default_options(solver=P.PHZ_SOLVER_TRICG, precision=P.PHZ_FP64, smoothing=P.PHZ_SMOOTH_QP)
    assert P._lib.phz_create(16, 16, 16, C.byref(m), C.byref(o), None, None, C.byref(h)) == -1
    with pytest.raises(ValueError):
        P.default_options(block_tile=[0, 1])


@pytest.mark.parametrize("name", ["d_h", "g_h", "B_voigt", "B_reuss", "k_h"])
def test_foms_match_oracle(name):
    """phz_foms is host code: values and closed-form gradients vs the oracle's
    definitions and complex-step gradients."""
    import synth
    import paper_2410_03148_amd as P
    from oracle import cell, foms
    r = cell.homogenise(6, synth.material_workload(), phi=synth.grf_levelset(6, seed=3), want_x=False)
    f, (gC, ge, gk) = P.foms(r.C, r.e, r.kappa, grad_of=name)
    fo = foms.foms(r.C, r.e, r.kappa)
    for k in fo:
        assert abs(f[k] - fo[k]) <= 1e-12 * abs(fo[k])
    oC, oe, ok = foms.fom_grads(r.C, r.e, r.kappa, name)
    for a, b in ((gC, oC), (ge, oe), (gk, ok)):
        assert np.abs(a - b).max() <= 1e-9 * max(np.abs(b).max(), 1e-300)


def test_foms_paper_base_value():
    import synth
    import paper_2410_03148_amd as P
    m = synth.material_pzt5a()
    f = P.foms(m.C, m.e, m.kappa)
    assert 31.7 <= f["d_h"] * 1e12 < 31.8
