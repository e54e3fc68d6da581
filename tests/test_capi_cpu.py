"""Host-side checks of the C ABI (no GPU work): the library loads and exports every function
that include/phasefield.h declares, parameter validation rejects bad input before touching the
device, and phasefield_check_params states the paper's criteria (Eq. 17, Eqs. 25 and 28)."""
import os
import re

import pytest

from oracle import params as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "phasefield.h")).read()
    return sorted(set(re.findall(r"\b(phasefield_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def pf():
    import paper_1803_01262_amd as pf
    return pf


def test_library_exports_every_declared_symbol(pf):
    names = header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(pf.lib, n), n  # ctypes resolves the symbol from the .so
    assert sorted(pf.EXPORTED) == names
    for n in names:
        assert callable(getattr(pf, n)), n


def test_default_params(pf):
    p = pf.phasefield_default_params()
    assert tuple(p.n) == (1, 1, 1) and p.dtype == pf.PF_F64 and p.scheme == pf.PF_RK4
    assert p.variant == -1 and p.use_graph == 1 and p.vel_mode == pf.PF_VEL_STEADY


@pytest.mark.parametrize("field,value", [("dx", 0.0), ("dx", -1.0), ("eps", -0.1),
                                         ("gamma", -1.0), ("dt", 0.0), ("delta", -1.0),
                                         ("dtype", 7), ("scheme", 5), ("vel_mode", 3),
                                         ("variant", 999)])
def test_invalid_params_rejected_before_device_work(pf, field, value):
    p = pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01)
    setattr(p, field, value)
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf.phasefield_create(p)
    assert ei.value.status == pf.PF_ERR_INVALID
    assert pf.phasefield_last_error()


def test_invalid_sizes_and_bcs(pf):
    p = pf.make_params((8, 0, 8), 0.1, 0.1, 1.0, 0.01)
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf.phasefield_create(p)
    assert ei.value.status == pf.PF_ERR_INVALID
    p = pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01, vel_mode=1, vel_T=0.0)
    with pytest.raises(pf.PhaseFieldError):
        pf.phasefield_create(p)
    p = pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01)
    p.bc[2] = 5
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf.phasefield_create(p)
    assert ei.value.status == pf.PF_ERR_INVALID
    # walls validate (the single-grid solver and the batched driver run them); the batched
    # driver declines mixed schemes and a time-varying velocity before any device work
    pw = pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01, walls=(False, False, True))
    assert pw.bc[2] == pf.PF_BC_WALL
    r = pf.phasefield_check_params(pw, 1.0)
    assert r.dt_max_scheme > 0
    for scheme in ("euler", "rk2", "rk3"):
        with pytest.raises(pf.PhaseFieldError) as ei:
            pf.phasefield_batch_create([pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01),
                                        pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01,
                                                       scheme=scheme)])
        assert ei.value.status == pf.PF_ERR_UNSUPPORTED
        assert "mixed schemes" in pf.phasefield_last_error()
    with pytest.raises(pf.PhaseFieldError) as ei:
        pf.phasefield_batch_create([pf.make_params((8, 8, 8), 0.1, 0.1, 1.0, 0.01, vel_mode=1)])
    assert ei.value.status == pf.PF_ERR_UNSUPPORTED


@pytest.mark.parametrize("n,scheme", [((64, 64, 1), "rk4"), ((32, 32, 32), "rk4"),
                                      ((50, 1, 1), "euler"), ((20, 30, 1), "euler"),
                                      ((40, 1, 1), "rk2"), ((16, 16, 16), "rk2"),
                                      ((30, 20, 1), "rk3"), ((12, 12, 12), "rk3")])
def test_check_params_states_eq17_and_dt_limits(pf, n, scheme):
    dx, eps, gamma, umax = 0.02, 0.017, 1.3, 0.9
    p = pf.make_params(n, dx, eps, gamma, 1e-4, scheme=scheme)
    r = pf.phasefield_check_params(p, umax)
    dims = sum(v > 1 for v in n)
    assert r.crossover_margin_eq17 == pytest.approx(P.margin_eq17(eps, dx, gamma, umax), rel=1e-14)
    assert r.dt_max_scheme == pytest.approx(P.dt_max(scheme, dims, dx, gamma, eps), rel=1e-14)
    assert r.dt_over_dtmax == pytest.approx(1e-4 / r.dt_max_scheme, rel=1e-14)


def test_variant_table(pf):
    nv = pf.phasefield_variant_count(pf.PF_F64)
    assert nv >= 2
    names = [pf.phasefield_variant_name(pf.PF_F64, v) for v in range(nv)]
    assert all(names) and len(set(names)) == nv
    assert pf.phasefield_variant_name(pf.PF_F64, nv) is None


def test_noalloc_step_refuses_oversized_grid_on_the_host(pf):
    """phasefield_step_noalloc checks the grid against its fixed scratch array before any device
    work (the pointers here are never dereferenced)."""
    import ctypes
    assert pf.phasefield_noalloc_scratch_bytes() == 64 << 20
    for n, dtype in ((150, "f64"), (190, "f32")):
        p = pf.make_params((n, n, n), 1.0 / n, 1.0 / n, 1.0, 1e-4, dtype=dtype)
        fake = ctypes.c_void_p(256)
        st = pf.lib.phasefield_step_noalloc(ctypes.byref(p), fake, fake, fake, fake, 0.0, 1, None)
        assert st == pf.PF_ERR_INVALID
        assert "scratch" in pf.phasefield_last_error()
    p = pf.make_params((8, 8, 8), 0.0, 0.1, 1.0, 0.01)  # dx = 0: parameter check first
    st = pf.lib.phasefield_step_noalloc(ctypes.byref(p), fake, fake, fake, fake, 0.0, 1, None)
    assert st == pf.PF_ERR_INVALID


def test_adjoint_form_setter_checks_its_arguments(pf):
    assert pf.lib.phasefield_set_adjoint_form(None, 0) == pf.PF_ERR_INVALID
    assert "NULL" in pf.phasefield_last_error()


def test_stage_entry_points_check_the_handle(pf):
    assert pf.lib.phasefield_step_stages(None, None, None, None, None, None, 0.0, None, None,
                                         None, None) == pf.PF_ERR_INVALID
    assert pf.lib.phasefield_adjoint_step_stages(None, None, None, None, None, None, None, None,
                                                 0.0, None, None, None, None,
                                                 None) == pf.PF_ERR_INVALID


def test_batch_shape_and_autotune_check_their_arguments(pf):
    import ctypes
    assert pf.lib.phasefield_batch_set_shape(None, 0) == pf.PF_ERR_INVALID
    bs, bp = ctypes.c_int32(), ctypes.c_int32()
    assert pf.lib.phasefield_batch_autotune(None, 1, ctypes.byref(bs), ctypes.byref(bp), None,
                                            None) == pf.PF_ERR_INVALID
