"""The C-ABI library loads, exports every symbol include/rt.h declares, and its
host-only logic behaves (no kernel launches: these run without a GPU)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle import angular_grid as AG
from paper_2302_04283_amd import rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rt.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(rt_\w+)\s*\(", src, re.M)))


def test_library_exports_declared_symbols():
    lib = rt.load()
    names = _declared()
    assert "rt_step" in names and "rt_init_grid" in names and "rt_moments" in names
    for name in names:
        assert hasattr(lib, name), name


def test_host_error_paths():
    lib = rt.load()
    out = C.c_void_p()
    assert lib.rt_init_grid(None, 0, C.byref(out)) == rt.RT_EINVAL
    assert b"NULL" in lib.rt_last_error()
    assert lib.rt_geodesic_angles(0, None, None) == rt.RT_EINVAL
    assert lib.rt_step(None, None, None, None, None, None, None, None, None, 0.1, None,
                       None, None) == rt.RT_EINVAL
    assert lib.rt_step_noalloc(None, None, None, None, None, None, None, None, None, 0.1, None,
                               None, None) == rt.RT_EINVAL
    assert lib.rt_step_adjoint(None, None, None, None, None, None, None, None, 0.1, 1.0,
                               None, None, None, None, None, None, None, None) == rt.RT_EINVAL
    assert lib.rt_gas_update(None, None, None, None, None, None, None, None) == rt.RT_EINVAL
    dt = C.c_double()
    assert lib.rt_max_dt(None, 0.3, C.byref(dt)) == rt.RT_EINVAL
    lib.rt_free(None)


def test_bad_descriptor_rejected_before_device_use():
    d = rt.RtGridDesc()
    d.n[0] = 0
    out = C.c_void_p()
    assert rt.load().rt_init_grid(C.byref(d), 0, C.byref(out)) == rt.RT_EINVAL
    assert out.value is None
    assert "rad_velocity" in dict(rt.RtGridDesc._fields_)


@pytest.mark.parametrize("nlev", [1, 2, 3, 4, 5, 6, 7])
def test_library_angle_table_matches_oracle(nlev):
    nh, do = rt.geodesic_angles(nlev)
    g = AG.build(nlev)
    assert nh.shape == (10 * nlev * nlev + 2, 3)
    assert np.abs(nh - g.nhat).max() <= 1e-14
    assert np.abs(do - g.domega).max() <= 1e-14
    assert abs(do.sum() - 4 * math.pi) <= 1e-13


@pytest.mark.parametrize("nz,npsi", [(2, 4), (8, 16), (16, 32)])
def test_library_latlong_table_matches_oracle(nz, npsi):
    nh, do = rt.latlong_angles(nz, npsi)
    g = AG.build_latlong(nz, npsi)
    assert np.abs(nh - g.nhat).max() <= 1e-14
    assert np.abs(do - g.domega).max() <= 1e-14


@pytest.mark.parametrize("field,value,msg", [
    ("latlong", (3, 5), b"latitude-longitude"),
    ("latlong", (40, 16), b"latitude-longitude"),
    ("ang_recon", 1, b"ang_recon"),
    ("ang_recon", 3, b"ang_recon"),
    ("integrator", 3, b"integrator"),
    ("tau_coeff", -1.0, b"tau_coeff"),
    ("rad_velocity", 2, b"rad_velocity"),
])
def test_option_validation_before_device_use(field, value, msg):
    """Malformed scheme options are rejected by the descriptor check, before
    any device call (so this runs without a GPU)."""
    from paper_2302_04283_amd import workloads as W
    p = W.make_problem("c3", scale=(4, 4, 4), nlev=1)
    setattr(p, field, value)
    with pytest.raises(rt.RtError):
        rt.Grid(p, rt.RT_F64)
    assert msg in rt.load().rt_last_error()


def test_mapr_on_latlong_rejected_before_device_use():
    from paper_2302_04283_amd import workloads as W
    p = W.make_problem("c3", scale=(4, 4, 4), nlev=1)
    p.latlong, p.ang_recon = (4, 8), 2
    with pytest.raises(rt.RtError):
        rt.Grid(p, rt.RT_F64)
    assert b"ang_recon" in rt.load().rt_last_error()
