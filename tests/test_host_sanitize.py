"""The library's host-only code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU).

The descriptor checks, the geodesic and latitude-longitude grids, the MAPR
tables and the FP64 geometry tables (csrc/rt_desc.cpp, rt_geodesic.cpp,
rt_latlong.cpp, rt_mapr.cpp, rt_geometry.cpp) are built with g++
-fsanitize=address,undefined together with the harness tests/host_check.cpp,
and driven in a child Python process (the sanitizer runtime preloaded)
with the descriptors rt_init_grid receives for every workload family, the
options, and rejected descriptors.  Any sanitizer report aborts the child.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2302_04283_amd", "csrc")
HOST_SOURCES = ["rt_desc.cpp", "rt_geodesic.cpp", "rt_latlong.cpp", "rt_mapr.cpp", "rt_geometry.cpp"]


def _runtime(name):
    out = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


CHILD = r'''
import ctypes as C, sys
import numpy as np
sys.path.insert(0, sys.argv[2])
from paper_2302_04283_amd import rt
from paper_2302_04283_amd import workloads as W

lib = C.CDLL(sys.argv[1])
lib.rt_host_check.argtypes = [C.c_void_p, C.c_char_p, C.c_int]
lib.rt_host_angles.argtypes = [C.c_int, C.c_int, C.c_int, C.c_char_p, C.c_int]
buf = C.create_string_buffer(512)

for lev in range(1, 8):
    assert lib.rt_host_angles(lev, 0, 0, buf, 512) == rt.RT_OK, (lev, buf.value)
for nz, npsi in ((2, 2), (4, 8), (8, 16), (16, 32)):
    assert lib.rt_host_angles(0, nz, npsi, buf, 512) == rt.RT_OK, (nz, npsi, buf.value)

def check(p, prec=rt.RT_F64, expect=rt.RT_OK, edit=None):
    d, keep = rt.make_desc(p, prec, 0 if getattr(p, "beam_mask", None) is not None else None)
    if edit:
        edit(d)
    rc = lib.rt_host_check(C.byref(d), buf, 512)
    assert rc == expect, (rc, expect, buf.value)
    if expect != rt.RT_OK:
        assert buf.value, "rejected without a reason"
    return rc

cases = [W.make_problem("c1"), W.make_problem("c2", scale=(8, 6, 5)),
         W.make_problem("c3", scale=(10, 6, 4)), W.make_problem("c4", scale=(6, 4, 5)),
         W.make_problem("c5", scale=(4, 4, 3))]
ks_out = W.make_custom("ks_sph", (6, 4, 5), [(2.0, 6.0), (1.0, 2.0), (0.0, 0.7)], 3,
                       [(1, 1), (1, 1), (1, 1)], M=1.0, a=0.9)
cases.append(ks_out)
mapr = W.make_problem("c3", scale=(6, 4, 3)); mapr.ang_recon = 2
cases.append(mapr)
ll = W.make_problem("c3", scale=(6, 4, 3)); ll.latlong = (6, 12); ll.ang_recon = 1
cases.append(ll)
opts = W.make_problem("c2", scale=(5, 4, 4))
opts.integrator, opts.tau_coeff, opts.rad_velocity = 2, 5.0, 1
cases.append(opts)
for p in cases:
    for prec in (rt.RT_F64, rt.RT_F32):
        check(p, prec)
print("host tables ok:", len(cases), "problems", flush=True)

p = W.make_problem("c4", scale=(6, 4, 5))
def setf(name, val):
    def f(d):
        setattr(d, name, val)
    return f
def set_n(d):
    d.n[0] = 0
def set_bc(d):
    d.bc[1][0] = 7
def half_periodic(d):
    d.bc[2][1] = 1 - d.bc[2][0]
def geo_extent(d):
    d.geo_extent[0] = 3
for edit in (setf("nlev", 0), setf("nlev", 8), setf("precision", 5), setf("recon", 9),
             setf("lum_axis", 3), setf("gamma_gas", 1.0), setf("integrator", 3),
             setf("tau_coeff", -1.0), setf("rad_velocity", 2), setf("kernel", 3),
             setf("seglen", -1), setf("ang_recon", 1), setf("n_zeta", 3), set_n, set_bc,
             half_periodic, geo_extent):
    check(p, rt.RT_F32, rt.RT_EINVAL, edit)
def neg_vol(d):
    d.vol[0] = -1.0
check(p, rt.RT_F32, rt.RT_EGEOM, neg_vol)
print("descriptor checks ok", flush=True)
'''


def test_host_code_under_address_and_undefined_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("g++ has no sanitizer runtime here")
    with tempfile.TemporaryDirectory() as tmp:
        so = os.path.join(tmp, "libhostcheck.so")
        cmd = (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-shared", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] +
               [os.path.join(CSRC, s) for s in HOST_SOURCES] +
               [os.path.join(ROOT, "tests", "host_check.cpp"), "-o", so])
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ)
        env["LD_PRELOAD"] = asan + ":" + ubsan
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        r = subprocess.run([sys.executable, "-c", CHILD, so, ROOT], capture_output=True, text=True,
                           env=env, timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
        assert "host tables ok" in out and "descriptor checks ok" in out, out[-2000:]
