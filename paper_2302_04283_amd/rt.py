"""Python binding of the HIP radiation-step library (ctypes over include/rt.h).

Argument marshalling only: every step of the method runs in the library's
kernels.  PyTorch provides device memory and the current HIP stream.  If the
compiled library is missing the import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpaper_rt.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_EGEOM = 0, -1, -2, -3, -4
RT_F64, RT_F32 = 0, 1
RT_RECON_DC, RT_RECON_PLM = 0, 1
RT_BC_PERIODIC, RT_BC_OUTFLOW_VACUUM = 0, 1

_dp = C.POINTER(C.c_double)


class RtGridDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("geo_extent", C.c_int32 * 3),
        ("nlev", C.c_int32),
        ("precision", C.c_int32),
        ("recon", C.c_int32),
        ("bc", (C.c_int32 * 2) * 3),
        ("lum_axis", C.c_int32),
        ("lum_side", C.c_int32),
        ("n0_crit", C.c_double),
        ("a_rad", C.c_double),
        ("gamma_gas", C.c_double),
        ("kb_mu_mp", C.c_double),
        ("x_faces", _dp * 3),
        ("vol", _dp),
        ("area", _dp * 3),
        ("gcov_c", _dp),
        ("dgcov_c", _dp),
        ("tet_c", _dp),
        ("dtet_c", _dp),
        ("gcov_f", _dp * 3),
        ("tet_f", _dp * 3),
        ("beam_mask", C.POINTER(C.c_uint8)),
        ("beam_I", C.c_double),
        ("beam_angle", C.c_int32),
        ("integrator", C.c_int32),
        ("tau_coeff", C.c_double),
        ("rad_velocity", C.c_int32),
        ("n_zeta", C.c_int32),
        ("n_psi", C.c_int32),
        ("ang_recon", C.c_int32),
        ("kernel", C.c_int32),
        ("seglen", C.c_int32),
    ]


class RtError(RuntimeError):
    pass


_LIB = None


def load():
    """Load the compiled library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RtError("HIP library %s is missing: run __graft_entry__.build() "
                      "(or python -m paper_2302_04283_amd.build)" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.rt_init_grid.argtypes = [C.POINTER(RtGridDesc), C.c_int, C.POINTER(vp)]
    lib.rt_geodesic_angles.argtypes = [C.c_int32, _dp, _dp]
    lib.rt_grid_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]
    lib.rt_angles.argtypes = [vp, _dp, _dp]
    lib.rt_max_dt.argtypes = [vp, C.c_double, _dp]
    lib.rt_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_double, vp, vp, vp]
    lib.rt_step_noalloc.argtypes = lib.rt_step.argtypes
    lib.rt_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.rt_step_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.c_double, C.c_double,
                                    vp, vp, vp, vp, vp, vp, vp, vp]
    lib.rt_stats.argtypes = [vp, C.POINTER(C.c_int64), _dp]
    lib.rt_gas_update.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.rt_latlong_angles.argtypes = [C.c_int32, C.c_int32, _dp, _dp]
    lib.rt_free.argtypes = [vp]
    lib.rt_free.restype = None
    lib.rt_last_error.restype = C.c_char_p
    for f in ("rt_init_grid", "rt_geodesic_angles", "rt_grid_info", "rt_angles",
              "rt_max_dt", "rt_step", "rt_step_noalloc", "rt_moments", "rt_stats", "rt_step_adjoint",
              "rt_gas_update", "rt_latlong_angles"):
        getattr(lib, f).restype = C.c_int
    _LIB = lib
    return lib


def _check(rc):
    if rc != RT_OK:
        raise RtError("rt error %d: %s" % (rc, load().rt_last_error().decode()))


def _ptr(a):
    return a.ctypes.data_as(_dp)


def geodesic_angles(nlev: int):
    """(nhat [nang,3], domega [nang]) of the library's grid, host numpy."""
    lib = load()
    nang = 10 * nlev * nlev + 2
    nh = np.zeros((nang, 3))
    do = np.zeros(nang)
    _check(lib.rt_geodesic_angles(nlev, _ptr(nh), _ptr(do)))
    return nh, do


def latlong_angles(n_zeta: int, n_psi: int):
    """(nhat [nang,3], domega [nang]) of the library's latitude-longitude grid."""
    lib = load()
    nh = np.zeros((n_zeta * n_psi, 3))
    do = np.zeros(n_zeta * n_psi)
    _check(lib.rt_latlong_angles(int(n_zeta), int(n_psi), _ptr(nh), _ptr(do)))
    return nh, do


def beam_direction(nlev: int, latlong=None) -> int:
    """Direction with the largest x^1 component (the c2 beam)."""
    nh, _ = latlong_angles(*latlong) if latlong is not None else geodesic_angles(nlev)
    return int(np.argmax(nh[:, 0]))


def _dev(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def make_desc(prob, precision, beam_angle=None):
    """The rt_grid_desc of a problem and the host arrays it points into
    (keep them alive while the descriptor is in use)."""
    keep = []

    def arr(x, dtype=np.float64):
        a = np.ascontiguousarray(x, dtype=dtype)
        keep.append(a)
        return a

    d = RtGridDesc()
    for a in range(3):
        d.n[a] = int(prob.n[a])
        d.geo_extent[a] = int(prob.geo_extent[a])
        d.bc[a][0] = int(prob.bc[a][0])
        d.bc[a][1] = int(prob.bc[a][1])
        d.x_faces[a] = _ptr(arr(prob.x_faces[a]))
        d.area[a] = _ptr(arr(prob.area[a]))
        d.gcov_f[a] = _ptr(arr(prob.gcov_f[a]))
        d.tet_f[a] = _ptr(arr(prob.tet_f[a]))
    d.nlev = int(prob.nlev)
    d.precision = int(precision)
    d.recon = int(prob.recon)
    d.lum_axis = int(prob.lum_axis)
    d.lum_side = int(prob.lum_side)
    d.n0_crit = float(prob.n0_crit)
    d.a_rad = float(prob.a_rad)
    d.gamma_gas = float(prob.gamma_gas)
    d.kb_mu_mp = float(prob.kb_mu_mp)
    d.integrator = int(getattr(prob, "integrator", 1))
    d.tau_coeff = float(getattr(prob, "tau_coeff", 0.0))
    d.rad_velocity = int(getattr(prob, "rad_velocity", 0))
    ll = getattr(prob, "latlong", None)
    if ll is not None:
        d.n_zeta, d.n_psi = int(ll[0]), int(ll[1])
    d.ang_recon = int(getattr(prob, "ang_recon", 0))
    d.kernel = int(getattr(prob, "kernel", 0))
    d.seglen = int(getattr(prob, "seglen", 0))
    d.vol = _ptr(arr(prob.vol))
    d.gcov_c = _ptr(arr(prob.gcov_c))
    d.dgcov_c = _ptr(arr(prob.dgcov_c))
    d.tet_c = _ptr(arr(prob.tet_c))
    d.dtet_c = _ptr(arr(prob.dtet_c))
    if getattr(prob, "beam_mask", None) is not None:
        bm = arr(prob.beam_mask, np.uint8)
        d.beam_mask = bm.ctypes.data_as(C.POINTER(C.c_uint8))
        d.beam_I = float(prob.beam_I)
        d.beam_angle = int(beam_angle)
    return d, keep


class Grid:
    """A problem's device tables; ``step``/``moments`` launch on the current stream."""

    def __init__(self, prob, precision=RT_F32, device: int = 0):
        import torch  # noqa: F401  (device memory comes from torch)
        lib = load()
        self.beam_angle = None
        if getattr(prob, "beam_mask", None) is not None:
            self.beam_angle = beam_direction(prob.nlev, getattr(prob, "latlong", None))
        d, keep = make_desc(prob, precision, self.beam_angle)
        h = C.c_void_p()
        _check(lib.rt_init_grid(C.byref(d), int(device), C.byref(h)))
        self._h = h
        self._lib = lib
        self.device = device
        self.precision = precision
        self.n = tuple(int(v) for v in prob.n)
        na, ne, fp = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.rt_grid_info(h, C.byref(na), C.byref(ne), C.byref(fp)))
        self.nang = na.value
        self.nedge = ne.value
        self.path = int(fp.value)             # 0 general, 1 tiled, 2 column
        self.fast_path = self.path == 1

    # -------------------------------------------------------------- queries
    def angles(self):
        nh = np.zeros((self.nang, 3))
        do = np.zeros(self.nang)
        _check(self._lib.rt_angles(self._h, _ptr(nh), _ptr(do)))
        return nh, do

    def max_dt(self, cfl: float) -> float:
        dt = C.c_double()
        _check(self._lib.rt_max_dt(self._h, float(cfl), C.byref(dt)))
        return dt.value

    def stats(self):
        nr = C.c_int64()
        me = C.c_double()
        _check(self._lib.rt_stats(self._h, C.byref(nr), C.byref(me)))
        return {"no_root": nr.value, "masked_energy": me.value}

    # -------------------------------------------------------------- checks
    def _state_shape(self):
        return (self.n[2], self.n[1], self.n[0], self.nang)

    def _cell_shape(self, *extra):
        return (self.n[2], self.n[1], self.n[0]) + tuple(extra)

    def _need(self, t, shape, dtype, name):
        import torch
        if t is None:
            return
        if not t.is_cuda or t.device.index != self.device:
            raise RtError("%s must live on cuda:%d" % (name, self.device))
        if t.dtype != dtype:
            raise RtError("%s must be %s, got %s" % (name, dtype, t.dtype))
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise RtError("%s must be a contiguous %s tensor, got %s" % (name, shape, tuple(t.shape)))
        del torch

    def real_dtype(self):
        import torch
        return torch.float32 if self.precision == RT_F32 else torch.float64

    # -------------------------------------------------------------- compute
    def step(self, I_in, I_out, T, rho, u, kappa_a, kappa_s, dt, dT0=None, lum=None,
             stream=None, I_star=None, noalloc=False):
        """rt_step, or with ``noalloc`` rt_step_noalloc (the same step with its
        partial sums in the library's static device scratch)."""
        import torch
        rd = self.real_dtype()
        f8 = torch.float64
        self._need(I_in, self._state_shape(), rd, "I_in")
        self._need(I_out, self._state_shape(), rd, "I_out")
        self._need(T, self._cell_shape(), f8, "T")
        self._need(rho, self._cell_shape(), f8, "rho")
        self._need(u, self._cell_shape(3), f8, "u")
        self._need(kappa_a, self._cell_shape(), f8, "kappa_a")
        self._need(kappa_s, self._cell_shape(), f8, "kappa_s")
        self._need(dT0, self._cell_shape(4), f8, "dT0")
        self._need(lum, (1,), f8, "lum")
        self._need(I_star, self._state_shape(), rd, "I_star")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        fn = self._lib.rt_step_noalloc if noalloc else self._lib.rt_step
        _check(fn(self._h, C.c_void_p(s.cuda_stream), _dev(I_in), _dev(I_out), _dev(T), _dev(rho),
                  _dev(u), _dev(kappa_a), _dev(kappa_s), float(dt), _dev(dT0), _dev(lum),
                  _dev(I_star)))

    def step_adjoint(self, I_n, T_n, rho, u, kappa_a, kappa_s, dt, lamI_next, lamT_next,
                     lamI_out, lamT_out, work, grad_kappa_a=None, grad_kappa_s=None,
                     lum_weight=1.0, stream=None, I_star=None):
        """Reverse of step() for J = sum dt * luminosity; see rt_step_adjoint.
        I_star: the I* that step(..., I_star=) wrote for the same inputs, or
        None to recompute the transport."""
        import torch
        rd = self.real_dtype()
        f8 = torch.float64
        for t, name in ((I_n, "I_n"), (lamI_next, "lamI_next"), (lamI_out, "lamI_out"),
                        (work, "work"), (I_star, "I_star")):
            self._need(t, self._state_shape(), rd, name)
        for t, name in ((T_n, "T_n"), (rho, "rho"), (kappa_a, "kappa_a"), (kappa_s, "kappa_s"),
                        (lamT_next, "lamT_next"), (lamT_out, "lamT_out"),
                        (grad_kappa_a, "grad_kappa_a"), (grad_kappa_s, "grad_kappa_s")):
            self._need(t, self._cell_shape(), f8, name)
        self._need(u, self._cell_shape(3), f8, "u")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self._lib.rt_step_adjoint(
            self._h, C.c_void_p(s.cuda_stream), _dev(I_n), _dev(T_n), _dev(rho), _dev(u),
            _dev(kappa_a), _dev(kappa_s), float(dt), float(lum_weight), _dev(lamI_next),
            _dev(lamT_next), _dev(lamI_out), _dev(lamT_out), _dev(work), _dev(grad_kappa_a),
            _dev(grad_kappa_s), _dev(I_star)))

    def moments(self, I, u=None, stream=None):
        import torch
        f8 = torch.float64
        self._need(I, self._state_shape(), self.real_dtype(), "I")
        self._need(u, self._cell_shape(3), f8, "u")
        dev = torch.device("cuda", self.device)
        R = torch.empty(self._cell_shape(10), dtype=f8, device=dev)
        R0 = torch.empty(self._cell_shape(4), dtype=f8, device=dev)
        E = torch.empty(self._cell_shape(), dtype=f8, device=dev) if u is not None else None
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self._lib.rt_moments(self._h, C.c_void_p(s.cuda_stream), _dev(I), _dev(u),
                                    _dev(R), _dev(R0), _dev(E)))
        return R, R0, E

    def gas_update(self, dT0, T_pre, rho, u, T, status=None, stream=None):
        """rt_gas_update: adds one step's dT0 to T^0_alpha of the gas state
        (rho, u, T_pre) and writes the recovered (rho, u, T) in place."""
        import torch
        f8 = torch.float64
        self._need(dT0, self._cell_shape(4), f8, "dT0")
        self._need(T_pre, self._cell_shape(), f8, "T_pre")
        self._need(rho, self._cell_shape(), f8, "rho")
        self._need(u, self._cell_shape(3), f8, "u")
        self._need(T, self._cell_shape(), f8, "T")
        self._need(status, self._cell_shape(), torch.int32, "status")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self._lib.rt_gas_update(self._h, C.c_void_p(s.cuda_stream), _dev(dT0), _dev(T_pre),
                                       _dev(rho), _dev(u), _dev(T), _dev(status)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rt_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
