"""Python access to the reference oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain serial FP64 C++ implementation of the LBsoft step
(Bonaccorso et al., arXiv 2004.04080, Sec. 2 and the eight-step sequence of
Sec. 3.1) built from ``lbo.cpp`` into ``liblbo.so``. Only ``tests/``, the smoke
check and the CPU-baseline leg of ``bench.py`` may import this package; the
product path never does.

Every function documented in ``lbo.h`` is mirrored here with numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBO_LIB selects another build of lbo.cpp (used by the mutation tests)
LIB_PATH = os.environ.get("LBO_LIB", os.path.join(HERE, "liblbo.so"))

PREC = 50   # doubles per particle record
NOBS = 36   # observables


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("walls", C.c_int32),
        ("wall_u_lo", C.c_double * 3), ("wall_u_hi", C.c_double * 3),
        ("ncomp", C.c_int32),
        ("tau", C.c_double * 2), ("G", C.c_double), ("sc_norm", C.c_double),
        ("g", C.c_double * 3),
        ("radius", C.c_double), ("particle_density", C.c_double),
        ("hertz_K", C.c_double), ("hertz_d0", C.c_double), ("hertz_rcap", C.c_double),
        ("zeta", C.c_double * 2), ("rho_fallback", C.c_double * 2),
        ("rotate", C.c_int32), ("particles_fixed", C.c_int32),
        ("janus", C.c_int32), ("janus_theta0", C.c_double), ("janus_width", C.c_double),
        ("janus_zeta", C.c_double * 2),
        ("lub_mu", C.c_double), ("lub_hn", C.c_double), ("lub_hcap", C.c_double),
        ("wall_type", C.c_int32 * 2), ("wall_rho", C.c_double * 4),
    ]


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    ncomp: int = 2
    tau: Sequence[float] = (1.0, 1.0)
    G: float = 0.0
    sc_norm: float = 1.0
    g: Sequence[float] = (0.0, 0.0, 0.0)
    walls: bool = False
    wall_u_lo: Sequence[float] = (0.0, 0.0, 0.0)
    wall_u_hi: Sequence[float] = (0.0, 0.0, 0.0)
    radius: float = 5.5
    particle_density: float = 1.0
    hertz_K: float = 20.0
    hertz_d0: Optional[float] = None      # default 2R + 1
    hertz_rcap: Optional[float] = None    # default 2R
    zeta: Sequence[float] = (0.0, 0.0)
    rho_fallback: Sequence[float] = (1.0, 1.0)
    rotate: bool = True
    particles_fixed: bool = False
    janus: bool = False
    janus_theta0: float = 108.0
    janus_width: float = 10.0
    janus_zeta: Sequence[float] = (0.1, 0.1)
    lub_mu: float = 0.0
    lub_hn: float = 0.67
    lub_hcap: float = 0.5
    wall_type: Sequence[int] = (0, 0)
    wall_rho: Sequence[Sequence[float]] = ((1.0, 1.0), (1.0, 1.0))

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def to_c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.walls = int(self.walls)
        p.wall_u_lo[:] = list(self.wall_u_lo)
        p.wall_u_hi[:] = list(self.wall_u_hi)
        p.ncomp = self.ncomp
        tau = list(self.tau) + [self.tau[0]] * (2 - len(self.tau))
        p.tau[:] = tau[:2]
        p.G = self.G
        p.sc_norm = self.sc_norm
        p.g[:] = list(self.g)
        p.radius = self.radius
        p.particle_density = self.particle_density
        p.hertz_K = self.hertz_K
        p.hertz_d0 = 2 * self.radius + 1 if self.hertz_d0 is None else self.hertz_d0
        p.hertz_rcap = 2 * self.radius if self.hertz_rcap is None else self.hertz_rcap
        p.zeta[:] = list(self.zeta)
        p.rho_fallback[:] = list(self.rho_fallback)
        p.rotate = int(self.rotate)
        p.particles_fixed = int(self.particles_fixed)
        p.janus = int(self.janus)
        p.janus_theta0 = self.janus_theta0
        p.janus_width = self.janus_width
        p.janus_zeta[:] = list(self.janus_zeta)
        p.lub_mu = self.lub_mu
        p.lub_hn = self.lub_hn
        p.lub_hcap = self.lub_hcap
        p.wall_type[:] = [int(v) for v in self.wall_type]
        p.wall_rho[:] = [float(v) for face in self.wall_rho for v in face]
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.lbo_create.restype = vp
        L.lbo_create.argtypes = [C.POINTER(_Params), dp, dp]
        L.lbo_destroy.argtypes = [vp]
        L.lbo_add_particles.argtypes = [vp, C.c_int32, dp, dp, dp, dp]
        L.lbo_step.argtypes = [vp, C.c_int32]
        L.lbo_lattice.argtypes = [ip, dp]
        for nm in ("lbo_get_f", "lbo_set_f", "lbo_get_rho", "lbo_get_psi", "lbo_get_u",
                   "lbo_get_particles", "lbo_set_particle_state", "lbo_observables"):
            getattr(L, nm).argtypes = [vp, dp]
        L.lbo_get_owner.argtypes = [vp, ip]
        L.lbo_set_owner.argtypes = [vp, ip]
        L.lbo_num_particles.argtypes = [vp]
        L.lbo_num_particles.restype = C.c_int32
        L.lbo_loss.argtypes = [vp]
        L.lbo_loss.restype = C.c_double
        L.lbo_loss_tangent.argtypes = [C.POINTER(_Params), dp, C.c_int32, dp, C.c_int32,
                                       C.c_double, dp, dp, dp, dp]
        L.lbo_psi_tangent.argtypes = [C.POINTER(_Params), dp, C.c_int32, dp, C.c_int32,
                                      C.c_double, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice():
    """(c [19,3] int, w [19]) in the oracle's direction order."""
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    lib().lbo_lattice(c.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w))
    return c, w


class Oracle:
    """One oracle simulation. Fields use node order n = x + nx*(y + ny*z)."""

    def __init__(self, params: Params, rho0: np.ndarray, u0: Optional[np.ndarray] = None):
        self.params = params
        self._cp = params.to_c()
        r = _f64(rho0).reshape(params.ncomp, params.N)
        u = None if u0 is None else _f64(u0).reshape(params.N, 3)
        self._h = lib().lbo_create(C.byref(self._cp), _dp(r), _dp(u))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def close(self):
        if self._h:
            lib().lbo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def N(self):
        return self.params.N

    def add_particles(self, x, v=None, w=None, q=None) -> None:
        x = _f64(x).reshape(-1, 3)
        n = x.shape[0]
        rc = lib().lbo_add_particles(self._h, n, _dp(x),
                                     _dp(None if v is None else _f64(v).reshape(n, 3)),
                                     _dp(None if w is None else _f64(w).reshape(n, 3)),
                                     _dp(None if q is None else _f64(q).reshape(n, 4)))
        if rc != 0:
            raise ValueError(f"lbo_add_particles: {rc}")

    def step(self, n: int = 1) -> int:
        return lib().lbo_step(self._h, n)

    def f(self) -> np.ndarray:
        out = np.empty((self.params.ncomp, 19, self.N))
        lib().lbo_get_f(self._h, _dp(out))
        return out

    def set_f(self, f: np.ndarray) -> None:
        a = _f64(f).reshape(self.params.ncomp, 19, self.N)
        lib().lbo_set_f(self._h, _dp(a))

    def rho(self) -> np.ndarray:
        out = np.empty((self.params.ncomp, self.N))
        lib().lbo_get_rho(self._h, _dp(out))
        return out

    def psi(self) -> np.ndarray:
        """Pseudo-potential: rho on fluid nodes, virtual densities on the
        frontier solid nodes, 0 elsewhere."""
        out = np.empty((self.params.ncomp, self.N))
        lib().lbo_get_psi(self._h, _dp(out))
        return out

    def u(self) -> np.ndarray:
        out = np.empty((self.N, 3))
        lib().lbo_get_u(self._h, _dp(out))
        return out

    def owner(self) -> np.ndarray:
        out = np.empty(self.N, dtype=np.int32)
        lib().lbo_get_owner(self._h, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def set_owner(self, own: np.ndarray) -> None:
        a = np.ascontiguousarray(own, dtype=np.int32)
        lib().lbo_set_owner(self._h, a.ctypes.data_as(C.POINTER(C.c_int32)))

    def num_particles(self) -> int:
        return lib().lbo_num_particles(self._h)

    def particles(self) -> np.ndarray:
        out = np.zeros((self.num_particles(), PREC))
        if out.size:
            lib().lbo_get_particles(self._h, _dp(out))
        return out

    def set_particle_state(self, rec: np.ndarray) -> None:
        a = _f64(rec).reshape(self.num_particles(), PREC)
        lib().lbo_set_particle_state(self._h, _dp(a))

    def observables(self) -> np.ndarray:
        out = np.zeros(NOBS)
        lib().lbo_observables(self._h, _dp(out))
        return out

    def loss(self) -> float:
        return lib().lbo_loss(self._h)


def loss_tangent(params: Params, rho0: np.ndarray, nsteps: int, dG: float = 0.0,
                 dg: Sequence[float] = (0.0, 0.0, 0.0), drhoA: Optional[np.ndarray] = None,
                 x: Optional[np.ndarray] = None):
    """(L, dL) from a dual-number run of nsteps from f = f_eq(rho0, 0)."""
    cp = params.to_c()
    r = _f64(rho0).reshape(params.ncomp, params.N)
    dgv = _f64(dg)
    dr = None if drhoA is None else _f64(drhoA).reshape(params.N)
    xx = None if x is None else _f64(x).reshape(-1, 3)
    np_ = 0 if xx is None else xx.shape[0]
    L = C.c_double()
    dL = C.c_double()
    rc = lib().lbo_loss_tangent(C.byref(cp), _dp(r), np_, _dp(xx), nsteps, dG, _dp(dgv),
                                _dp(dr), C.byref(L), C.byref(dL))
    if rc != 0:
        raise ValueError(f"lbo_loss_tangent: {rc}")
    return L.value, dL.value


def psi_tangent(params: Params, rho0: np.ndarray, nsteps: int, dG: float = 0.0,
                dg: Sequence[float] = (0.0, 0.0, 0.0), drhoA: Optional[np.ndarray] = None,
                x: Optional[np.ndarray] = None):
    """(psi, dpsi) [ncomp][N] of the final state of a dual-number run of nsteps
    from f = f_eq(rho0, 0): the tangent-linear map applied to (dG, dg, drhoA)."""
    cp = params.to_c()
    r = _f64(rho0).reshape(params.ncomp, params.N)
    dgv = _f64(dg)
    dr = None if drhoA is None else _f64(drhoA).reshape(params.N)
    xx = None if x is None else _f64(x).reshape(-1, 3)
    np_ = 0 if xx is None else xx.shape[0]
    psi = np.zeros((params.ncomp, params.N))
    dpsi = np.zeros((params.ncomp, params.N))
    rc = lib().lbo_psi_tangent(C.byref(cp), _dp(r), np_, _dp(xx), nsteps, dG, _dp(dgv),
                               _dp(dr), _dp(psi), _dp(dpsi))
    if rc != 0:
        raise ValueError(f"lbo_psi_tangent: {rc}")
    return psi, dpsi


# record offsets (see lbo.h)
REC = dict(x=0, v=3, w=6, q=9, Fprev=13, Tprev=16, Fd=19, Td=22, Fc=25, Tc=28, FH=31,
           FSC=34, TSC=37, Fliq=40, Tliq=43, flabs=46, mass=47, inertia=48, have_prev=49)
OBS = dict(mass=0, mom=2, rho_min=5, rho_max=7, umax=9, nfluid=10, pmom=11, ke=14, ke_rot=15,
           led_destroyed=16, led_created=18, led_link=20, led_body=22, led_sc=25, led_wall=28,
           step=31)
