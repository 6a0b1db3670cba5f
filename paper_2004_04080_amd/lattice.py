"""Python front end of liblbhip: parameters, caller-owned device buffers
(torch tensors on the GPU) and one object per simulation context.

PyTorch provides only device memory and the HIP stream; every step of the
method runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import binding as B


@dataclass
class Params:
    """Mirror of lb_params (include/lbhip.h) with the defaults of this build."""
    nx: int
    ny: int
    nz: int
    ncomp: int = 2
    tau: Sequence[float] = (1.0, 1.0)
    G: float = 0.0
    sc_norm: float = 1.0
    g: Sequence[float] = (0.0, 0.0, 0.0)
    rho0: Sequence[float] = (1.0, 1.0)
    precision: str = "fp32"
    walls: bool = False
    wall_u_lo: Sequence[float] = (0.0, 0.0, 0.0)
    wall_u_hi: Sequence[float] = (0.0, 0.0, 0.0)
    max_particles: int = 0
    radius: float = 5.5
    particle_density: float = 1.0
    hertz_K: float = 20.0
    hertz_d0: Optional[float] = None     # default 2R + 1
    hertz_rcap: Optional[float] = None   # default 2R
    zeta: Sequence[float] = (0.0, 0.0)
    rho_fallback: Sequence[float] = (1.0, 1.0)
    rotate: bool = True
    particles_fixed: bool = False
    checkpoint_every: int = 0
    max_record_steps: int = 0
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

    def to_c(self) -> B.lb_params:
        p = B.lb_params()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.walls = int(self.walls)
        p.wall_u_lo[:] = [float(v) for v in self.wall_u_lo]
        p.wall_u_hi[:] = [float(v) for v in self.wall_u_hi]
        p.ncomp = self.ncomp
        tau = list(self.tau) + [self.tau[0]] * (2 - len(self.tau))
        p.tau[:] = [float(v) for v in tau[:2]]
        p.G = self.G
        p.sc_norm = self.sc_norm
        p.g[:] = [float(v) for v in self.g]
        r0 = list(self.rho0) + [self.rho0[0]] * (2 - len(self.rho0))
        p.rho0[:] = [float(v) for v in r0[:2]]
        p.precision = {"fp32": B.LB_FP32, "fp64": B.LB_FP64}[self.precision]
        p.max_particles = self.max_particles
        p.radius = self.radius
        p.particle_density = self.particle_density
        p.hertz_K = self.hertz_K
        p.hertz_d0 = 2 * self.radius + 1 if self.hertz_d0 is None else self.hertz_d0
        p.hertz_rcap = 2 * self.radius if self.hertz_rcap is None else self.hertz_rcap
        p.zeta[:] = [float(v) for v in self.zeta]
        p.rho_fallback[:] = [float(v) for v in self.rho_fallback]
        p.rotate = int(self.rotate)
        p.particles_fixed = int(self.particles_fixed)
        p.checkpoint_every = self.checkpoint_every
        p.max_record_steps = self.max_record_steps
        p.janus = int(self.janus)
        p.janus_theta0 = self.janus_theta0
        p.janus_width = self.janus_width
        p.janus_zeta[:] = [float(v) for v in self.janus_zeta]
        p.lub_mu = self.lub_mu
        p.lub_hn = self.lub_hn
        p.lub_hcap = self.lub_hcap
        p.wall_type[:] = [int(v) for v in self.wall_type]
        p.wall_rho[:] = [float(v) for face in self.wall_rho for v in face]
        return p


def lattice():
    """(c [19,3], w [19]) in the library's direction order."""
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    B.check(B.lib().lb_lattice(c.ctypes.data_as(C.POINTER(C.c_int32)),
                               w.ctypes.data_as(C.POINTER(C.c_double))), "lb_lattice")
    return c, w


def required_sizes(params: Params) -> B.lb_sizes:
    s = B.lb_sizes()
    cp = params.to_c()
    B.check(B.lib().lb_required_sizes(C.byref(cp), C.byref(s)), "lb_required_sizes")
    return s


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


@dataclass
class Observables:
    step: int
    fluid_nodes: int
    mass: np.ndarray
    momentum: np.ndarray
    rho_min: np.ndarray
    rho_max: np.ndarray
    u_max: float
    particle_momentum: np.ndarray
    particle_ke: float
    particle_ke_rot: float
    nparticles: int
    flags: int
    phys_momentum: np.ndarray = None
    flink_abs: float = 0.0
    status: int = 0


class Lattice:
    """One simulation context on one GPU (lb_ctx)."""

    def __init__(self, params: Params, rho0: np.ndarray, u0: Optional[np.ndarray] = None,
                 device: str = "cuda:0"):
        import torch  # device memory and streams only

        self.params = params
        self._cp = params.to_c()
        self.device = torch.device(device)
        sizes = required_sizes(params)
        self.sizes = sizes

        def alloc(n):
            return torch.empty(max(int(n), 1), dtype=torch.uint8, device=self.device)

        self._mem = dict(f0=alloc(sizes.f), f1=alloc(sizes.f), rho=alloc(sizes.rho),
                         o0=alloc(sizes.owner), o1=alloc(sizes.owner),
                         particles=alloc(sizes.particles), work=alloc(sizes.work),
                         adjoint=alloc(sizes.adjoint))
        bufs = B.lb_buffers()
        m = self._mem
        bufs.f[0], bufs.f[1] = m["f0"].data_ptr(), m["f1"].data_ptr()
        bufs.rho = m["rho"].data_ptr()
        bufs.owner[0], bufs.owner[1] = m["o0"].data_ptr(), m["o1"].data_ptr()
        bufs.particles = m["particles"].data_ptr()
        bufs.work = m["work"].data_ptr()
        bufs.adjoint = m["adjoint"].data_ptr()
        bufs.bytes = sizes
        self._bufs = bufs
        self.stream = torch.cuda.current_stream(self.device)
        r = _f64(rho0, (params.ncomp, params.N))
        u = None if u0 is None else _f64(u0, (params.N, 3))
        ctx = C.c_void_p()
        B.check(B.lib().lb_init(C.byref(self._cp), C.byref(bufs), _dp(r), _dp(u),
                                C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), "lb_init")
        self._ctx = ctx

    # -- lifetime ------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            B.lib().lb_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, where):
        B.check(rc, where, self._ctx)

    @property
    def N(self) -> int:
        return self.params.N

    # -- stepping --------------------------------------------------------------
    def add_particles(self, x, v=None, w=None, q=None) -> None:
        x = _f64(x, (-1, 3))
        n = x.shape[0]
        self._chk(B.lib().lb_add_particles(
            self._ctx, n, _dp(x), _dp(None if v is None else _f64(v, (n, 3))),
            _dp(None if w is None else _f64(w, (n, 3))),
            _dp(None if q is None else _f64(q, (n, 4)))), "lb_add_particles")

    def step(self, n: int = 1) -> None:
        self._chk(B.lib().lb_step(self._ctx, int(n)), "lb_step")

    def sync(self) -> None:
        self._chk(B.lib().lb_sync(self._ctx), "lb_sync")

    def timing(self, enable: bool) -> None:
        """Start (clearing the totals) or stop per-phase HIP-event timing."""
        self._chk(B.lib().lb_timing(self._ctx, int(enable)), "lb_timing")

    def timing_read(self) -> dict:
        """{phase: (total ms, launches)} since timing was enabled (synchronises)."""
        ms = (C.c_double * B.NPHASE)()
        n = (C.c_int64 * B.NPHASE)()
        self._chk(B.lib().lb_timing_read(self._ctx, ms, n), "lb_timing_read")
        return {name: (ms[i], n[i]) for i, name in enumerate(B.PHASES)}

    # -- queries ---------------------------------------------------------------
    def observables(self, raise_on_flag: bool = True, noalloc: bool = False) -> Observables:
        """lb_observables, or with noalloc=True lb_observables_noalloc (the
        reduction scratch in the library's static device array)."""
        o = B.lb_obs()
        name = "lb_observables_noalloc" if noalloc else "lb_observables"
        rc = getattr(B.lib(), name)(self._ctx, C.byref(o))
        if rc not in (B.LB_OK, B.LB_E_PARTICLE_SPEED, B.LB_E_NONFINITE) or (
                raise_on_flag and rc != B.LB_OK):
            self._chk(rc, name)
        return Observables(o.step, o.fluid_nodes, np.array(o.mass[:]), np.array(o.momentum[:]),
                           np.array(o.rho_min[:]), np.array(o.rho_max[:]), o.u_max,
                           np.array(o.particle_momentum[:]), o.particle_ke, o.particle_ke_rot,
                           o.nparticles, o.flags, np.array(o.phys_momentum[:]), o.flink_abs,
                           rc)

    def fields(self):
        rho = np.empty((self.params.ncomp, self.N))
        u = np.empty((self.N, 3))
        self._chk(B.lib().lb_get_fields(self._ctx, _dp(rho), _dp(u)), "lb_get_fields")
        return rho, u

    def psi(self) -> np.ndarray:
        out = np.empty((self.params.ncomp, self.N))
        self._chk(B.lib().lb_get_psi(self._ctx, _dp(out)), "lb_get_psi")
        return out

    def populations(self) -> np.ndarray:
        out = np.empty((self.params.ncomp, 19, self.N))
        self._chk(B.lib().lb_get_populations(self._ctx, _dp(out)), "lb_get_populations")
        return out

    def set_populations(self, f: np.ndarray) -> None:
        a = _f64(f, (self.params.ncomp, 19, self.N))
        self._chk(B.lib().lb_set_populations(self._ctx, _dp(a)), "lb_set_populations")

    def owner(self) -> np.ndarray:
        out = np.empty(self.N, dtype=np.int32)
        self._chk(B.lib().lb_get_owner(self._ctx, out.ctypes.data_as(C.POINTER(C.c_int32))),
                  "lb_get_owner")
        return out

    def num_particles(self) -> int:
        return B.lib().lb_num_particles(self._ctx)

    def particles(self) -> np.ndarray:
        out = np.zeros((self.num_particles(), B.PREC))
        if out.size:
            self._chk(B.lib().lb_get_particles(self._ctx, _dp(out)), "lb_get_particles")
        return out

    def set_particles(self, rec: np.ndarray) -> None:
        a = _f64(rec, (self.num_particles(), B.PREC))
        self._chk(B.lib().lb_set_particles(self._ctx, _dp(a)), "lb_set_particles")

    # -- differentiation ---------------------------------------------------------
    def state(self) -> np.ndarray:
        """Restart snapshot (lb_get_state) as a host uint8 array."""
        n = C.c_size_t()
        self._chk(B.lib().lb_state_bytes(self._ctx, C.byref(n)), "lb_state_bytes")
        blob = np.empty(n.value, dtype=np.uint8)
        self._chk(B.lib().lb_get_state(self._ctx, C.c_void_p(blob.ctypes.data), n.value),
                  "lb_get_state")
        return blob

    def set_state(self, blob: np.ndarray) -> None:
        """Replace the state with a snapshot taken by state() (lb_set_state)."""
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        self._chk(B.lib().lb_set_state(self._ctx, C.c_void_p(b.ctypes.data), b.nbytes),
                  "lb_set_state")

    def domain_size(self):
        """(L, S) of the phase field: the average domain size and the shell
        means of the structure factor (lb_domain_size)."""
        import torch
        n = C.c_size_t()
        ns = C.c_int32()
        self._chk(B.lib().lb_domain_workspace(self._ctx, C.byref(n), C.byref(ns)),
                  "lb_domain_workspace")
        work = torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)
        L = C.c_double()
        S = np.zeros(ns.value)
        self._chk(B.lib().lb_domain_size(self._ctx, C.c_void_p(work.data_ptr()), n.value,
                                         C.byref(L), _dp(S), ns.value), "lb_domain_size")
        return L.value, S

    def loss(self, seeds: bool = False):
        """L (host float); with seeds=True also dL/dpsi_k as device FP64 tensors."""
        import torch
        L = C.c_double()
        if not seeds:
            self._chk(B.lib().lb_loss(self._ctx, C.byref(L), None, None), "lb_loss")
            return L.value
        sA = torch.empty(self.N, dtype=torch.float64, device=self.device)
        sB = torch.empty(self.N, dtype=torch.float64, device=self.device)
        self._chk(B.lib().lb_loss(self._ctx, C.byref(L), C.c_void_p(sA.data_ptr()),
                                  C.c_void_p(sB.data_ptr())), "lb_loss")
        return L.value, sA, sB

    def backward(self, seedA, seedB=None):
        """(dL/drho0_A device FP64 [N], dL/dG, dL/dg[3]) through every recorded step."""
        import torch
        out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        dG = C.c_double()
        dg = (C.c_double * 3)()
        self._chk(B.lib().lb_backward(
            self._ctx, C.c_void_p(seedA.data_ptr()),
            None if seedB is None else C.c_void_p(seedB.data_ptr()),
            C.c_void_p(out.data_ptr()), C.byref(dG), dg), "lb_backward")
        return out, dG.value, np.array(dg[:])
