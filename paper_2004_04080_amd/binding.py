"""ctypes mirror of include/lbhip.h (argument marshalling only).

Every computation happens inside liblbhip.so on the GPU; this module only
declares the C structures and function signatures and turns status codes
into exceptions. Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LBHIP_LIB selects another build of the same sources (timing experiments)
LIB_PATH = os.environ.get("LBHIP_LIB", os.path.join(HERE, "_lib", "liblbhip.so"))

LB_OK = 0
LB_E_ARG, LB_E_SHAPE, LB_E_OVERLAP, LB_E_CAPACITY = -1, -2, -3, -4
LB_E_NONFINITE, LB_E_PARTICLE_SPEED, LB_E_HIP, LB_E_STATE = -5, -6, -7, -8
LB_FP32, LB_FP64 = 0, 1

PREC = 50
REC = dict(x=0, v=3, w=6, q=9, Fprev=13, Tprev=16, Fd=19, Td=22, Fc=25, Tc=28, FH=31, FSC=34,
           TSC=37, Fliq=40, Tliq=43, flabs=46, mass=47, inertia=48, have_prev=49)

EXPORTED = [
    "lb_version", "lb_strerror", "lb_last_error", "lb_lattice", "lb_required_sizes", "lb_init",
    "lb_add_particles", "lb_step", "lb_observables", "lb_get_fields", "lb_get_psi",
    "lb_get_populations", "lb_set_populations", "lb_get_owner", "lb_get_particles",
    "lb_set_particles", "lb_num_particles", "lb_loss", "lb_backward", "lb_sync", "lb_free",
    "lb_timing", "lb_timing_read", "lb_state_bytes", "lb_get_state", "lb_set_state",
    "lb_domain_workspace", "lb_domain_size", "lb_observables_noalloc", "lb_probe_stream",
    "lb_debug_count_writes",
]
NPHASE = 5
PHASES = ("density", "spheres", "fill", "collide", "integrate")


class lb_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls", C.c_int32),
        ("wall_u_lo", C.c_double * 3), ("wall_u_hi", C.c_double * 3),
        ("ncomp", C.c_int32), ("tau", C.c_double * 2), ("G", C.c_double),
        ("sc_norm", C.c_double), ("g", C.c_double * 3), ("rho0", C.c_double * 2),
        ("precision", C.c_int32), ("max_particles", C.c_int32), ("radius", C.c_double),
        ("particle_density", C.c_double), ("hertz_K", C.c_double), ("hertz_d0", C.c_double),
        ("hertz_rcap", C.c_double), ("zeta", C.c_double * 2), ("rho_fallback", C.c_double * 2),
        ("rotate", C.c_int32), ("particles_fixed", C.c_int32), ("checkpoint_every", C.c_int32),
        ("max_record_steps", C.c_int32),
        ("janus", C.c_int32), ("janus_theta0", C.c_double), ("janus_width", C.c_double),
        ("janus_zeta", C.c_double * 2),
        ("lub_mu", C.c_double), ("lub_hn", C.c_double), ("lub_hcap", C.c_double),
        ("wall_type", C.c_int32 * 2), ("wall_rho", C.c_double * 4),
    ]


class lb_sizes(C.Structure):
    _fields_ = [("f", C.c_size_t), ("rho", C.c_size_t), ("owner", C.c_size_t),
                ("particles", C.c_size_t), ("work", C.c_size_t), ("adjoint", C.c_size_t)]


class lb_buffers(C.Structure):
    _fields_ = [("f", C.c_void_p * 2), ("rho", C.c_void_p), ("owner", C.c_void_p * 2),
                ("particles", C.c_void_p), ("work", C.c_void_p), ("adjoint", C.c_void_p),
                ("bytes", lb_sizes)]


class lb_obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("fluid_nodes", C.c_int64), ("mass", C.c_double * 2),
                ("momentum", C.c_double * 3), ("rho_min", C.c_double * 2),
                ("rho_max", C.c_double * 2), ("u_max", C.c_double),
                ("particle_momentum", C.c_double * 3), ("particle_ke", C.c_double),
                ("particle_ke_rot", C.c_double), ("nparticles", C.c_int32),
                ("flags", C.c_int32), ("phys_momentum", C.c_double * 3),
                ("flink_abs", C.c_double)]


class LBError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {strerror(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None


def lib():
    """The loaded liblbhip.so. Raises if the HIP library is missing: there is
    no other implementation to fall back to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"liblbhip.so not found at {LIB_PATH}; build it with "
            "`python -m paper_2004_04080_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    L.lb_version.restype = C.c_char_p
    L.lb_strerror.restype = C.c_char_p
    L.lb_strerror.argtypes = [C.c_int]
    L.lb_last_error.restype = C.c_char_p
    L.lb_last_error.argtypes = [vp]
    L.lb_lattice.argtypes = [ip, dp]
    L.lb_required_sizes.argtypes = [C.POINTER(lb_params), C.POINTER(lb_sizes)]
    L.lb_init.argtypes = [C.POINTER(lb_params), C.POINTER(lb_buffers), dp, dp, vp,
                          C.POINTER(vp)]
    L.lb_add_particles.argtypes = [vp, C.c_int32, dp, dp, dp, dp]
    L.lb_step.argtypes = [vp, C.c_int32]
    L.lb_observables.argtypes = [vp, C.POINTER(lb_obs)]
    L.lb_observables_noalloc.argtypes = [vp, C.POINTER(lb_obs)]
    L.lb_get_fields.argtypes = [vp, dp, dp]
    L.lb_get_psi.argtypes = [vp, dp]
    L.lb_get_populations.argtypes = [vp, dp]
    L.lb_set_populations.argtypes = [vp, dp]
    L.lb_get_owner.argtypes = [vp, ip]
    L.lb_get_particles.argtypes = [vp, dp]
    L.lb_set_particles.argtypes = [vp, dp]
    L.lb_num_particles.argtypes = [vp]
    L.lb_loss.argtypes = [vp, dp, vp, vp]
    L.lb_backward.argtypes = [vp, vp, vp, vp, dp, dp]
    L.lb_sync.argtypes = [vp]
    L.lb_free.argtypes = [vp]
    L.lb_free.restype = None
    L.lb_timing.argtypes = [vp, C.c_int]
    L.lb_timing_read.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    L.lb_state_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.lb_get_state.argtypes = [vp, vp, C.c_size_t]
    L.lb_set_state.argtypes = [vp, vp, C.c_size_t]
    L.lb_domain_workspace.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_int32)]
    L.lb_domain_size.argtypes = [vp, vp, C.c_size_t, dp, dp, C.c_int32]
    L.lb_debug_count_writes.argtypes = [vp, vp]
    L.lb_probe_stream.argtypes = [C.c_int32, vp, vp, C.c_size_t, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_int32, vp, dp]
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().lb_strerror(status).decode()


def last_error(ctx=None) -> str:
    s = lib().lb_last_error(ctx)
    return s.decode() if s else ""


def check(status: int, where: str, ctx=None) -> None:
    if status != LB_OK:
        raise LBError(status, where, last_error(ctx))
