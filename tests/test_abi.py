"""The C interface without a GPU: the library loads, exports every function
declared in include/lbhip.h, and rejects bad parameters on the host with the
documented status codes before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2004_04080_amd import binding as B
from paper_2004_04080_amd.lattice import Params, lattice, required_sizes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "lbhip.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(lb_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = B.lib()
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(B.EXPORTED)
    assert b"gfx950" in lib.lb_version()


def test_lattice_is_d3q19():
    c, w = lattice()
    n2 = (c ** 2).sum(1)
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert abs(w.sum() - 1) < 1e-15 and np.abs(w @ c).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3)


def test_required_sizes_scale_with_the_box():
    s = required_sizes(Params(64, 32, 16, precision="fp32"))
    N = 64 * 32 * 16
    assert s.f >= 2 * 19 * N * 4 and s.f < 2 * 19 * N * 4 + 256
    assert s.rho >= 2 * N * 4
    assert s.owner == 0 and s.particles == 0 and s.adjoint == 0
    s64 = required_sizes(Params(64, 32, 16, precision="fp64", walls=True, max_particles=10,
                                radius=3.0))
    assert s64.f >= 2 * 19 * N * 8 and s64.owner >= 2 * N and s64.particles > 0
    sa = required_sizes(Params(16, 16, 16, checkpoint_every=5, max_record_steps=20))
    assert sa.adjoint >= (4 + 5) * sa.f


def test_work_buffer_holds_the_node_lists_at_their_bound():
    """A sphere owns only nodes closer than R to its centre, and the unit cubes
    around them lie inside the ball of radius R + 1: the frontier list needs at
    most 4/3 pi (R + 1)^3 entries per sphere and the event list twice that
    (8 bytes an entry), both capped by the node count."""
    import math
    shape = (96, 96, 96)
    N = math.prod(shape)
    base = required_sizes(Params(*shape, max_particles=0)).work
    for P, R in ((40, 5.5), (200, 3.0)):
        w = required_sizes(Params(*shape, max_particles=P, radius=R)).work
        per = math.ceil(4.0 / 3.0 * math.pi * (R + 1.0) ** 3)
        need = 8 * (min(N, P * per) + min(N, 2 * P * per))
        assert w - base >= need, (P, R, w - base, need)
    # when the bound passes the node count, the node count caps both lists
    big = required_sizes(Params(24, 24, 24, max_particles=60, radius=5.5)).work
    small = required_sizes(Params(24, 24, 24, max_particles=0)).work
    assert big - small < 8 * 3 * 24 ** 3 + 64 * 1024


@pytest.mark.parametrize("change,code", [
    (dict(tau=(0.5, 1.0)), B.LB_E_ARG),
    (dict(tau=(1.0, 0.3)), B.LB_E_ARG),
    (dict(ncomp=3), B.LB_E_ARG),
    (dict(nx=0), B.LB_E_ARG),
    (dict(walls=True, nz=2), B.LB_E_ARG),
    (dict(max_particles=4, radius=9.0), B.LB_E_ARG),
    (dict(max_particles=4, radius=0.0), B.LB_E_ARG),
    (dict(max_particles=70000), B.LB_E_ARG),
    (dict(max_particles=4, radius=2.0, hertz_d0=3.0, hertz_rcap=4.0), B.LB_E_ARG),
    (dict(checkpoint_every=-1), B.LB_E_ARG),
    (dict(checkpoint_every=5, max_record_steps=0), B.LB_E_ARG),
    (dict(precision="fp32", nx=2048, ny=2048, nz=1024), B.LB_E_SHAPE),
])
def test_invalid_parameters_are_rejected_on_the_host(change, code):
    p = Params(16, 16, 16, G=0.65)
    for k, v in change.items():
        setattr(p, k, v)
    s = B.lb_sizes()
    cp = p.to_c()
    assert B.lib().lb_required_sizes(C.byref(cp), C.byref(s)) == code
    assert B.last_error()


def _fake_buffers(sizes, shrink=None):
    bufs = B.lb_buffers()
    addr = 0x100000
    for name in ("f", "rho", "owner", "particles", "work", "adjoint"):
        pass
    bufs.f[0], bufs.f[1] = addr, addr + (1 << 40)
    bufs.rho = addr + (2 << 40)
    bufs.owner[0], bufs.owner[1] = addr + (3 << 40), addr + (4 << 40)
    bufs.particles = addr + (5 << 40)
    bufs.work = addr + (6 << 40)
    bufs.adjoint = addr + (7 << 40)
    bufs.bytes = sizes
    if shrink:
        setattr(bufs.bytes, shrink, getattr(sizes, shrink) - 1)
    return bufs


def test_init_rejects_bad_buffers_and_densities_before_device_work():
    """Every case here fails during host validation, so the fake device
    addresses are never dereferenced."""
    p = Params(8, 8, 8, G=0.65, max_particles=2, radius=2.0)
    sizes = required_sizes(p)
    cp = p.to_c()
    rho = np.ones((2, p.N))
    ctx = C.c_void_p()
    dp = rho.ctypes.data_as(C.POINTER(C.c_double))
    L = B.lib()
    assert L.lb_init(C.byref(cp), None, dp, None, None, C.byref(ctx)) == B.LB_E_ARG
    for field in ("f", "rho", "owner", "work", "particles"):
        bufs = _fake_buffers(sizes, shrink=field)
        assert L.lb_init(C.byref(cp), C.byref(bufs), dp, None, None, C.byref(ctx)) == B.LB_E_SHAPE
    bufs = _fake_buffers(sizes)
    bufs.work = None
    assert L.lb_init(C.byref(cp), C.byref(bufs), dp, None, None, C.byref(ctx)) == B.LB_E_ARG
    bufs = _fake_buffers(sizes)
    bufs.rho = 0x100004  # misaligned
    assert L.lb_init(C.byref(cp), C.byref(bufs), dp, None, None, C.byref(ctx)) == B.LB_E_ARG
    bad = rho.copy()
    bad[1, 7] = np.nan
    bufs = _fake_buffers(sizes)
    assert L.lb_init(C.byref(cp), C.byref(bufs), bad.ctypes.data_as(C.POINTER(C.c_double)), None,
                     None, C.byref(ctx)) == B.LB_E_ARG
    bad[1, 7] = -0.1
    assert L.lb_init(C.byref(cp), C.byref(bufs), bad.ctypes.data_as(C.POINTER(C.c_double)), None,
                     None, C.byref(ctx)) == B.LB_E_ARG


def test_null_context_calls_fail_cleanly():
    L = B.lib()
    assert L.lb_step(None, 1) == B.LB_E_ARG
    assert L.lb_sync(None) == B.LB_E_ARG
    o = B.lb_obs()
    assert L.lb_observables(None, C.byref(o)) == B.LB_E_ARG
    L.lb_free(None)
    assert B.strerror(B.LB_E_PARTICLE_SPEED)


def test_stream_probe_rejects_bad_arguments_on_the_host():
    """lb_probe_stream checks its arguments before any device call."""
    import ctypes as C
    from paper_2004_04080_amd import binding as B
    lib = B.lib()
    ms = C.c_double()
    buf = C.c_void_p(16)       # never dereferenced: every call below is refused first
    assert lib.lb_probe_stream(7, buf, buf, 1024, 0, 0, 0, 1, None, C.byref(ms)) == B.LB_E_ARG
    assert lib.lb_probe_stream(2, buf, buf, 1024, 0, 0, 0, 0, None, C.byref(ms)) == B.LB_E_ARG
    assert lib.lb_probe_stream(2, buf, buf, 1024, 0, 0, 0, 1, None, None) == B.LB_E_ARG
    assert lib.lb_probe_stream(1, None, None, 1024, 0, 0, 0, 1, None, C.byref(ms)) == B.LB_E_ARG
    # the collide pattern: a plane above 4 GiB, and buffers smaller than 2 x 19 planes
    assert lib.lb_probe_stream(3, buf, buf, 1 << 40, 2048, 1024, 1024, 1, None,
                               C.byref(ms)) == B.LB_E_SHAPE
    assert lib.lb_probe_stream(3, buf, buf, 38 * 4 * 64 - 4, 4, 4, 4, 1, None,
                               C.byref(ms)) == B.LB_E_SHAPE
    # the march pattern: columns of 128 x 8 nodes must tile the x-y plane
    big = 38 * 4 * 256 * 16 * 4
    for nx, ny in ((120, 16), (256, 12), (64, 8)):
        assert lib.lb_probe_stream(4, buf, buf, big, nx, ny, 4, 1, None,
                                   C.byref(ms)) == B.LB_E_SHAPE, (nx, ny)
    assert lib.lb_probe_stream(5, buf, buf, big, 256, 16, 4, 1, None, C.byref(ms)) == B.LB_E_ARG
