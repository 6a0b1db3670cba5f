"""lb_observables_noalloc (reduction scratch in the library's static device
array) against lb_observables (the context's work buffer), through the C
interface, on two calls in a row: a larger box with moving spheres between
walls, then a smaller one. Both entry points run the same fluid kernels over
the same partial-record layout, so the fluid observables must agree bit for
bit; the sphere sums are added in another order (a tree against a serial
compensated sum) and must agree to 1e-12 relative."""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

FLUID = ("step", "fluid_nodes", "mass", "momentum", "phys_momentum", "rho_min", "rho_max",
         "u_max", "nparticles", "flags")
SPHERE = ("particle_momentum", "particle_ke", "particle_ke_rot", "flink_abs")


def _lattice(shape, n, precision, seed, walls):
    from paper_2004_04080_amd import Lattice, Params
    w = synth.Workload("noalloc", *shape, nparticles=n, radius=3.0, seed=seed, walls=walls)
    rng = np.random.default_rng(seed % 1000)
    p = Params(*shape, ncomp=2, G=0.65, g=(1e-5, 0.0, -2e-5), precision=precision, walls=walls,
               wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0), max_particles=n, radius=3.0,
               particle_density=1.5)
    lat = Lattice(p, w.densities())
    x = w.centres()
    lat.add_particles(x, 0.04 * (2 * rng.random((len(x), 3)) - 1),
                      0.02 * (2 * rng.random((len(x), 3)) - 1))
    return lat


def _call(lat, name):
    from paper_2004_04080_amd import binding as B
    o = B.lb_obs()
    rc = getattr(B.lib(), name)(lat._ctx, C.byref(o))
    assert rc == B.LB_OK, (name, rc, B.last_error(lat._ctx))
    return o


def _value(o, k):
    v = getattr(o, k)
    return np.array(v[:]) if hasattr(v, "__len__") else np.array(v)


def test_noalloc_observables_match_lb_observables_on_two_boxes():
    big = _lattice((40, 36, 30), 8, "fp64", synth.BASE_SEED + 91, True)
    small = _lattice((20, 18, 16), 2, "fp32", synth.BASE_SEED + 92, False)
    big.step(12)
    small.step(7)
    for lat, what in ((big, "larger box"), (small, "smaller box")):
        print(f"[noalloc] {what}", flush=True)
        a = _call(lat, "lb_observables_noalloc")
        b = _call(lat, "lb_observables")
        for k in FLUID:
            assert np.array_equal(_value(a, k), _value(b, k)), (what, k, _value(a, k),
                                                              _value(b, k))
        for k in SPHERE:
            va, vb = _value(a, k), _value(b, k)
            assert np.abs(va - vb).max() <= 1e-12 * max(np.abs(vb).max(), 1e-300), (what, k)
        assert a.nparticles > 0 and a.flink_abs > 0
    big.close()
    small.close()
