"""Open z-faces (pressure by anti-bounce-back Eq. bbp, velocity by Eq. bbv with
extrapolated density, equilibrium inflow) through the HIP path against the
oracle: FP64 at 1e-12 over 1, 10 and 50 steps, two components, several face
combinations, one with moving spheres; FP32 step parity at 1e-5.

With G = 0.3 the components stay mixed, so phi = rho_A - rho_B is ~1e-2 of
the densities and its error relative to max|phi| carries the FP64 rounding
of rho about a hundredfold. Up to 10 steps phi is gated relative to itself;
at 50 steps its error is measured on the density scale (max|rho_k|), the
scale of the rounding it carries, at the same 1e-12."""
import numpy as np
import pytest

import synth
from gpu_util import compare, compare_particles, make_pair, requires_gpu, sync_state

pytestmark = [pytest.mark.gpu, requires_gpu]

SHAPE = (20, 18, 24)
CASES = {
    "pressure-pressure": dict(wall_type=(1, 1), wall_rho=((1.03, 0.99), (0.97, 1.01))),
    "velocity-pressure": dict(wall_type=(2, 1), wall_u_lo=(0.002, 0.0, 0.01),
                              wall_rho=((1.0, 1.0), (1.0, 1.0))),
    "equilibrium-velocity": dict(wall_type=(3, 2), wall_u_lo=(0.0, 0.0, 0.008),
                                 wall_u_hi=(0.0, 0.0, 0.008), wall_rho=((1.01, 0.99), (1.0, 1.0))),
    "wall-pressure": dict(wall_type=(0, 1), wall_u_lo=(0.01, 0.0, 0.0),
                          wall_rho=((1.0, 1.0), (1.02, 0.98))),
}


def _rho():
    return synth.Workload("open", *SHAPE, walls=True, seed=synth.BASE_SEED + 81).densities()


def _check(o, lat, tol, what, short=True):
    e = compare(o, lat)
    print(what, {k: (f"{v:.1e}" if isinstance(v, float) else v) for k, v in e.items()},
          flush=True)
    assert e.pop("owner_equal")
    e.pop("df")
    if not short:
        fluid = o.owner() == 0
        ro = o.rho()[:, fluid]
        rg = lat.fields()[0][:, fluid]
        e["phi"] = float(np.abs((rg[0] - rg[1]) - (ro[0] - ro[1])).max() / np.abs(ro).max())
        print(what, f"phi on the density scale {e['phi']:.1e}", flush=True)
    for k, v in e.items():
        assert v <= (5 * tol if (k == "u" and tol > 1e-9) else tol), (what, k, v)


@pytest.mark.parametrize("name", list(CASES))
def test_open_faces_fp64(name):
    o, lat = make_pair(SHAPE, _rho(), G=0.3, tau=(0.9, 0.9), walls=True, **CASES[name])
    done = 0
    for h in (1, 10, 50):
        assert o.step(h - done) == 0
        lat.step(h - done)
        done = h
        _check(o, lat, 1e-12, f"[open] {name} t={h}", short=h <= 10)


def test_open_faces_with_moving_spheres_fp64():
    w = synth.Workload("opensph", *SHAPE, nparticles=3, radius=3.0, walls=True,
                       seed=synth.BASE_SEED + 82)
    x = w.centres()
    v = np.random.default_rng(8).uniform(-0.01, 0.01, (len(x), 3))
    o, lat = make_pair(SHAPE, w.densities(), x=x, v=v, G=0.3, tau=(1.0, 1.0), walls=True,
                       radius=3.0, particle_density=2.0, hertz_K=0.5,
                       **CASES["velocity-pressure"])
    done = 0
    for h in (1, 10, 30):
        assert o.step(h - done) == 0
        lat.step(h - done)
        done = h
        _check(o, lat, 1e-12, f"[open] spheres t={h}", short=h <= 10)
        ep = compare_particles(o, lat)
        assert ep["x"] < 1e-12 and ep["v"] < 1e-12 and ep["Fliq"] < 1e-12


def test_open_faces_fp32_step_parity():
    o, lat = make_pair(SHAPE, _rho(), precision="fp32", G=0.3, tau=(0.9, 0.9), walls=True,
                       **CASES["pressure-pressure"])
    lat.step(20)
    sync_state(o, lat)
    for t in range(2):
        assert o.step(1) == 0
        lat.step(1)
        _check(o, lat, 1e-5, f"[open] fp32 step {t}")
