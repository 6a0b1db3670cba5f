"""Lubrication (Eq. libric) and Janus wetting through the HIP path against the
oracle: pairs of spheres approaching within the lubrication range, with the
orientation-dependent wetting of the benchmark input (108 +- 5 degrees,
constants 0.1), moving and rotating. FP64 at the bounds of the other
moving-sphere tests (fields, sphere state and force terms 1e-12), FP32 step
parity at 1e-5."""
import numpy as np
import pytest

import synth
from gpu_util import compare, compare_particles, make_pair, requires_gpu, sync_state

pytestmark = [pytest.mark.gpu, requires_gpu]

KW = dict(G=0.65, tau=(1.0, 1.0), radius=3.5, particle_density=2.0, hertz_K=0.5,
          janus=True, janus_theta0=108.0, janus_width=10.0, janus_zeta=(0.1, 0.1),
          lub_mu=0.1, lub_hn=0.67, lub_hcap=0.5)


def _setup(seed):
    shape = (36, 30, 28)
    w = synth.Workload("f1", *shape, seed=seed)
    rng = np.random.default_rng(seed % 1000)
    x, v, om = [], [], []
    for c in ([9.0, 8.0, 7.0], [26.0, 20.0, 19.0], [10.0, 22.0, 20.0]):
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        c = np.array(c)
        half = 0.5 * (2 * 3.5 + 0.6)                   # gap 0.6 < h_n
        x += [c - half * e, c + half * e]
        v += [0.004 * e, -0.004 * e]                     # approaching
        om += [rng.uniform(-2e-3, 2e-3, 3), rng.uniform(-2e-3, 2e-3, 3)]
    q = []
    for _ in range(6):
        a = rng.standard_normal(4)
        q.append(a / np.linalg.norm(a))
    return shape, w.densities(), np.array(x), np.array(v), np.array(om), np.array(q)


def test_lubrication_and_janus_fp64():
    shape, rho, x, v, om, q = _setup(synth.BASE_SEED + 71)
    o, lat = make_pair(shape, rho, x=x, v=v, w=om, **KW)
    # orientations: the same quaternions on both sides
    rec = o.particles()
    rec[:, 9:13] = q
    o.set_particle_state(rec)
    rg = lat.particles()
    rg[:, 9:13] = q
    lat.set_particles(rg)
    done = 0
    for h in (1, 10, 30):
        assert o.step(h - done) == 0
        lat.step(h - done)
        done = h
        e = compare(o, lat)
        ep = compare_particles(o, lat)
        print(f"[f1] t={h}", {k: (f"{v:.1e}" if isinstance(v, float) else v) for k, v in e.items()},
              {k: f"{v:.1e}" for k, v in ep.items()}, flush=True)
        assert e.pop("owner_equal")
        e.pop("df")
        for k, val in e.items():
            assert val <= 1e-12, (h, k, val)
        assert ep["x"] < 1e-12 and ep["v"] < 1e-12 and ep["w"] < 1e-12 and ep["q"] < 1e-12
        for k in ("FH", "FSC", "TSC", "Fliq", "Tliq"):
            assert ep[k] < 1e-12, (h, k, ep[k])
    # the lubrication force was active
    assert np.abs(o.particles()[:, 31:34]).max() > 1e-5


def test_lubrication_and_janus_fp32_step_parity():
    shape, rho, x, v, om, q = _setup(synth.BASE_SEED + 72)
    o, lat = make_pair(shape, rho, x=x, v=v, w=om, precision="fp32", **KW)
    rg = lat.particles()
    rg[:, 9:13] = q
    lat.set_particles(rg)
    lat.step(8)
    sync_state(o, lat)
    for t in range(2):
        assert o.step(1) == 0
        lat.step(1)
        e = compare(o, lat)
        ep = compare_particles(o, lat)
        print(f"[f1] fp32 step {t}", {k: (f"{v:.1e}" if isinstance(v, float) else v)
                                      for k, v in e.items()}, flush=True)
        assert e.pop("owner_equal")
        for k, val in e.items():
            assert val <= (5e-5 if k == "u" else 1e-5), (t, k, val)
        for k in ("FH", "FSC", "TSC", "Fliq", "Tliq"):
            assert ep[k] < 1e-5, (t, k, ep[k])
