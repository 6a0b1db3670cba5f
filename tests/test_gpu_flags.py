"""The moving-boundary scheme's speed limit (Sec. 2.3: a sphere may cross at
most half a node per step, so that every node event is a neighbour of the
surface): a sphere moving faster than 0.5 along an axis makes the oracle
refuse the step (LBO_E_SPEED) and the HIP path raise its speed flag, which
lb_observables reports as LB_E_PARTICLE_SPEED; a sphere just under the limit
steps on both sides, with many node events per step, within the FP64 gate."""
import numpy as np
import pytest

import synth
from gpu_util import compare, compare_particles, make_pair, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

SHAPE = (28, 22, 20)
LBO_E_SPEED = -6


def _pair(vx):
    w = synth.Workload("speed", *SHAPE, seed=synth.BASE_SEED + 81)
    x = np.array([[8.3, 10.6, 9.2], [20.1, 11.4, 10.7]])
    v = np.array([[vx, 0.0, 0.0], [0.0, -0.1, 0.05]])
    return make_pair(SHAPE, w.densities(), x=x, v=v, precision="fp64", ncomp=2, G=0.65,
                     radius=3.0, particle_density=1.5)


def test_too_fast_sphere_is_flagged_on_both_sides():
    from paper_2004_04080_amd import binding as B
    o, lat = _pair(0.6)
    assert o.step(1) == LBO_E_SPEED
    lat.step(1)
    ob = lat.observables(raise_on_flag=False)
    print(f"[speed] fast: flags {ob.flags} status {ob.status}", flush=True)
    assert ob.flags & 1 and ob.status == B.LB_E_PARTICLE_SPEED
    with pytest.raises(RuntimeError):
        lat.observables()
    lat.close()


def test_sphere_just_under_the_limit_follows_the_oracle():
    o, lat = _pair(0.45)
    done = 0
    for h in (1, 4):
        assert o.step(h - done) == 0
        lat.step(h - done)
        done = h
        ob = lat.observables()
        assert ob.flags == 0
        e = compare(o, lat)
        ep = compare_particles(o, lat)
        print(f"[speed] slow t={h}", {k: (f"{v:.2e}" if isinstance(v, float) else v)
                                      for k, v in {**e, **ep}.items()}, flush=True)
        assert e.pop("owner_equal")
        e.pop("df")
        for k, v in e.items():
            assert v <= 1e-12, (h, k, v)
        for k, v in ep.items():
            assert v <= 1e-12, (h, k, v)
    lat.close()
