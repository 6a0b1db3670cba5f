"""State written from the host and the per-phase timing, through the C
interface.

lb_set_populations: the oracle's FP64 populations after 12 steps of a box
with fixed spheres and walls are written into a fresh context at step 0
(same map, sphere records at rest): reading them back gives the same values
bit for bit (FP64), and both sides then step on together within 1e-12 (FP64;
in FP32 the written values are rounded to the storage once, and the two
paths agree within the FP32 gate after one step). The map of the
populations is the context's own, so every pulled slot of every fluid node
is written, including those a bounce-back link fills.

lb_timing / lb_timing_read: with timing on, every phase that runs records its
intervals per step (moments, fill, collide and, with moving spheres, the
integration once; the sphere phase twice, the map update on the side stream
and the node events on the library's stream), the main-stream phases sum to
less than the wall time of the steps, turning timing off stops the counts,
and turning it on again clears them."""
import time

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import compare, make_pair, perm_gpu_for_oracle, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

SHAPE = (22, 18, 16)


def _kw():
    return dict(ncomp=2, G=0.65, g=(2e-5, 0.0, -1e-5), walls=True, wall_u_lo=(-0.01, 0, 0),
                wall_u_hi=(0.01, 0, 0), radius=3.0, particles_fixed=True)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_set_populations_from_the_oracle(precision, tol):
    w = synth.Workload("xfer", *SHAPE, nparticles=4, radius=3.0, seed=synth.BASE_SEED + 71,
                       walls=True)
    o, lat = make_pair(SHAPE, w.densities(), x=w.centres(), precision=precision, **_kw())
    o.step(12)                                  # the GPU context stays at step 0
    assert np.array_equal(o.owner(), lat.owner())
    inv = np.argsort(perm_gpu_for_oracle())     # oracle direction of each GPU direction
    f_o = o.f()
    lat.set_populations(f_o[:, inv, :])
    back = lat.populations()[:, perm_gpu_for_oracle(), :]
    fluid = o.owner() == 0
    if precision == "fp64":
        assert np.array_equal(back[:, :, fluid], f_o[:, :, fluid])
    else:
        rel = np.abs(back[:, :, fluid] - f_o[:, :, fluid]).max() / np.abs(f_o[:, :, fluid]).max()
        assert rel < 2 ** -20                   # one rounding of each deviation to FP32
    assert np.all(back[:, :, ~fluid] == 0.0)
    for h in (1, 5):
        o.step(1 if h == 1 else 4)
        lat.step(1 if h == 1 else 4)
        e = compare(o, lat)
        print(f"[transfer] {precision} +{h}", {k: (f"{v:.2e}" if isinstance(v, float) else v)
                                               for k, v in e.items()}, flush=True)
        assert e.pop("owner_equal")
        if precision == "fp32":
            e.pop("df")                          # the oracle's df carries no FP32 rounding
            if h > 1:
                break
        for k, v in e.items():
            assert v <= (5 * tol if k == "u" else tol), (precision, h, k, v)
    lat.close()


def test_phase_timing_counts_and_clears():
    from paper_2004_04080_amd import Lattice, Params
    w = synth.Workload("tim", 40, 36, 32, nparticles=6, radius=4.0, seed=synth.BASE_SEED + 72)
    p = Params(40, 36, 32, ncomp=2, G=0.65, radius=4.0, max_particles=6)
    lat = Lattice(p, w.densities())
    lat.add_particles(w.centres())
    lat.step(2)
    lat.timing(True)
    lat.sync()
    t0 = time.perf_counter()
    lat.step(3)
    lat.sync()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ph = lat.timing_read()
    print("[timing]", {k: (round(v[0], 4), v[1]) for k, v in ph.items()}, f"wall {wall_ms:.3f} ms",
          flush=True)
    for name, per_step in (("density", 1), ("spheres", 2), ("fill", 1), ("collide", 1),
                           ("integrate", 1)):
        assert ph[name][1] == 3 * per_step and ph[name][0] > 0.0, name
    # the side stream overlaps the moments, so only the main-stream phases add up
    main = sum(ph[k][0] for k in ("density", "fill", "collide", "integrate"))
    assert main <= wall_ms
    lat.timing(False)
    lat.step(2)
    assert lat.timing_read()["collide"][1] == 3
    lat.timing(True)
    assert all(v == (0.0, 0) for v in lat.timing_read().values())
    lat.close()
