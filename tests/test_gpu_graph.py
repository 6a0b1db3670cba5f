"""Steps captured into a HIP graph replay like steps run one by one.

lb_step issues only kernel launches, event records and event waits on the
context's stream and on its side stream (which is joined back by an event),
and it clears its buffers with a fill kernel rather than memsets. A caller can
therefore capture steps into a graph. A graph of an even number of steps ends
on the buffers it starts from (the two population buffers and the old and new
owner maps alternate every step), so it can be replayed any number of times.
Each replay here is checked against a second context stepped eagerly from the
same state, with eager work of both contexts (observables, reads of the
populations, the maps and the spheres, and their synchronisations) between
the replays.

Without moving spheres nothing on the path depends on the order of atomics, so
the two contexts agree bit for bit. With moving spheres the per-sphere FP64
force sums are atomics whose order varies from run to run: the contexts then
agree to the replay tolerance of the restart test (1e-12 of the population
scale in FP64, 1e-6 in FP32) and exactly in the owner maps.
"""
import numpy as np
import pytest

import synth
from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = [
    # precision, spheres ("none", "fixed", "moving"), walls, tolerance (0: bit for bit)
    ("fp64", "none", False, 0.0),
    ("fp32", "none", True, 0.0),
    ("fp64", "fixed", False, 0.0),
    ("fp64", "moving", False, 1e-12),
    ("fp32", "moving", True, 1e-6),
]


@pytest.mark.parametrize("precision,spheres,walls,tol", CASES)
def test_captured_steps_replay_like_eager_steps(precision, spheres, walls, tol):
    import torch
    from paper_2004_04080_amd import Lattice, Params
    print(f"[graph] {precision} spheres={spheres} walls={walls}", flush=True)
    w = synth.Workload("graph", 40, 36, 32, walls=walls, nparticles=6, radius=4.0,
                       seed=synth.BASE_SEED + 71)
    p = Params(40, 36, 32, ncomp=2, tau=(1.0, 1.0), G=0.65, precision=precision,
               walls=walls, wall_u_lo=(0.01, 0.0, 0.0), wall_u_hi=(-0.01, 0.005, 0.0),
               max_particles=0 if spheres == "none" else 8, radius=4.0,
               particle_density=2.0, hertz_K=1.0, particles_fixed=spheres == "fixed")
    rho = w.densities()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager, graph = Lattice(p, rho), Lattice(p, rho)
        if spheres != "none":
            x = w.centres()
            v = np.random.default_rng(5).uniform(-0.02, 0.02, (len(x), 3))
            if spheres == "fixed":
                v = None
            eager.add_particles(x, v)
            graph.add_particles(x, v)
        # eager steps first: the side stream, its events and the frontier
        # list of fixed spheres exist before the capture
        eager.step(2)
        graph.step(2)
        eager.sync()
        graph.sync()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        graph.step(2)                       # recorded, not run

    scale = None
    for r in range(3):
        with torch.cuda.stream(s):
            g.replay()
            eager.step(2)
        fa, fb = eager.populations(), graph.populations()
        oa, ob = eager.owner(), graph.owner()
        if scale is None:
            scale = np.abs(fa).max()
        err = np.abs(fb - fa).max() / scale
        print(f"[graph] replay {r + 1}: populations differ by {err:.1e} of max|f|", flush=True)
        assert np.array_equal(oa, ob)
        if tol == 0.0:
            assert np.array_equal(fa, fb)
        else:
            assert err <= tol
        if spheres == "moving":
            pa, pb = eager.particles(), graph.particles()
            assert np.abs(pb[:, :13] - pa[:, :13]).max() <= 1e-9
        # eager work on the graph's context between replays
        ob_ = graph.observables()
        oe = eager.observables()
        assert ob_.flags == 0 and oe.flags == 0
        np.testing.assert_allclose(ob_.mass, oe.mass, rtol=1e-12 if tol == 0.0 else 1e-9)
        torch.cuda.synchronize()
    eager.close()
    graph.close()
