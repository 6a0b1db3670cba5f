"""One writer per slot of the fused step's output (Sec. 3.1, steps 6 and 8):
the counting variant of the collide adds 1 for every population it stores,
the post-collision values of fluid nodes, the zeros of solid nodes and the
reflections of the bounce-back links. After s steps every slot of every
component and direction must have been written exactly s times: no
reflected slot has two writers and none is left unwritten. Moving spheres
(node events), walls, open faces and the FP32 and FP64 paths."""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_util import make_pair, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = {
    "spheres-walls-fp32": dict(precision="fp32", walls=True, wall_u_lo=(-0.01, 0, 0),
                               wall_u_hi=(0.01, 0, 0)),
    "spheres-open-fp64": dict(precision="fp64", walls=True, wall_type=(2, 1),
                              wall_u_lo=(0.0, 0.0, 0.01), wall_rho=((1.0, 1.0), (1.0, 1.0))),
    "spheres-periodic-fp32": dict(precision="fp32"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_every_slot_has_one_writer(name):
    import torch
    from paper_2004_04080_amd import binding as B
    shape = (40, 34, 30)
    kw = dict(CASES[name])
    w = synth.Workload("writes", *shape, nparticles=10, radius=4.0, walls=kw.get("walls", False),
                       seed=synth.BASE_SEED + 95)
    rng = np.random.default_rng(95)
    x = w.centres()
    v = 0.05 * (2 * rng.random((len(x), 3)) - 1)
    _, lat = make_pair(shape, w.densities(), x=x, v=v, G=0.65, radius=4.0,
                       particle_density=1.5, **kw)
    counts = torch.zeros(2 * 19 * w.N, dtype=torch.int32, device=lat.device)
    B.check(B.lib().lb_debug_count_writes(lat._ctx, C.c_void_p(counts.data_ptr())),
            "lb_debug_count_writes")
    steps = 4
    own0 = lat.owner()
    lat.step(steps)
    B.check(B.lib().lb_debug_count_writes(lat._ctx, None), "lb_debug_count_writes")
    got = counts.cpu().numpy().reshape(2, 19, w.N)
    bad = np.argwhere(got != steps)
    print(f"[writes] {name}: {int(np.count_nonzero(lat.owner() != own0))} node events, "
          f"counts min {got.min()} max {got.max()}, {len(bad)} slots off", flush=True)
    assert len(bad) == 0, bad[:10]
    assert lat.observables().flags == 0
    lat.close()
