"""Fixed spheres in a uniform two-component fluid at rest (G = 0), through the
C interface, in FP64 and FP32. Every link then carries the bounce-back of the
equilibrium, 2 w_i rho c_i, and the links into any finite solid set sum to
zero in force and torque. A sphere on its own, also across the periodic
seams, therefore feels no force and no torque. Two spheres 7.58 apart
(R = 3.7: no shared node, but solid nodes of one next to solid nodes of the
other, so neither has the links the other covers) feel opposite forces
whose torques cancel about a common point. The oracle pins the same
identities on the CPU (test_oracle_particles.py, with overlapping spheres,
which lb_add_particles refuses); here the HIP path must reproduce them to
the rounding of its FP64 sums, and its forces must equal the oracle's."""
import numpy as np
import pytest

import oracle as O
from gpu_util import make_pair, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

SHAPE = (26, 22, 24)
X = np.array([[5.3, 4.1, 6.9], [10.8, 9.3, 7.3],     # pair with neighbouring solid nodes
              [25.4, 11.3, 12.6],                     # across the x seam
              [14.1, 17.6, 1.2],                      # across the z seam
              [18.9, 3.3, 17.7]])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resting_spheres_in_resting_fluid(precision):
    print(f"[rest] {precision}", flush=True)
    n = int(np.prod(SHAPE))
    o, lat = make_pair(SHAPE, np.ones((2, n)), x=X, precision=precision, ncomp=2, G=0.0,
                       radius=3.7, particles_fixed=True)
    o.step(1)
    lat.step(1)
    R = O.REC
    rg, ro = lat.particles(), o.particles()
    scale = ro[:, R["flabs"]].max()
    Fg, Tg = rg[:, R["Fliq"]:R["Fliq"] + 3], rg[:, R["Tliq"]:R["Tliq"] + 3]
    Fo = ro[:, R["Fliq"]:R["Fliq"] + 3]
    print(f"[rest] {precision}: max |F| of lone spheres {np.abs(Fg[2:]).max():.1e}, "
          f"|F| of the pair {np.abs(Fg[0]).max():.2f}, scale {scale:.1f}", flush=True)
    assert np.abs(rg[:, R["flabs"]] - ro[:, R["flabs"]]).max() <= 1e-12 * scale
    assert np.abs(Fg[2:]).max() <= 1e-13 * scale and np.abs(Tg[2:]).max() <= 1e-12 * scale
    assert np.abs(Fg - Fo).max() <= 1e-12 * scale
    assert np.abs(Fo[0]).max() > 1.0                 # the pair does feel a force
    assert np.abs(Fg[0] + Fg[1]).max() <= 1e-13 * scale
    Tc = Tg[0] + Tg[1] + np.cross(X[1] - X[0], Fg[1])
    assert np.abs(Tc).max() <= 1e-12 * scale
    assert np.array_equal(lat.owner(), o.owner())
    lat.close()
