"""Average domain size (lb_domain_size) against the oracle's numpy definition
(oracle/domain.py) on the HIP path's own fields, and against the closed form
of a single Fourier mode.

Both sides evaluate the same FP64 quantities from the same densities and
assign modes to shells by the same exact integer rule; they differ by the
FFT algorithms and summation orders only, so the bar is 1e-12 relative for
L and for every shell mean (relative to the largest); observed ~1e-15."""
import numpy as np
import pytest

import synth
from gpu_util import requires_gpu
from oracle import domain as D

pytestmark = [pytest.mark.gpu, requires_gpu]


def _lattice(shape, rho, precision="fp32", x=None, **kw):
    from paper_2004_04080_amd import Lattice, Params
    p = Params(*shape, ncomp=2, tau=(1.0, 1.0), G=0.65, precision=precision,
               max_particles=0 if x is None else len(x), radius=kw.pop("radius", 4.0),
               particles_fixed=True, **kw)
    lat = Lattice(p, rho)
    if x is not None:
        lat.add_particles(x)
    return lat


def test_single_mode_closed_form():
    shape = (40, 40, 40)
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = 0.3 * np.cos(2 * np.pi * (3 * x / nx + 4 * y / ny)).ravel()
    lat = _lattice(shape, np.stack([1 + phi, 1 - phi]), precision="fp64")
    L, S = lat.domain_size()
    print(f"[domain] single mode L = {L!r}", flush=True)
    assert abs(L - 8.0) < 1e-11 and S.argmax() == 5
    lat.close()


@pytest.mark.parametrize("spheres", [False, True])
def test_domain_size_matches_oracle(spheres):
    shape = (48, 40, 36)
    w = synth.Workload("dom", *shape, nparticles=5 if spheres else 0, radius=4.0,
                       particles_fixed=True, seed=synth.BASE_SEED + 61)
    lat = _lattice(shape, w.densities(), x=w.centres() if spheres else None)
    lat.step(400)
    L, S = lat.domain_size()
    rho, _ = lat.fields()
    fluid = lat.owner() == 0
    Lo, So = D.domain_size(rho, fluid, shape)
    eS = np.abs(S - So).max() / np.abs(So).max()
    print(f"[domain] spheres={spheres}: L {L:.6f} oracle {Lo:.6f} rel {abs(L - Lo) / Lo:.1e}, "
          f"shells {eS:.1e}", flush=True)
    assert abs(L - Lo) <= 1e-12 * Lo
    assert eS <= 1e-12
    lat.close()
