"""The largest boxes the interface accepts: one population plane (nodes x
element size) just below 4 GiB, the bound up to which the kernels address a
plane with 32-bit byte offsets (lb_init rejects larger). One component,
tau = 0.8, a density wave rho(z) = 1 + 0.01 sin(2 pi M z / nz) at rest, with
M = 31 periods along z so that the pressure gradient sets the fluid moving
(max |u| ~ 4e-3 after three steps) well above the rounding of u = j / rho:
* FP32, 1024 x 1024 x 1023 nodes (plane 4 GiB - 4 MiB, 163 GB of populations);
* FP64, 1024 x 1024 x 511 nodes (plane 4 GiB - 8 MiB).
The state depends on z only, so after three steps every x-y column must hold
bit-identical densities and velocities: a column near the end of the
arrays, where the offsets approach 2^32, against one at the start. A column
is compared with the oracle stepping the same wave on a 1 x 1 x nz box (the
same per-node arithmetic, periodic in x and y): FP32 within the FP32 gate
(1e-5; 5e-5 for u), FP64 within 1e-12. Mass is conserved to 2e-9 in FP32
and 1e-13 in FP64: each store of a node's 19 deviations (about 3.3e-3 for the
rest population, 5.6e-4 and 2.8e-4 for the others at this amplitude) rounds
each by at most half an FP32 ulp, 0.5 (2.3e-10 + 6 x 5.8e-11 + 12 x 2.9e-11)
~ 4.7e-10 of a node's unit mass per store, and the state is stored four
times (initial state and three steps)."""
import numpy as np
import pytest

import oracle as O
from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

STEPS = 3
M = 31


def _eps(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision,nz,tol,tol_u,tol_m",
                         [("fp32", 1023, 1e-5, 5e-5, 2e-9), ("fp64", 511, 1e-12, 1e-12, 1e-13)])
def test_largest_plane_box(precision, nz, tol, tol_u, tol_m):
    import torch
    from paper_2004_04080_amd import Lattice, Params
    nx = ny = 1024
    N = nx * ny * nz
    es = 4 if precision == "fp32" else 8
    assert N * es < 2 ** 32 and (N + nx * ny) * es > 2 ** 32 - 2 ** 24
    z = np.arange(nz, dtype=np.float64)
    wave = 1.0 + 0.01 * np.sin(2 * np.pi * M * z / nz)
    print(f"[maxsize] {precision} {nx}x{ny}x{nz}: plane {N * es} bytes", flush=True)
    lat = Lattice(Params(nx, ny, nz, ncomp=1, tau=(0.8, 0.8), precision=precision),
                  np.repeat(wave, nx * ny)[None, :])
    m0 = float(wave.sum()) * nx * ny
    print(f"[maxsize] {precision}: initial state on the GPU", flush=True)
    lat.step(STEPS)
    ob = lat.observables()
    print(f"[maxsize] {precision}: {STEPS} steps done, mass drift {abs(ob.mass[0] - m0) / m0:.2e}",
          flush=True)
    assert ob.flags == 0 and ob.fluid_nodes == N
    assert abs(ob.mass[0] - m0) <= tol_m * m0
    rho, u = lat.fields()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    rho = rho[0].reshape(nz, ny, nx)
    u = u.reshape(nz, ny, nx, 3)
    ref_r, ref_u = rho[:, 0, 0].copy(), u[:, 0, 0].copy()
    for (y, x) in ((ny - 1, nx - 1), (ny - 1, 0), (0, nx - 1), (777, 511)):
        assert np.array_equal(rho[:, y, x], ref_r), ("rho", y, x)
        assert np.array_equal(u[:, y, x], ref_u), ("u", y, x)
    del rho, u
    o = O.Oracle(O.Params(1, 1, nz, ncomp=1, tau=(0.8, 0.8)), wave[None, :])
    assert o.step(STEPS) == 0
    e_r, e_u = _eps(ref_r, o.rho()[0]), _eps(ref_u, o.u())
    print(f"[maxsize] {precision}: column against the oracle: rho {e_r:.1e} u {e_u:.1e} "
          f"(max|u| {np.abs(o.u()).max():.1e})", flush=True)
    assert e_r <= tol and e_u <= tol_u
