"""Reverse-mode derivative of the loss through the HIP step (lb_backward)
against the oracle's forward-mode (dual number) derivative, and against
central differences of the HIP forward run itself.

Loss: L = sum over fluid nodes of |3 sum_i w_i phi(n + c_i) c_i|^2 with
phi = psi_A - psi_B on the final state. Parameters: the coupling G, the body
acceleration g and the initial density field of component A. Spheres are
static obstacles, so the map is fixed and L is differentiable.

Tolerances. FP64: the adjoint and the tangent-linear run compute the same
derivative by different summation orders, so they agree to rounding
amplified by the step count: gated at 1e-10 relative (about 1e-13 is
observed; each test prints what it observes). The per-step dot-product test
<J d, s> = <d, J^T s> pairs the oracle's tangent of the whole final
pseudo-potential field with the reverse sweep seeded by an arbitrary s, at
1e-10 of the sum of |s_n (J d)_n|. The bar of 1e-4 relative against central differences is
checked on the HIP forward in FP64. FP32: the reverse sweep is exact for the FP32
forward, whose trajectory departs from FP64 by the storage rounding of the
deviations (2^-24 of O(1) populations, about 1e-5 of the O(1e-2) deviations
that carry the loss), so FP32 gradients are gated at 1e-4 relative to FP64
(observed 3e-7 on the small box and 1e-5 on the 64^3 box over 500 steps).
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _case(shape=(14, 12, 10), walls=False, nsph=2, steps=13, every=5):
    nx, ny, nz = shape
    w = synth.Workload("adj", nx, ny, nz, nparticles=nsph, radius=2.5, particles_fixed=True,
                       walls=walls, seed=synth.BASE_SEED + 41)
    rho = w.densities()
    x = np.array([[3.2, 3.6, 3.3], [9.1, 8.4, 5.6], [6.0, 2.0, 5.0]])[:nsph]
    kw = dict(ncomp=2, tau=(1.0, 1.0), G=0.65, g=(1e-6, 2e-7, 0.0), walls=walls,
              radius=2.5, particles_fixed=True)
    return shape, rho, x, kw, steps, every


def _gpu_grad(shape, rho, x, kw, steps, every, precision="fp64", G=None, g=None):
    from paper_2004_04080_amd import Lattice, Params
    kw = dict(kw)
    if G is not None:
        kw["G"] = G
    if g is not None:
        kw["g"] = g
    p = Params(*shape, precision=precision, max_particles=len(x), checkpoint_every=every,
               max_record_steps=steps, **kw)
    lat = Lattice(p, rho)
    if len(x):
        lat.add_particles(x)
    lat.step(steps)
    L, sA, sB = lat.loss(seeds=True)
    dA0, dG, dg = lat.backward(sA, sB)
    out = (L, dA0.cpu().numpy(), dG, dg)
    lat.close()
    return out


def _gpu_loss(shape, rho, x, kw, steps, precision="fp64", **over):
    from paper_2004_04080_amd import Lattice, Params
    kw = {**kw, **over}
    p = Params(*shape, precision=precision, max_particles=len(x), **kw)
    lat = Lattice(p, rho)
    if len(x):
        lat.add_particles(x)
    lat.step(steps)
    L = lat.loss()
    lat.close()
    return L


def _oracle_params(shape, kw):
    return O.Params(*shape, ncomp=2, tau=kw["tau"], G=kw["G"], sc_norm=1.0, g=kw["g"],
                    walls=kw["walls"], radius=kw["radius"], particles_fixed=True)


@pytest.mark.parametrize("walls,every", [(False, 5), (True, 4), (False, 13)])
def test_adjoint_matches_oracle_tangent_fp64(walls, every):
    shape, rho, x, kw, steps, _ = _case(walls=walls, every=every)
    print(f"[adjoint] walls={walls} every={every} steps={steps}", flush=True)
    L, dA0, dG, dg = _gpu_grad(shape, rho, x, kw, steps, every)
    po = _oracle_params(shape, kw)
    Lo, dGo = O.loss_tangent(po, rho, steps, dG=1.0, x=x)
    assert abs(L - Lo) <= 1e-12 * abs(Lo)
    print(f"[adjoint] rel err dL/dG {abs(dG - dGo) / abs(dGo):.2e}", flush=True)
    assert abs(dG - dGo) <= 1e-10 * abs(dGo), (dG, dGo)
    for d in range(2):
        e = np.zeros(3)
        e[d] = 1.0
        _, dgo = O.loss_tangent(po, rho, steps, dg=e, x=x)
        print(f"[adjoint] rel err dL/dg[{d}] {abs(dg[d] - dgo) / abs(dgo):.2e}", flush=True)
        assert abs(dg[d] - dgo) <= 1e-10 * abs(dgo), (d, dg[d], dgo)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(po.N)
    _, dvo = O.loss_tangent(po, rho, steps, drhoA=v, x=x)
    print(f"[adjoint] rel err v.dL/drhoA0 {abs(dA0 @ v - dvo) / abs(dvo):.2e}", flush=True)
    assert abs(dA0 @ v - dvo) <= 1e-10 * np.abs(dA0).sum() * np.abs(v).max()
    # single entries: a node next to a sphere surface and a node in the bulk
    o = O.Oracle(po, rho)
    o.add_particles(x)
    own = o.owner()
    fluid = np.flatnonzero(own == 0)
    near = [n for n in fluid if dA0[n] != 0.0][:1]
    for n in near + [int(fluid[len(fluid) // 2])]:
        e = np.zeros(po.N)
        e[n] = 1.0
        _, dno = O.loss_tangent(po, rho, steps, drhoA=e, x=x)
        assert abs(dA0[n] - dno) <= 1e-10 * np.abs(dA0).max(), (n, dA0[n], dno)
    assert np.all(dA0[own != 0] == 0.0)


@pytest.mark.parametrize("steps,walls", [(1, False), (1, True), (2, False), (6, True)])
def test_adjoint_dot_product(steps, walls):
    """<J d, s> = <d, J^T s> for the map from (rho_A0, G, g) to the final
    pseudo-potential field (fluid densities and the virtual densities of the
    frontier): J d from the oracle's dual-number run, J^T s from lb_backward
    seeded with a random s on every node that carries a pseudo-potential.
    One step checks the adjoint of a single step (collide, bounce-back, fill,
    moments); more steps check their composition through the checkpoints."""
    import torch
    from paper_2004_04080_amd import Lattice, Params
    shape, rho, x, kw, _, _ = _case(walls=walls)
    p = Params(*shape, precision="fp64", max_particles=len(x), checkpoint_every=max(1, steps // 2),
               max_record_steps=steps, **kw)
    lat = Lattice(p, rho)
    lat.add_particles(x)
    lat.step(steps)
    po = _oracle_params(shape, kw)
    rng = np.random.default_rng(100 + steps)
    v = rng.standard_normal(po.N)
    dGd, dgd = 0.7, (0.4, -0.3, 0.2)
    psi, Jd = O.psi_tangent(po, rho, steps, dG=dGd, dg=dgd, drhoA=v, x=x)
    carries = (lat.owner() == 0) | (np.abs(psi).sum(0) > 0)
    s = rng.standard_normal((2, po.N)) * carries[None, :]
    sA = torch.tensor(s[0], dtype=torch.float64, device=lat.device)
    sB = torch.tensor(s[1], dtype=torch.float64, device=lat.device)
    dA0, dG, dg = lat.backward(sA, sB)
    lat.close()
    lhs = float((s * Jd).sum())
    rhs = float(dA0.cpu().numpy() @ v + dG * dGd + np.dot(dg, dgd))
    scale = float(np.abs(s * Jd).sum())
    print(f"[adjoint-dot] steps={steps} walls={walls} <Jd,s>={lhs:.15e} <d,J^T s>={rhs:.15e} "
          f"rel {abs(lhs - rhs) / scale:.2e}", flush=True)
    assert abs(lhs - rhs) <= 1e-10 * scale


def test_adjoint_matches_central_differences_fp64():
    """The 1e-4 bar against central differences of the HIP forward run, on a
    32^3 box with 6 fixed spheres of radius 4 over 40 steps (checkpoints
    every 15)."""
    shape = (32, 32, 32)
    w = synth.Workload("adjfd", *shape, nparticles=6, radius=4.0, particles_fixed=True,
                       g=(1e-6, 0.0, 0.0), seed=synth.BASE_SEED + 43)
    rho, x = w.densities(), w.centres()
    kw = dict(ncomp=2, tau=(1.0, 1.0), G=0.65, g=(1e-6, 0.0, 0.0), walls=False, radius=4.0,
              particles_fixed=True)
    steps = 40
    L, dA0, dG, dg = _gpu_grad(shape, rho, x, kw, steps, 15)
    h = 1e-4 * kw["G"]
    fd = (_gpu_loss(shape, rho, x, kw, steps, G=kw["G"] + h)
          - _gpu_loss(shape, rho, x, kw, steps, G=kw["G"] - h)) / (2 * h)
    print(f"[adjoint-fd] rel err dL/dG {abs(dG - fd) / abs(fd):.2e}", flush=True)
    assert abs(dG - fd) <= 1e-4 * abs(fd), (dG, fd)
    h = 1e-5
    fd = (_gpu_loss(shape, rho, x, kw, steps, g=(1e-6 + h, 0, 0))
          - _gpu_loss(shape, rho, x, kw, steps, g=(1e-6 - h, 0, 0))) / (2 * h)
    print(f"[adjoint-fd] rel err dL/dg_x {abs(dg[0] - fd) / abs(fd):.2e}", flush=True)
    assert abs(dg[0] - fd) <= 1e-4 * abs(fd), (dg[0], fd)
    v = np.random.default_rng(11).standard_normal(w.N)
    h = 1e-4
    rp, rm = rho.copy(), rho.copy()
    rp[0] += h * v
    rm[0] -= h * v
    fd = (_gpu_loss(shape, rp, x, kw, steps) - _gpu_loss(shape, rm, x, kw, steps)) / (2 * h)
    print(f"[adjoint-fd] rel err v.dL/drhoA0 {abs(dA0 @ v - fd) / abs(fd):.2e}", flush=True)
    assert abs(dA0 @ v - fd) <= 1e-4 * abs(fd), (dA0 @ v, fd)


def test_adjoint_fp32_close_to_fp64():
    shape, rho, x, kw, steps, every = _case()
    _, a64, g64, dg64 = _gpu_grad(shape, rho, x, kw, steps, every, "fp64")
    _, a32, g32, dg32 = _gpu_grad(shape, rho, x, kw, steps, every, "fp32")
    print(f"[adjoint-fp32] rel err dL/dG {abs(g32 - g64) / abs(g64):.2e}, dL/drhoA0 "
          f"{np.abs(a32 - a64).max() / np.abs(a64).max():.2e}", flush=True)
    assert abs(g32 - g64) <= 1e-4 * abs(g64)
    assert np.abs(np.array(dg32) - dg64)[:2].max() <= 1e-4 * np.abs(dg64[:2]).max()
    assert np.abs(a32 - a64).max() <= 1e-4 * np.abs(a64).max()


def test_backward_rejects_what_it_cannot_differentiate():
    from paper_2004_04080_amd import Lattice, LBError, Params
    shape, rho, x, kw, steps, every = _case(steps=3)
    # moving spheres
    p = Params(*shape, precision="fp64", max_particles=2, checkpoint_every=2,
               max_record_steps=3, **{**kw, "particles_fixed": False})
    lat = Lattice(p, rho)
    lat.add_particles(x)
    lat.step(2)
    L, sA, sB = lat.loss(seeds=True)
    with pytest.raises(LBError):
        lat.backward(sA, sB)
    lat.close()
    # nothing recorded
    p = Params(*shape, precision="fp64", max_particles=2, checkpoint_every=2,
               max_record_steps=3, **kw)
    lat = Lattice(p, rho)
    lat.add_particles(x)
    L, sA, sB = lat.loss(seeds=True)
    with pytest.raises(LBError):
        lat.backward(sA, sB)
    lat.close()


def test_autograd_function_matches_backward():
    import torch
    from paper_2004_04080_amd import Params
    from paper_2004_04080_amd.autograd import rollout_loss
    shape, rho, x, kw, steps, every = _case()
    base = {k: v for k, v in kw.items() if k not in ("G", "g")}
    p = Params(*shape, precision="fp64", **base)
    rA = torch.tensor(rho[0], dtype=torch.float64, requires_grad=True)
    G = torch.tensor(kw["G"], dtype=torch.float64, requires_grad=True)
    g = torch.tensor(kw["g"], dtype=torch.float64, requires_grad=True)
    L = rollout_loss(p, rA, G, g, torch.tensor(rho[1]), steps=steps, x=x, checkpoint_every=every)
    (2.0 * L).backward()
    L0, dA0, dG, dg = _gpu_grad(shape, rho, x, kw, steps, every)
    assert float(L.detach()) == L0
    np.testing.assert_allclose(rA.grad.numpy(), 2.0 * dA0, rtol=1e-13, atol=0)
    assert abs(float(G.grad) - 2.0 * dG) <= 1e-13 * abs(dG)
    np.testing.assert_allclose(g.grad.numpy(), 2.0 * np.asarray(dg), rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_differentiation_box_full_size(precision):
    """The differentiation box at full size: 64^3, 50 fixed spheres of radius
    4, g_x = 1e-6, 500 steps with a checkpoint every 50. FP64: adjoint against
    central differences of the HIP forward (G relative step 1e-4, g_x absolute
    1e-8, rho_A0 along a random direction absolute 1e-4), 1e-4 relative.
    FP32: gradients against the FP64 adjoint, 1e-4 relative.

    The g_x step is 1e-8 (1% of g_x): over 500 steps of spinodal growth L
    bends in g_x enough that a step of 1e-5 leaves a truncation error of
    2.5e-3, while a step of 1e-10 meets the run-to-run rounding of L (about
    1e-13 of L after amplification by the unstable modes)."""
    w = synth.workload("C5")
    shape = (w.nx, w.ny, w.nz)
    rho, x = w.densities(), w.centres()
    kw = dict(ncomp=2, tau=w.tau, G=w.G, g=w.g, walls=False, radius=w.radius,
              particles_fixed=True)
    steps, every = w.steps, 50
    print(f"[adjoint-C5] {precision} {shape} {len(x)} spheres {steps} steps", flush=True)
    L, dA0, dG, dg = _gpu_grad(shape, rho, x, kw, steps, every, precision)
    if precision == "fp32":
        _, a64, g64, dg64 = _gpu_grad(shape, rho, x, kw, steps, every, "fp64")
        eG = abs(dG - g64) / abs(g64)
        eg = abs(dg[0] - dg64[0]) / abs(dg64[0])
        eA = np.abs(dA0 - a64).max() / np.abs(a64).max()
        print(f"[adjoint-C5] fp32 vs fp64: dG {eG:.2e} dg_x {eg:.2e} drhoA0 {eA:.2e}", flush=True)
        assert eG <= 1e-4 and eg <= 1e-4 and eA <= 1e-4
        return
    h = 1e-4 * w.G
    fd = (_gpu_loss(shape, rho, x, kw, steps, G=w.G + h)
          - _gpu_loss(shape, rho, x, kw, steps, G=w.G - h)) / (2 * h)
    print(f"[adjoint-C5] dL/dG adjoint {dG:.10e} fd {fd:.10e}", flush=True)
    assert abs(dG - fd) <= 1e-4 * abs(fd)
    h = 1e-8
    gp, gm = list(w.g), list(w.g)
    gp[0] += h
    gm[0] -= h
    fd = (_gpu_loss(shape, rho, x, kw, steps, g=tuple(gp))
          - _gpu_loss(shape, rho, x, kw, steps, g=tuple(gm))) / (2 * h)
    print(f"[adjoint-C5] dL/dg_x adjoint {dg[0]:.10e} fd {fd:.10e}", flush=True)
    assert abs(dg[0] - fd) <= 1e-4 * abs(fd)
    v = np.random.default_rng(13).standard_normal(w.N)
    h = 1e-4
    rp, rm = rho.copy(), rho.copy()
    rp[0] += h * v
    rm[0] -= h * v
    fd = (_gpu_loss(shape, rp, x, kw, steps) - _gpu_loss(shape, rm, x, kw, steps)) / (2 * h)
    print(f"[adjoint-C5] v.dL/drhoA0 adjoint {dA0 @ v:.10e} fd {fd:.10e}", flush=True)
    assert abs(dA0 @ v - fd) <= 1e-4 * abs(fd)
