"""Sphere map of the HIP path against the oracle where spheres share nodes.

A map update writes the nodes of a sphere with plain stores when no other
centre lies within 2R + 1/2, and by an atomic lowest-index-wins claim
otherwise; the frontier and node-event lists are then built per sphere. Here
two spheres without Hertz repulsion run into each other (their balls
overlap, so nodes lie inside both) beside an isolated sphere, once in the
middle of the box and once across the periodic boundary; the maps must agree
bit for bit with the oracle's and the fields and sphere forces to the FP64
bound. A last case checks that a restored state replaces the cached
frontier list of fixed spheres.
"""
import numpy as np
import pytest

import synth
from gpu_util import compare, compare_particles, make_pair, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

R = 4.0
SHAPE = (40, 36, 32)


def _shared_nodes(x, shape, R):
    """Nodes within R of both of the first two centres (periodic)."""
    L = np.array(shape, dtype=float)
    g = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1).reshape(-1, 3)
    d = [g - x[i] for i in (0, 1)]
    d = [di - L * np.round(di / L) for di in d]
    inside = [(di ** 2).sum(1) < R * R for di in d]
    return int((inside[0] & inside[1]).sum())


@pytest.mark.parametrize("where", ["middle", "periodic"])
def test_overlapping_spheres_share_nodes_like_the_oracle(where):
    if where == "middle":
        x = np.array([[16.0, 18.0, 16.0], [24.04, 18.2, 16.1], [8.0, 6.0, 25.0]])
    else:   # the pair straddles x = 0
        x = np.array([[36.0, 18.0, 16.0], [4.04, 18.2, 15.9], [20.0, 6.0, 25.0]])
    v = np.array([[0.05, 0.0, 0.001], [-0.05, 0.001, 0.0], [0.005, -0.004, 0.003]])
    om = np.array([[0.0, 0.0, 0.01], [0.01, 0.0, 0.0], [0.0, 0.004, 0.0]])
    w = synth.Workload("near", *SHAPE, seed=synth.BASE_SEED + 61)
    o, lat = make_pair(SHAPE, w.densities(), x=x, v=v, w=om, G=0.65, radius=R,
                       particle_density=40.0, hertz_K=0.0, zeta=(0.05, -0.05))
    done = 0
    shared = 0
    for h in (1, 10, 25):
        assert o.step(h - done) == 0
        lat.step(h - done)
        done = h
        e = compare(o, lat)
        print(f"[map] {where} t={h}", {k: (f"{v:.1e}" if isinstance(v, float) else v)
                                       for k, v in e.items()}, flush=True)
        assert e.pop("owner_equal"), f"maps differ at t={h}"
        e.pop("df")
        for k, val in e.items():
            assert val <= 1e-12, (h, k, val)
        ep = compare_particles(o, lat)
        assert ep["x"] < 1e-12 and ep["v"] < 1e-12 and ep["w"] < 1e-12
        for k in ("Fliq", "Tliq", "Fd", "Td", "Fc", "Tc", "FSC", "TSC"):
            assert ep[k] < 1e-12, (h, k, ep[k])
        rec = o.particles()
        d = rec[1, 0:3] - rec[0, 0:3]
        d -= np.array(SHAPE) * np.round(d / np.array(SHAPE))
        shared = max(shared, _shared_nodes(rec[:, 0:3], SHAPE, R))
        print(f"[map] {where} t={h}: centre distance {np.linalg.norm(d):.3f}, "
              f"nodes inside both balls {_shared_nodes(rec[:, 0:3], SHAPE, R)}", flush=True)
    assert shared > 0, "the pair never overlapped: the shared-node path went untested"
    assert lat.observables().flags == 0


def test_restored_state_replaces_the_cached_frontier_of_fixed_spheres():
    from paper_2004_04080_amd import Lattice, Params
    w = synth.Workload("fixmap", *SHAPE, seed=synth.BASE_SEED + 62)
    kw = dict(G=0.65, radius=R, particles_fixed=True, max_particles=3, zeta=(0.1, -0.1))
    xa = np.array([[10.0, 10.0, 10.0], [28.0, 20.0, 12.0], [20.0, 28.0, 24.0]])
    xb = xa + np.array([3.0, -2.0, 4.0])
    a = Lattice(Params(*SHAPE, precision="fp64", **kw), w.densities())
    a.add_particles(xa)
    a.step(5)
    blob = a.state()
    b = Lattice(Params(*SHAPE, precision="fp64", **kw), w.densities())
    b.add_particles(xb)
    b.step(3)               # b now holds the frontier list of its own map
    b.set_state(blob)
    a.step(6)
    b.step(6)
    fa, fb = a.populations(), b.populations()
    assert np.array_equal(a.owner(), b.owner())
    err = np.abs(fb - fa).max()
    print(f"[map] restored fixed spheres: max |df| = {err:.1e}", flush=True)
    assert err <= 1e-14
    a.close()
    b.close()


def test_sphere_wider_than_the_box_is_listed_once():
    """A sphere of radius 5.2 in a 12 x 13 x 14 box: its bounding box (up to
    13 nodes a side) is wider than the 12-node axis, so its walk sees a node
    twice unless it walks one period only. Moving, in FP64, against the
    oracle."""
    shape = (12, 13, 14)
    w = synth.Workload("tiny", *shape, seed=synth.BASE_SEED + 63)
    x = np.array([[5.7, 6.1, 7.3]])
    v = np.array([[0.03, -0.02, 0.01]])
    om = np.array([[0.0, 0.01, 0.02]])
    o, lat = make_pair(shape, w.densities(), x=x, v=v, w=om, G=0.65, radius=5.2,
                       particle_density=2.0, zeta=(0.1, -0.1))
    done = 0
    for h in (1, 10, 30):
        assert o.step(h - done) == 0
        lat.step(h - done)
        done = h
        e = compare(o, lat)
        print(f"[map] tiny box t={h}", {k: (f"{v:.1e}" if isinstance(v, float) else v)
                                        for k, v in e.items()}, flush=True)
        assert e.pop("owner_equal")
        e.pop("df")
        for k, val in e.items():
            assert val <= 1e-12, (h, k, val)
        ep = compare_particles(o, lat)
        assert ep["x"] < 1e-12 and ep["v"] < 1e-12
        for k in ("Fliq", "Tliq", "Fd", "Td", "Fc", "Tc", "FSC", "TSC"):
            assert ep[k] < 1e-12, (h, k, ep[k])
    assert (o.owner() == 0).sum() > 0 and (o.owner() == 1).sum() > 0


def test_capacity_without_spheres_steps_like_no_spheres():
    """A context sized for spheres but given none steps as one without sphere
    capacity. It runs the collide that reads the owner map (all fluid here),
    a separate instance of the same arithmetic, so rounding may differ in the
    last place; the fields must agree to the FP32 bound."""
    from paper_2004_04080_amd import Lattice, Params
    shape = (24, 20, 16)
    w = synth.Workload("nosph", *shape, seed=synth.BASE_SEED + 64)
    a = Lattice(Params(*shape, precision="fp32", G=0.65), w.densities())
    b = Lattice(Params(*shape, precision="fp32", G=0.65, max_particles=8, radius=3.0),
                w.densities())
    a.step(25)
    b.step(25)
    fa, fb = a.populations(), b.populations()
    err = float(np.abs(fb - fa).max() / np.abs(fa).max())
    print(f"[map] capacity without spheres: {err:.1e}", flush=True)
    assert err <= 1e-6
    assert b.num_particles() == 0 and b.observables().flags == 0
    a.close()
    b.close()
