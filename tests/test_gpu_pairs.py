"""Hertz pair forces through a cell list of many cells, against the oracle.

Spheres of radius 1.5 give cells of side d0 = 2R + 1 = 4, so the 160x160x64
box holds 40 x 40 x 16 = 25,600 cells: the cell-start scan then runs over
several tiles of 8,192 cells and carries its running sum from tile to tile.
600 pairs of spheres, 3.6 apart (inside the contact range d0 = 4, outside the
cap 2R), are spread over the whole box, so non-empty cells lie in every tile.
FP64, moving spheres; the pair forces, the other sphere forces, the sphere
state, the map and the fields must agree with the oracle at the bounds of the
other moving-sphere tests.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import compare, compare_particles, make_pair, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

SHAPE = (160, 160, 64)
R = 1.5
GAP = 3.6


def _pairs(seed, npairs=600, excl=6.5):
    rng = np.random.default_rng(seed)
    L = np.array(SHAPE, dtype=float)
    mids = []
    while len(mids) < npairs:
        c = rng.uniform(0, 1, 3) * L
        if mids:
            d = np.array(mids) - c
            d -= L * np.round(d / L)
            if (d ** 2).sum(1).min() < excl * excl:
                continue
        mids.append(c)
    x = []
    for c in mids:
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        x += [(c - 0.5 * GAP * e) % L, (c + 0.5 * GAP * e) % L]
    return np.array(x)


def test_pair_forces_over_many_cells():
    x = _pairs(synth.BASE_SEED + 81)
    side = max(1.0, 2 * R + 1, 2 * R + 0.5)
    ncell = int(np.prod([int(n // side) for n in SHAPE]))
    print(f"[pairs] {len(x)} spheres, {ncell} cells of side {side}", flush=True)
    assert ncell > 3 * 8192
    w = synth.Workload("pairs", *SHAPE, seed=synth.BASE_SEED + 82)
    o, lat = make_pair(SHAPE, w.densities(), x=x, G=0.65, radius=R, particle_density=2.0,
                       hertz_K=0.01, zeta=(0.05, -0.05))
    done = 0
    for h in (1, 2):
        assert o.step(h - done) == 0
        lat.step(h - done)
        done = h
        e = compare(o, lat)
        ep = compare_particles(o, lat)
        print(f"[pairs] t={h}", {k: (f"{v:.1e}" if isinstance(v, float) else v)
                                 for k, v in e.items()},
              {k: f"{v:.1e}" for k, v in ep.items()}, flush=True)
        assert e.pop("owner_equal"), f"maps differ at t={h}"
        e.pop("df")
        for k, val in e.items():
            assert val <= 1e-12, (h, k, val)
        assert ep["x"] < 1e-12 and ep["v"] < 1e-12 and ep["w"] < 1e-12
        for k in ("FH", "Fliq", "Tliq", "FSC", "TSC", "Fd", "Td", "Fc", "Tc"):
            assert ep[k] < 1e-12, (h, k, ep[k])
    # every pair is in contact: the Hertz force acts on every sphere
    fh = np.linalg.norm(o.particles()[:, O.REC["FH"]:O.REC["FH"] + 3], axis=1)
    assert (fh > 0).all(), int((fh == 0).sum())
    assert lat.observables().flags == 0
    lat.close()


def test_pair_paths_agree_across_the_all_pairs_threshold():
    """Up to 1,024 spheres the pair forces come from one kernel over all
    pairs, above that from the cell list. 512 touching pairs (1,024 spheres,
    the first path) and the same pairs with a 1,025th sphere far from all of
    them (the second path) must give the same Hertz and lubrication forces to
    rounding, and the same map outside the added sphere."""
    from paper_2004_04080_amd import Lattice, Params
    x = _pairs(synth.BASE_SEED + 83, npairs=512)
    L = np.array(SHAPE, dtype=float)
    extra = None
    rng = np.random.default_rng(5)
    while extra is None:
        c = rng.uniform(0, 1, 3) * L
        d = x - c
        d -= L * np.round(d / L)
        if np.sqrt((d ** 2).sum(1)).min() > 2 * R + 3:
            extra = c
    v = np.random.default_rng(6).uniform(-0.01, 0.01, (len(x), 3))
    w = synth.Workload("pairs2", *SHAPE, seed=synth.BASE_SEED + 84)
    rho = w.densities()

    def run(xs, vs):
        p = Params(*SHAPE, G=0.65, precision="fp64", radius=R, particle_density=2.0,
                   hertz_K=0.01, lub_mu=0.1, max_particles=len(xs))
        lat = Lattice(p, rho)
        lat.add_particles(xs, vs)
        lat.step(1)
        rec, own = lat.particles(), lat.owner()
        lat.close()
        return rec, own

    ra, oa = run(x, v)
    rb, ob = run(np.vstack([x, extra]), np.vstack([v, np.zeros(3)]))
    fa, fb = ra[:, 31:34], rb[:len(x), 31:34]
    scale = np.abs(fa).max()
    err = np.abs(fb - fa).max() / scale
    print(f"[pairs] {len(x)} against {len(x) + 1} spheres: pair forces differ by {err:.1e} "
          f"of max|F_H| = {scale:.2e}", flush=True)
    assert scale > 0 and err < 1e-13
    keep = ob != len(x) + 1
    assert np.array_equal(oa[keep], ob[keep])
