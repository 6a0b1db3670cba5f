"""Whole-step brute force: the oracle against an independent 50-digit
transcription of the step (tests/brute_lb.py) on tiny boxes.

The cases cover one and two components, body force, unequal relaxation
times (mixture viscosity), moving walls, wetting constants, moving and
spinning spheres whose motion destroys and creates fluid nodes, and Hertz
contacts between spheres and with the walls. Agreement is required to
1e-12 relative (FP64 rounding of the oracle), three steps deep.
"""
import numpy as np
import pytest

import oracle as O
from brute_lb import Brute


def _rel(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale


def _compare(o, br, parts_report=None, tol=1e-12):
    c, _ = O.lattice()
    fo = o.f()
    fb = br.populations(c)
    assert _rel(fo, fb) < tol
    own_b = np.array([br.own[n] for n in br.nodes])
    assert np.array_equal(o.owner(), own_b)
    rec = o.particles()
    for p, P in enumerate(br.parts):
        for key, n in (("x", 3), ("v", 3), ("w", 3), ("q", 4)):
            ref = np.array([float(a) for a in P[key]])
            got = rec[p, O.REC[key]:O.REC[key] + n]
            scale = max(np.abs(ref).max(), 1.0 if key in ("x", "q") else 1e-30)
            assert np.abs(got - ref).max() / scale < tol, (key, p, got, ref)
    if parts_report is not None:
        names = dict(Fd="Fd", Td="Td", Fc="Fc", Tc="Tc", FH="FH", FSC="FSC", TSC="TSC",
                     Fl="Fliq", Tl="Tliq")
        for p, A in enumerate(parts_report):
            # forces are sums of many terms of both signs: compare against the
            # size of their terms (sum over links of |F_link|)
            scale = max(rec[p, O.REC["flabs"]], 1e-12)
            for kb, ko in names.items():
                ref = np.array([float(a) for a in A[kb]])
                got = rec[p, O.REC[ko]:O.REC[ko] + 3]
                assert np.abs(got - ref).max() / scale < tol, (kb, p, got, ref)


def _density(shape, ncomp, seed):
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    return 1.0 + 0.05 * (2 * rng.random((ncomp, N)) - 1)


def test_brute_one_component_body_force():
    shape = (5, 4, 3)
    rho = _density(shape, 1, 1)
    rng = np.random.default_rng(2)
    u0 = 0.03 * (2 * rng.random((60, 3)) - 1)
    p = O.Params(*shape, ncomp=1, tau=(0.8,), g=(1e-3, -2e-3, 5e-4))
    o = O.Oracle(p, rho, u0)
    br = Brute(shape, 1, (0.8,), 0.0, 1.0, (1e-3, -2e-3, 5e-4), rho, u0)
    for _ in range(3):
        o.step(1)
        br.step()
        _compare(o, br)


def test_brute_two_components_shan_chen():
    shape = (4, 5, 4)
    rho = _density(shape, 2, 3)
    p = O.Params(*shape, ncomp=2, tau=(0.7, 1.3), G=0.9, sc_norm=1.0, g=(0, 1e-3, 0))
    o = O.Oracle(p, rho)
    br = Brute(shape, 2, (0.7, 1.3), 0.9, 1.0, (0, 1e-3, 0), rho)
    for _ in range(3):
        o.step(1)
        br.step()
        _compare(o, br)


@pytest.mark.parametrize("case", ["moving", "contact", "walls"])
def test_brute_with_spheres(case):
    if case == "moving":
        shape, R = (5, 5, 5), 1.4
        x = np.array([[1.3, 1.6, 2.2], [3.7, 3.4, 1.1]])
        v = np.array([[0.31, -0.12, 0.07], [-0.2, 0.25, 0.33]])
        w = np.array([[0.05, -0.02, 0.11], [0.0, 0.07, -0.04]])
        kw = dict(walls=False)
        hertz = (20.0, 2 * R + 1, 2 * R)
    elif case == "contact":
        shape, R = (6, 5, 5), 1.2
        x = np.array([[1.5, 2.1, 2.4], [3.9, 2.6, 2.2]])   # closer than 2R+1
        v = np.array([[0.1, 0.0, 0.05], [-0.15, 0.02, 0.0]])
        w = np.array([[0.0, 0.0, 0.2], [0.1, 0.0, 0.0]])
        kw = dict(walls=False)
        hertz = (0.5, 2 * R + 1, 2 * R)
    else:
        shape, R = (5, 4, 7), 1.3
        x = np.array([[2.2, 1.7, 2.3], [0.6, 2.9, 4.6]])
        v = np.array([[0.2, 0.1, -0.25], [0.05, -0.3, 0.2]])
        w = np.array([[0.1, 0.0, 0.0], [0.0, -0.1, 0.05]])
        kw = dict(walls=True, wall_u_lo=(-0.02, 0.0, 0.0), wall_u_hi=(0.01, 0.03, 0.0))
        hertz = (0.5, 2 * R + 1, 2 * R)
    rho = _density(shape, 2, 4)
    zeta = (0.1, -0.05)
    p = O.Params(*shape, ncomp=2, tau=(1.0, 0.9), G=0.65, sc_norm=1.0, g=(2e-4, 0, 0),
                 radius=R, particle_density=6.0, hertz_K=hertz[0], hertz_d0=hertz[1],
                 hertz_rcap=hertz[2], zeta=zeta, **kw)
    o = O.Oracle(p, rho)
    o.add_particles(x, v, w)
    br = Brute(shape, 2, (1.0, 0.9), 0.65, 1.0, (2e-4, 0, 0), rho,
               walls=kw["walls"], u_lo=kw.get("wall_u_lo", (0, 0, 0)),
               u_hi=kw.get("wall_u_hi", (0, 0, 0)), radius=R, pdens=6.0, hertz=hertz, zeta=zeta)
    br.add_particles(x, v, w)
    _compare(o, br)
    events = 0
    for _ in range(3):
        before = o.owner().copy()
        assert o.step(1) == 0
        rep = br.step()
        _compare(o, br, rep)
        events += int((before != o.owner()).sum())
    # the motion must actually have destroyed and created fluid nodes
    assert events > 0
