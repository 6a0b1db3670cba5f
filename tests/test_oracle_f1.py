"""Pins of the oracle's lubrication force (Eq. libric) and Janus wetting
(Eq. soliddens with an orientation-dependent zeta) against properties the
physics fixes: antisymmetry, direction along the line of centres, Galilean
invariance, no response to tangential motion, the sign that resists approach,
the cut-off and the cap; and, for wetting, which face of a sphere takes
which component as the sphere is turned."""
import numpy as np

import oracle as O

REC = O.REC


def _pair(gap, vp, vq, axis=(1.0, 0.0, 0.0), **kw):
    """Pair force of two spheres R = 4 after one step (Hertz off, fluid at rest)."""
    R = 4.0
    shape = (40, 32, 30)
    p = O.Params(*shape, ncomp=1, tau=(1.0, 1.0), radius=R, hertz_K=0.0,
                 lub_mu=kw.get("mu", 0.1), lub_hn=0.67, lub_hcap=0.5)
    o = O.Oracle(p, np.ones((1, np.prod(shape))))
    e = np.array(axis) / np.linalg.norm(axis)
    c = np.array([20.0, 16.0, 15.0])
    x = np.array([c - 0.5 * (2 * R + gap) * e, c + 0.5 * (2 * R + gap) * e])
    o.add_particles(x, np.array([vp, vq], dtype=float))
    assert o.step(1) == 0
    rec = o.particles()
    return rec[:, REC["FH"]:REC["FH"] + 3], e


def test_lubrication_resists_approach_along_the_line_of_centres():
    F, e = _pair(0.55, (0.01, 0.0, 0.0), (-0.005, 0.0, 0.0))
    assert np.allclose(F[0], -F[1], rtol=0, atol=1e-18)          # antisymmetric
    assert np.allclose(np.cross(F[0], e), 0.0, atol=1e-18)        # along e
    assert F[0] @ e < 0                                           # pushes p away from q
    Fs, _ = _pair(0.55, (-0.01, 0.0, 0.0), (0.005, 0.0, 0.0))
    assert np.allclose(Fs, -F, rtol=1e-14)                        # separation pulls back


def test_lubrication_is_galilean_and_ignores_tangential_motion():
    F, e = _pair(0.55, (0.01, 0.0, 0.0), (-0.005, 0.0, 0.0))
    Fg, _ = _pair(0.55, (0.03, 0.02, -0.01), (0.015, 0.02, -0.01))    # + common (0.02, .02, -.01)
    assert np.allclose(Fg, F, rtol=1e-12, atol=1e-18)
    Ft, _ = _pair(0.55, (0.0, 0.01, 0.0), (0.0, -0.01, 0.003))        # tangential only
    assert np.abs(Ft).max() < 1e-18
    F2, _ = _pair(0.55, (0.02, 0.0, 0.0), (-0.01, 0.0, 0.0))          # linear in v
    assert np.allclose(F2, 2 * F, rtol=1e-13)


def test_lubrication_cutoff_cap_and_magnitude():
    v = ((0.01, 0.0, 0.0), (-0.005, 0.0, 0.0))
    far, _ = _pair(0.70, *v)                    # gap above h_n = 0.67
    assert np.abs(far).max() == 0.0
    near, e = _pair(0.30, *v)                   # below the cap 0.5: as at 0.5
    cap, _ = _pair(0.50, *v)
    assert np.allclose(near, cap, rtol=1e-13)
    F, _ = _pair(0.55, *v)
    # Eq. libric with the coefficient 0.1, R = 4, h = 0.55, h_n = 0.67, v_rel.e = 0.015
    ref = -6 * np.pi * 0.1 * 16 / 4 * (1 / 0.55 - 1 / 0.67) * 0.015
    assert abs(F[0] @ e - ref) < 1e-12 * abs(ref)


def _janus_psi(q):
    shape = (24, 24, 24)
    N = np.prod(shape)
    rho = np.stack([np.full(N, 1.2), np.full(N, 0.8)])
    p = O.Params(*shape, ncomp=2, tau=(1.0, 1.0), G=0.0, radius=5.0, particles_fixed=True,
                 janus=True, janus_theta0=108.0, janus_width=10.0, janus_zeta=(0.1, 0.15))
    o = O.Oracle(p, rho)
    o.add_particles(np.array([[12.0, 12.0, 12.0]]), q=np.array([q]))
    return o.psi(), o.owner(), shape


def _node(shape, x, y, z):
    return x + shape[0] * (y + shape[1] * z)


def test_janus_faces_take_their_components():
    psi, own, shape = _janus_psi((1.0, 0.0, 0.0, 0.0))        # body x axis = +x
    a = _node(shape, 16, 12, 12)      # frontier node on the +x side (theta = 0)
    b = _node(shape, 8, 12, 12)       # on the -x side (theta = 180)
    assert own[a] > 0 and own[b] > 0
    # zeta_A = +0.1 S, zeta_B = -0.15 S; S = +1 at theta = 0, -1 at theta = 180
    assert abs(psi[0, a] - 1.1 * 1.2) < 1e-14 and abs(psi[1, a] - 0.85 * 0.8) < 1e-14
    assert abs(psi[0, b] - 0.9 * 1.2) < 1e-14 and abs(psi[1, b] - 1.15 * 0.8) < 1e-14


def test_janus_pattern_turns_with_the_sphere():
    # a quarter turn about z takes the body x axis to +y
    c, s = np.cos(np.pi / 4), np.sin(np.pi / 4)
    psi, own, shape = _janus_psi((c, 0.0, 0.0, s))
    a = _node(shape, 12, 16, 12)      # +y side: now the A face
    b = _node(shape, 12, 8, 12)
    side = _node(shape, 16, 12, 12)   # +x side: theta = 90, below theta0 - width/2
    assert abs(psi[0, a] - 1.1 * 1.2) < 1e-13 and abs(psi[0, b] - 0.9 * 1.2) < 1e-13
    assert abs(psi[0, side] - 1.1 * 1.2) < 1e-13
