"""Pins of the oracle's open z-faces (pressure: anti-bounce-back Eq. bbp;
velocity: Eq. bbv with extrapolated density; equilibrium inflow) against what
they must reproduce: a uniform equilibrium flow or rest state that matches the
face data is an exact steady state; a density difference between two
pressure faces drives the flow from the denser face; a velocity inlet with a
pressure outlet drives the box monotonically towards the inlet velocity."""
import numpy as np
import pytest

import oracle as O

SHAPE = (6, 5, 20)
CS2 = 1.0 / 3.0


def _run(wall_type, wall_rho, u_lo, u_hi, u0, steps, ncomp=1):
    N = np.prod(SHAPE)
    p = O.Params(*SHAPE, ncomp=ncomp, tau=(0.8, 0.8), walls=True, wall_type=wall_type,
                 wall_rho=wall_rho, wall_u_lo=u_lo, wall_u_hi=u_hi)
    rho = np.ones((ncomp, N))
    u = np.tile(np.array(u0, float), (N, 1))
    o = O.Oracle(p, rho, u)
    assert o.step(steps) == 0
    fluid = o.owner() == 0
    return o, fluid


@pytest.mark.parametrize("types", [(2, 2), (3, 3), (3, 2), (2, 3)])
def test_uniform_flow_matching_the_faces_is_steady(types):
    U = (0.0, 0.0, 0.02)
    o, fluid = _run(types, ((1.0, 1.0), (1.0, 1.0)), U, U, U, 60)
    assert np.abs(o.rho()[:, fluid] - 1.0).max() < 1e-14
    u = o.u()[fluid]
    assert np.abs(u - np.array(U)).max() < 1e-14


def test_rest_between_pressure_faces_at_the_same_density_is_steady():
    o, fluid = _run((1, 1), ((1.0, 1.0), (1.0, 1.0)), (0, 0, 0), (0, 0, 0), (0, 0, 0), 60)
    assert np.abs(o.rho()[:, fluid] - 1.0).max() < 1e-14
    assert np.abs(o.u()[fluid]).max() < 1e-15


def test_pressure_difference_drives_flow_towards_the_lower_density():
    o, fluid = _run((1, 1), ((1.02, 1.0), (0.98, 1.0)), (0, 0, 0), (0, 0, 0), (0, 0, 0), 400)
    uz = o.u()[fluid][:, 2]
    assert uz.mean() > 1e-4 and uz.min() > 0
    rz = o.rho()[0].reshape(SHAPE[::-1])[1:-1].mean(axis=(1, 2))
    assert np.all(np.diff(rz) < 0)          # density falls from the lo face to the hi face


def test_velocity_inlet_with_pressure_outlet_approaches_the_inlet_velocity():
    U = (0.0, 0.0, 0.01)
    means = []
    for steps in (1500, 4000):
        o, fluid = _run((2, 1), ((1.0, 1.0), (1.0, 1.0)), U, (0, 0, 0), (0, 0, 0), steps)
        uz = o.u()[:, 2].reshape(SHAPE[::-1])[1:-1].mean(axis=(1, 2))
        assert np.all(uz > 0) and np.all(np.diff(uz) <= 0)    # fastest at the inlet
        means.append(uz.mean())
    assert abs(means[1] - 0.01) < abs(means[0] - 0.01) and abs(means[1] - 0.01) < 1e-3


@pytest.mark.parametrize("types,ncomp", [((1, 1), 1), ((2, 1), 1), ((1, 3), 1), ((1, 2), 2)])
def test_pressure_face_keeps_a_uniform_moving_flow_exact(types, ncomp):
    """Anti-bounce-back (Eq. bbp) of the equilibrium of a uniform flow u with
    the face density rho_w = rho returns exactly f_eq(rho, u) along -c_i:
    -w rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2) + 2 w rho (1 + 4.5 (c.u)^2 - 1.5 u^2)
    = w rho (1 - 3 c.u + 4.5 (c.u)^2 - 1.5 u^2). The extrapolated velocity of
    a uniform flow is u itself, so every face type keeps the flow uniform."""
    U = (0.004, -0.002, 0.02)
    o, fluid = _run(types, ((1.0, 1.0), (1.0, 1.0)), U, U, U, 60, ncomp=ncomp)
    assert np.abs(o.rho()[:, fluid] - 1.0).max() < 1e-14
    assert np.abs(o.u()[fluid] - np.array(U)).max() < 1e-14


def _one_step(shape, wall_type, rho_z, ux_z, u_face):
    """One step from the equilibrium of a state with density rho(z) and
    velocity (ux(z), 0, 0), one component, no forces: the collision keeps the
    equilibrium, so the populations that enter the first fluid layer from a
    face are the face's reflection of f_eq(rho(r_b), u(r_b))."""
    nx, ny, nz = shape
    z = np.repeat(np.arange(nz), nx * ny)
    rho = rho_z(z.astype(float))[None, :]
    u = np.zeros((z.size, 3))
    u[:, 0] = ux_z(z.astype(float))
    p = O.Params(*shape, ncomp=1, tau=(0.8, 0.8), walls=True, wall_type=wall_type,
                 wall_rho=((1.0, 1.0), (1.0, 1.0)), wall_u_lo=u_face, wall_u_hi=u_face)
    o = O.Oracle(p, rho, u)
    assert o.step(1) == 0
    return o.f()[0]


def _entering(f, c, shape, face, cxy):
    """f_j at the middle node of the first fluid layer next to `face`, for the
    direction j = (cx, cy, +-1) that points away from the face."""
    nx, ny, nz = shape
    cz = 1 if face == 0 else -1
    j = int(np.where((c == (cxy[0], cxy[1], cz)).all(1))[0][0])
    zb = 1 if face == 0 else nz - 2
    n = nx // 2 + nx * (ny // 2 + ny * zb)
    return f[j, n], j


@pytest.mark.parametrize("face", [0, 1])
def test_velocity_face_density_is_extrapolated_to_the_halfway_wall(face):
    """Eq. bbv returns f*_i - 2 w_i rho_w (U.c_i)/c_s^2 along -c_i, so rho_w can
    be read back from the entering populations. Its extrapolation
    X(r_b) + (X(r_b) - X(r_b'))/2 is exact for a linear profile and equals the
    profile at the wall, halfway between the face layer and r_b."""
    shape = (6, 5, 12)
    beta = 2e-3
    rho_z = lambda z: 1.0 + beta * z            # noqa: E731
    U = (0.01, 0.0, 0.0)
    f = _one_step(shape, (2, 2), rho_z, lambda z: 0 * z, U)
    c, w = O.lattice()
    zb = 1 if face == 0 else shape[2] - 2
    zwall = 0.5 if face == 0 else shape[2] - 1.5
    for cx in (1, -1):
        fin, j = _entering(f, c, shape, face, (cx, 0))
        i = int(np.where((c == -c[j]).all(1))[0][0])     # the link direction, into the face
        fstar = w[i] * rho_z(float(zb))                   # f_eq of the rest state at r_b
        uc = float(np.dot(U, c[i]))
        rho_w = (fstar - fin) / (2 * w[i] * uc / CS2)
        assert abs(rho_w - rho_z(zwall)) < 1e-12


@pytest.mark.parametrize("face", [0, 1])
def test_pressure_face_velocity_is_extrapolated_to_the_halfway_wall(face):
    """Eq. bbp returns -f*_i + 2 w_i rho_w B_i along -c_i, with
    B_i = 1 + (u_w.c_i)^2/(2 c_s^4) - u_w^2/(2 c_s^2). For u_w along x the
    directions (1, 0, -+1) and (0, 0, -+1) differ by (u_w,x)^2/(2 c_s^4), which
    gives |u_w|; for a linear shear profile it must be the profile at the
    halfway wall."""
    shape = (6, 5, 12)
    a, b = 0.02, 0.002
    ux_z = lambda z: a + b * z                  # noqa: E731
    f = _one_step(shape, (1, 1), lambda z: 1.0 + 0 * z, ux_z, (0.0, 0.0, 0.0))
    c, w = O.lattice()
    zb = 1 if face == 0 else shape[2] - 2
    zwall = 0.5 if face == 0 else shape[2] - 1.5
    ub = np.array([ux_z(float(zb)), 0.0, 0.0])

    def bracket(cxy):
        fin, j = _entering(f, c, shape, face, cxy)
        i = int(np.where((c == -c[j]).all(1))[0][0])
        cu, uu = float(c[i] @ ub), float(ub @ ub)
        fstar = w[i] * (1 + cu / CS2 + 0.5 * (cu * cu / CS2 - uu) / CS2)
        return (fin + fstar) / (2 * w[i] * 1.0)
    uw2 = (bracket((1, 0)) - bracket((0, 0))) * 2 * CS2 * CS2
    assert abs(np.sqrt(uw2) - ux_z(zwall)) < 1e-10
    # the isotropic part: B = 1 - u_w^2 / (2 c_s^2) for a direction normal to u_w
    assert abs(bracket((0, 1)) - (1 - ux_z(zwall) ** 2 / (2 * CS2))) < 1e-13
