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
