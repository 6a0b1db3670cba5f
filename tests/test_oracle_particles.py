"""Pins of the oracle's particle coupling and integrator (Sec. 2.4-2.5).

* Hertz contact (Eq. hertzpot, repulsive reading): closed-form magnitude,
  exact antisymmetry, mirror repulsion from walls.
* Rotational mid-step leap-frog (Eq. lf, quatder, svanimpl): for constant
  angular velocity the scheme is an exact rotation by a closed-form angle per
  step; it is compared over 1000 steps.
* Momentum and mass ledgers: every change of the fluid's momentum and mass in
  a step is accounted for by the particle force terms (Eq. LADDFORCE, distr,
  creat, shanchen2), the body force and the wall links, exactly.
* Ladd bounce-back kinematics (Eq. LADDFLBE, UPI): drag along the flow on a
  sphere at rest, braking torque on a spinning sphere, plain bounce-back at rest.
"""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import synth


def _qmul(a, b):
    a0, av = a[0], np.asarray(a[1:])
    b0, bv = b[0], np.asarray(b[1:])
    return np.concatenate([[a0 * b0 - av @ bv], a0 * bv + b0 * av + np.cross(av, bv)])


def test_quaternion_update_is_exact_discrete_rotation():
    """At constant w the implicit mid-step update maps q to
    (cos t, sin t w_hat) (x) q with t = 2 atan(s |w| / 4), where s = |q_h|^2
    solves s (1 + s^2 |w|^2 / 16) = 1 (derived from q' = 1/2 Q(q) R(q)^T w
    with the unnormalised rotation matrix of the paper)."""
    lib = O.lib()
    lib.lbo_test_rotate.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32]
    rng = np.random.default_rng(5)
    for wmag in (0.003, 0.05, 0.3):
        q0 = rng.standard_normal(4)
        q0 /= np.linalg.norm(q0)
        w = rng.standard_normal(3)
        w *= wmag / np.linalg.norm(w)
        q = q0.copy()
        n = 1000
        lib.lbo_test_rotate(q.ctypes.data_as(C.POINTER(C.c_double)),
                            w.ctypes.data_as(C.POINTER(C.c_double)), n)
        s = 1.0
        for _ in range(100):
            s = s - (s * (1 + s * s * wmag ** 2 / 16) - 1) / (1 + 3 * s * s * wmag ** 2 / 16)
        theta = 2 * np.arctan(s * wmag / 4)
        rot = np.concatenate([[np.cos(n * theta)], np.sin(n * theta) * w / wmag])
        ref = _qmul(rot, q0)
        assert np.abs(q - ref).max() < 1e-12
        # and it approximates the exact rotation by |w| per step to O(|w|^3)
        assert abs(2 * theta - wmag) < wmag ** 3 / 4 + 1e-15


def _run_one_step(p, x, v=None, w=None):
    o = O.Oracle(p, np.ones((p.ncomp, p.N)))
    o.add_particles(x, v, w)
    assert o.step(1) == 0
    return o.particles()


def test_hertz_pair_closed_form_and_antisymmetry():
    R, K = 3.0, 20.0
    d0, rcap = 2 * R + 1, 2 * R
    for r in (6.6, 6.2, 5.7):         # between cap and onset, at/below the cap
        p = O.Params(24, 16, 16, ncomp=1, radius=R, hertz_K=K, particle_density=50.0)
        e = np.array([0.6, 0.8, 0.0])
        x = np.array([[8.0, 8.0, 8.0], [8.0, 8.0, 8.0] + r * e])
        rec = _run_one_step(p, x)
        FH = rec[:, O.REC["FH"]:O.REC["FH"] + 3]
        mag = 2.5 * K * (d0 - max(r, rcap)) ** 1.5
        assert np.abs(FH[0] + mag * e).max() < 1e-12 * mag
        assert np.array_equal(FH[0], -FH[1])
    # beyond the onset: no force
    p = O.Params(24, 16, 16, ncomp=1, radius=R, hertz_K=K, particle_density=50.0)
    rec = _run_one_step(p, np.array([[6.0, 8.0, 8.0], [6.0 + d0 + 0.01, 8.0, 8.0]]))
    assert np.all(rec[:, O.REC["FH"]:O.REC["FH"] + 3] == 0)


def test_hertz_wall_mirror():
    R, K, nz = 3.0, 20.0, 20
    p = O.Params(16, 16, nz, ncomp=1, radius=R, hertz_K=K, walls=True, particle_density=50.0)
    zlo = 0.5 + 3.2          # distance to the lower wall plane
    rec = _run_one_step(p, np.array([[8.0, 8.0, zlo], [8.0, 8.0, nz - 1.5 - 3.4]]))
    d0, rcap = 2 * R + 1, 2 * R
    m0 = 2.5 * K * (d0 - max(2 * 3.2, rcap)) ** 1.5
    m1 = 2.5 * K * (d0 - max(2 * 3.4, rcap)) ** 1.5
    FH = rec[:, O.REC["FH"]:O.REC["FH"] + 3]
    assert np.allclose(FH[0], [0, 0, m0], rtol=1e-13, atol=0)
    assert np.allclose(FH[1], [0, 0, -m1], rtol=1e-13, atol=0)


@pytest.mark.parametrize("walls", [False, True])
def test_momentum_and_mass_ledgers_with_moving_spheres(walls):
    """P(t+1) - P(t) = -sum_p (F_d + F_c + F_liq) + sum_fluid F_SC + sum rho g
    - sum_wall-links F_link, and M_k(t+1) - M_k(t) = -destroyed + created
    + moving-link corrections, to rounding."""
    L = (20, 18, 22)
    w = synth.Workload("led", *L, nparticles=5, radius=3.0, seed=77, walls=walls)
    p = O.Params(*L, ncomp=2, G=0.65, sc_norm=1.0, g=(1e-4, -5e-5, 0.0), radius=3.0,
                 particle_density=1.5, walls=walls,
                 wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0.005, 0))
    o = O.Oracle(p, w.densities())
    rng = np.random.default_rng(3)
    x = w.centres()
    o.add_particles(x, 0.08 * (2 * rng.random((5, 3)) - 1), 0.02 * (2 * rng.random((5, 3)) - 1))
    events = 0
    for t in range(12):
        ob0 = o.observables()
        own0 = o.owner()
        assert o.step(1) == 0
        ob1 = o.observables()
        rec = o.particles()
        events += int((own0 != o.owner()).sum())
        Fd = rec[:, O.REC["Fd"]:O.REC["Fd"] + 3].sum(0)
        Fc = rec[:, O.REC["Fc"]:O.REC["Fc"] + 3].sum(0)
        Fl = rec[:, O.REC["Fliq"]:O.REC["Fliq"] + 3].sum(0)
        scale = rec[:, O.REC["flabs"]].sum()
        pred = -(Fd + Fc + Fl) + ob1[25:28] + ob1[22:25] - ob1[28:31]
        assert np.abs((ob1[2:5] - ob0[2:5]) - pred).max() < 1e-13 * scale
        for k in range(2):
            dm = ob1[k] - ob0[k]
            predm = -ob1[16 + k] + ob1[18 + k] + ob1[20 + k]
            assert abs(dm - predm) < 1e-13 * ob0[k]
        if not walls:
            # Newton's third law between fluid and frontier solids (Eq. shanchen2)
            FSC = rec[:, O.REC["FSC"]:O.REC["FSC"] + 3].sum(0)
            assert np.abs(ob1[25:28] + FSC).max() < 1e-13 * scale
    assert events > 0


@pytest.mark.parametrize("walls", [False, True])
def test_physical_momentum_matches_the_force_of_the_next_step(walls):
    """Physical momentum = bare momentum + half the force density summed over
    the fluid (Sec. 2.3 after Eq. lbsbgk). With fixed spheres the map does not
    change, so the force of the current state is the force the next step
    applies, which the momentum ledger above accounts for exactly: Shan-Chen
    over the fluid nodes (with the virtual densities of the frontier) plus
    rho g."""
    L = (18, 16, 20)
    w = synth.Workload("phys", *L, nparticles=4, radius=3.0, seed=91, walls=walls)
    p = O.Params(*L, ncomp=2, G=0.65, sc_norm=1.0, g=(1e-4, -5e-5, 2e-5), radius=3.0,
                 particles_fixed=True, walls=walls, zeta=(0.05, -0.05))
    o = O.Oracle(p, w.densities())
    o.add_particles(w.centres())
    assert o.step(3) == 0
    for _ in range(3):
        ob0 = o.observables()
        assert o.step(1) == 0
        ob1 = o.observables()
        force = ob1[25:28] + ob1[22:25]
        assert np.abs(force).max() > 1e-6              # the frontier makes it non-zero
        half = ob0[32:35] - ob0[2:5]
        assert np.abs(half - 0.5 * force).max() < 1e-14 * (ob0[0] + ob0[1])
    # the link-force magnitude summed over the spheres
    assert abs(ob1[35] - o.particles()[:, O.REC["flabs"]].sum()) < 1e-12 * ob1[35]


def test_ladd_drag_and_braking_torque_signs():
    # a sphere held at rest in a uniform stream is dragged along the stream
    L = 20
    p = O.Params(L, L, L, ncomp=1, radius=4.0, particles_fixed=True)
    u0 = np.zeros((p.N, 3))
    u0[:, 0] = 0.01
    o = O.Oracle(p, np.ones((1, p.N)), u0)
    o.add_particles(np.array([[10.2, 9.7, 10.1]]))
    for _ in range(5):
        o.step(1)
        rec = o.particles()
        assert rec[0, O.REC["Fliq"]] > 0
        # at rest the reflection is plain bounce-back: no moving-link mass change
        assert o.observables()[20] == 0.0
    # a sphere spinning in fluid at rest feels a torque against its spin
    p = O.Params(L, L, L, ncomp=1, radius=4.0, particle_density=5.0)
    o = O.Oracle(p, np.ones((1, p.N)))
    wv = np.array([[0.0, 0.0, 0.01]])
    o.add_particles(np.array([[10.0, 10.0, 10.0]]), None, wv)
    o.step(1)
    T = o.particles()[0, O.REC["Tliq"]:O.REC["Tliq"] + 3]
    assert T @ wv[0] < 0
    # and a translating sphere is braked
    o = O.Oracle(p, np.ones((1, p.N)))
    vv = np.array([[0.02, -0.01, 0.0]])
    o.add_particles(np.array([[10.0, 10.0, 10.0]]), vv)
    o.step(1)
    F = o.particles()[0, O.REC["Fliq"]:O.REC["Fliq"] + 3]
    assert F @ vv[0] < 0


def test_resting_solids_in_resting_fluid_feel_no_force_or_torque():
    """For any finite set of solid nodes, the D3Q19 links from fluid into it
    satisfy sum w_i c_i = 0 and sum r x w_i c_i = 0: every pair of solid
    neighbours would contribute a link twice with opposite c_i, and the full
    stencil has sum_i w_i c_i = 0. In a uniform fluid at rest every link
    carries 2 w_i rho c_i (plain bounce-back of the equilibrium). So a fixed
    sphere on its own, also across the periodic seams, feels no force and no
    torque; two overlapping spheres share their nodes (the lower index takes
    them), each has only part of the union's links and feels a force, and
    the two forces and torques about a common point cancel."""
    L = (26, 22, 24)
    p = O.Params(*L, ncomp=2, G=0.0, radius=3.7, particles_fixed=True)
    x = np.array([[5.3, 4.1, 6.9], [9.8, 6.2, 8.0],      # overlapping pair
                  [25.4, 11.3, 12.6],                     # across the x seam
                  [14.1, 17.6, 1.2],                      # across the z seam
                  [18.9, 3.3, 17.7]])
    o = O.Oracle(p, np.ones((2, p.N)))
    o.add_particles(x)
    assert (o.owner() > 0).sum() > 700
    o.step(1)
    rec = o.particles()
    F = rec[:, O.REC["Fliq"]:O.REC["Fliq"] + 3]
    T = rec[:, O.REC["Tliq"]:O.REC["Tliq"] + 3]
    scale = rec[:, O.REC["flabs"]].max()
    assert scale > 1.0
    tol_f, tol_t = 1e-14 * scale, 1e-13 * scale
    assert np.abs(F[2:]).max() <= tol_f and np.abs(T[2:]).max() <= tol_t
    # the overlapping pair: opposite forces, and torques that cancel about one point
    assert np.abs(F[0]).max() > 1.0
    assert np.abs(F[0] + F[1]).max() <= tol_f
    Tc = T[0] + T[1] + np.cross(x[1] - x[0], F[1])     # both torques about x[0]
    assert np.abs(Tc).max() <= tol_t
