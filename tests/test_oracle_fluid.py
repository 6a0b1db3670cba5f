"""Pins of the oracle's fluid step against facts the method and mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an invariant, a special case that reduces to a simpler model, or an
independent linear analysis written here from the scheme's definition
(Sec. 2.1-2.3: Eq. bgk, bgk2, viscosity, LEQ, bb, bbv, shanchen, twobgk,
scvel, edm, lbsbgk).
"""
import numpy as np
import pytest

import oracle as O
import synth

CS2 = 1.0 / 3.0


def test_streaming_is_an_exact_permutation():
    """With collision switched off (omega -> 0) and no force, one step moves
    f_i(n) to f_i(n + c_i) (Eq. bgk2): an index or direction mix-up fails."""
    p = O.Params(5, 4, 3, ncomp=1, tau=(1e15,))
    o = O.Oracle(p, np.ones((1, p.N)))
    rng = np.random.default_rng(1)
    f0 = rng.uniform(0.1, 1.0, size=(1, 19, p.N))
    o.set_f(f0)
    o.step(1)
    f1 = o.f()
    c, _ = O.lattice()
    n = np.arange(p.N)
    x, y, z = n % 5, (n // 5) % 4, n // 20
    for i in range(19):
        dst = (x + c[i, 0]) % 5 + 5 * ((y + c[i, 1]) % 4 + 4 * ((z + c[i, 2]) % 3))
        assert np.abs(f1[0, i, dst] - f0[0, i, n]).max() < 1e-13


def test_c1_conservation_and_shear_wave_viscosity():
    """Config C1: mass and momentum are invariants of BGK collision+streaming,
    and a shear wave decays as exp(-nu k^2 t) with nu = c_s^2 (tau - 1/2)
    (Eq. viscosity). The wave varies only along z, so a 1x1x32 column is the
    same flow as the 32^3 box."""
    tau, L = 0.8, 32
    p = O.Params(1, 1, L, ncomp=1, tau=(tau,))
    u0 = synth.shear_wave_velocity(1, 1, L)
    o = O.Oracle(p, np.ones((1, L)), u0)
    s = np.sin(2 * np.pi * np.arange(L) / L)
    m0 = o.observables()
    amps = []
    for t in range(201):
        amps.append(o.u()[:, 0] @ s / (L / 2))
        if t < 200:
            o.step(1)
    m1 = o.observables()
    assert abs(m1[0] - m0[0]) / m0[0] < 1e-13
    assert np.abs(m1[2:5] - m0[2:5]).max() < 1e-14
    k = 2 * np.pi / L
    nu_fit = -np.polyfit(np.arange(201), np.log(amps), 1)[0] / k ** 2
    nu = CS2 * (tau - 0.5)
    assert abs(nu_fit - nu) / nu < 0.01


def test_c1_full_box_mass_and_momentum():
    w = synth.workload("C1")
    p = O.Params(w.nx, w.ny, w.nz, ncomp=1, tau=w.tau)
    o = O.Oracle(p, np.ones((1, w.N)), synth.shear_wave_velocity(w.nx, w.ny, w.nz))
    m0 = o.observables()
    o.step(20)
    m1 = o.observables()
    assert abs(m1[0] - m0[0]) / m0[0] < 1e-13
    assert np.abs(m1[2:5] - m0[2:5]).max() / m0[0] < 1e-15


def test_couette_is_exact_between_moving_walls():
    """Halfway bounce-back with the moving-wall correction (Eq. bbv): the
    linear Couette profile between the wall planes z = 1/2 and z = nz - 3/2
    is an exact steady state."""
    nz, U = 12, 0.01
    p = O.Params(1, 1, nz, ncomp=1, tau=(1.0,), walls=True,
                 wall_u_lo=(-U, 0, 0), wall_u_hi=(U, 0, 0))
    o = O.Oracle(p, np.ones((1, nz)))
    o.step(3000)
    ux = o.u()[:, 0]
    z = np.arange(1, nz - 1)
    exact = -U + 2 * U * (z - 0.5) / (nz - 2)
    assert np.abs(ux[1:-1] - exact).max() < 1e-10


def test_poiseuille_profile():
    """Body-force driven flow between resting halfway walls: parabolic
    profile u = g/(2 nu) (z - z0)(z1 - z); physical velocity = bare + g/2
    (momentum at half step, Sec. 2.3)."""
    H, g = 32, 1e-6
    nz = H + 2
    p = O.Params(1, 1, nz, ncomp=1, tau=(1.0,), walls=True, g=(g, 0, 0))
    o = O.Oracle(p, np.ones((1, nz)))
    o.step(30000)
    ux = o.u()[1:-1, 0] + 0.5 * g
    z = np.arange(1, nz - 1)
    nu = CS2 * 0.5
    exact = g / (2 * nu) * (z - 0.5) * (nz - 1.5 - z)
    assert np.sqrt(np.mean((ux - exact) ** 2) / np.mean(exact ** 2)) < 0.01


def test_two_components_without_coupling_reduce_to_one():
    """G = 0, equal tau: f_eq is linear in rho at fixed u and the mixture
    velocity is the total velocity, so f_A + f_B follows one-component BGK."""
    w = synth.Workload("g0", 6, 5, 7, G=0.0, seed=11)
    rho = w.densities()
    p2 = O.Params(6, 5, 7, ncomp=2, tau=(0.9, 0.9), G=0.0, g=(1e-5, 0, 0))
    p1 = O.Params(6, 5, 7, ncomp=1, tau=(0.9,), g=(1e-5, 0, 0))
    o2 = O.Oracle(p2, rho)
    o1 = O.Oracle(p1, rho.sum(0, keepdims=True))
    o2.step(15)
    o1.step(15)
    f2 = o2.f().sum(0)
    f1 = o1.f()[0]
    assert np.abs(f2 - f1).max() < 1e-14


def test_shan_chen_conserves_global_momentum():
    """The pairwise antisymmetric stencil makes sum_n sum_k F_k = 0, so total
    momentum is invariant in a periodic box."""
    w = synth.Workload("sc", 10, 9, 8, seed=12)
    p = O.Params(10, 9, 8, ncomp=2, G=0.65, sc_norm=1.0)
    o = O.Oracle(p, w.densities())
    M = o.observables()[0] * 2
    for _ in range(10):
        o.step(5)
        ob = o.observables()
        assert np.abs(ob[2:5]).max() / M < 1e-15
        assert np.abs(ob[25:28]).max() / M < 1e-15


def test_physical_momentum_under_a_body_force_closed_form():
    """With a uniform acceleration g in a periodic box every step adds M g to
    the bare momentum (the Shan-Chen forces sum to zero), so from rest
    P_bare(t) = t M g, and the physical momentum (bare plus half the force
    density, Sec. 2.3 after Eq. lbsbgk) is P_phys(t) = (t + 1/2) M g."""
    w = synth.Workload("pm", 10, 9, 8, seed=21)
    g = np.array([2e-5, -1e-5, 3e-6])
    p = O.Params(10, 9, 8, ncomp=2, G=0.65, sc_norm=1.0, g=tuple(g))
    o = O.Oracle(p, w.densities())
    ob = o.observables()
    M = ob[0] + ob[1]
    for t in range(0, 31, 10):
        if t:
            o.step(10)
            ob = o.observables()
        assert np.abs(ob[2:5] - t * M * g).max() < 1e-14 * M * np.abs(g).max() * (t + 1)
        assert np.abs(ob[32:35] - (t + 0.5) * M * g).max() < 1e-14 * M * np.abs(g).max() * (t + 1)


def _growth_matrix(k, omega, Gs, rho0=1.0):
    """Linearised composition dynamics of one Fourier mode exp(i k z) about a
    uniform 50/50 mixture at rest, written from the scheme's definition:
    g_i = f^A_i - f^B_i, phi = sum_i g_i, the common velocity cancels, and
    g*_i = w_i phi + 3 rho0 w_i c_i.(a_A - a_B) + (1 - omega)(g_i - w_i phi)
    with a_A - a_B = G s sum_j w_j phi(z + c_j) c_j, then g_i(z+c_i) = g*_i(z)."""
    c, w = O.lattice()
    cz = c[:, 2].astype(float)
    stencil = 1j * np.sin(k) * CS2       # sum_j w_j exp(i k c_jz) c_jz
    b = omega * w + 3.0 * rho0 * w * cz * Gs * stencil
    A = (1.0 - omega) * np.eye(19) + np.outer(b, np.ones(19))
    D = np.diag(np.exp(-1j * k * cz))
    return D @ A


@pytest.mark.parametrize("Gs,m", [(0.45, 1), (0.65, 2), (0.9, 8), (0.55, 4)])
def test_shan_chen_linear_growth_exact_at_tau_one(Gs, m):
    """At tau = 1 the mode amplitude is multiplied each step by
    lambda(k) = 2/3 + cos(k)/3 + (G s rho0 / 3) sin^2 k exactly (linear regime).
    The long-wave threshold G s rho0 = 1/2 is the paper's critical coupling
    G_crit = 1/(rho_k + rho_kbar) at sc_norm = 1."""
    nz = 64
    k = 2 * np.pi * m / nz
    z = np.arange(nz)
    eps = 1e-9
    d = eps * np.cos(k * z)
    p = O.Params(1, 1, nz, ncomp=2, G=Gs, sc_norm=1.0)
    o = O.Oracle(p, np.stack([1 + d, 1 - d]))
    lam = 2 / 3 + np.cos(k) / 3 + Gs / 3 * np.sin(k) ** 2
    lam_mat = np.abs(np.linalg.eigvals(_growth_matrix(k, 1.0, Gs))).max()
    assert abs(lam - lam_mat) < 1e-12
    amp = []
    for _ in range(12):
        r = o.rho()
        amp.append((r[0] - r[1]) @ np.cos(k * z) / (nz / 2))
        o.step(1)
    ratios = np.array(amp[1:]) / np.array(amp[:-1])
    assert np.abs(ratios / lam - 1).max() < 1e-6


def test_shan_chen_growth_matches_linear_analysis_at_other_tau():
    """tau = 0.8: the asymptotic per-step growth equals the dominant
    eigenvalue of the linearised map (non-equilibrium memory included)."""
    nz, m, Gs, tau = 48, 3, 0.75, 0.8
    k = 2 * np.pi * m / nz
    z = np.arange(nz)
    d = 1e-10 * np.cos(k * z)
    p = O.Params(1, 1, nz, ncomp=2, tau=(tau, tau), G=Gs, sc_norm=1.0)
    o = O.Oracle(p, np.stack([1 + d, 1 - d]))
    ev = np.linalg.eigvals(_growth_matrix(k, 1 / tau, Gs))
    lead = ev[np.argmax(np.abs(ev))]
    assert abs(lead.imag) < 1e-12 and lead.real > 1.0
    o.step(250)
    r = o.rho()
    a0 = (r[0] - r[1]) @ np.cos(k * z)
    o.step(1)
    r = o.rho()
    a1 = (r[0] - r[1]) @ np.cos(k * z)
    assert abs(a1 / a0 / lead.real - 1) < 1e-6


@pytest.mark.slow
def test_laplace_law_for_cylinders():
    """Young-Laplace: the pressure jump across a circular interface is
    sigma/R with no offset. p = c_s^2 (rho_A + rho_B) + c_s^2 G s rho_A rho_B
    is the equation of state of the force (Eq. SCEOS); a force whose strength
    disagrees with its parameter leaves a finite intercept and a poor fit.
    The radius is the one of a disc with the area where rho_A > rho_B."""
    L, Gs = 60, 0.65
    rows = []
    for R in (8.0, 10.0, 12.0, 15.0):
        x, y = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
        r = np.hypot(x - L / 2 + 0.5, y - L / 2 + 0.5).ravel()
        a = 0.25 + 1.5 * 0.5 * (1 - np.tanh((r - R) / 1.5))
        p = O.Params(L, L, 1, ncomp=2, G=Gs, sc_norm=1.0)
        o = O.Oracle(p, np.stack([a, 2 - a]))
        o.step(3000)
        rho = o.rho()
        req = np.sqrt((rho[0] > rho[1]).sum() / np.pi)
        pr = CS2 * (rho[0] + rho[1]) + CS2 * Gs * rho[0] * rho[1]
        rows.append((req, pr[r < req - 4].mean() - pr[r > req + 5].mean()))
    req, dps = np.array(rows).T
    A = np.stack([1 / req, np.ones(len(req))], 1)
    (sigma, b), *_ = np.linalg.lstsq(A, dps, rcond=None)
    fit = A @ np.array([sigma, b])
    r2 = 1 - ((dps - fit) ** 2).sum() / ((dps - dps.mean()) ** 2).sum()
    assert sigma > 0
    assert r2 > 0.999
    assert abs(b) < 0.05 * dps[0]
