"""Pin of the oracle's forward-mode (dual number) derivative of the loss
L = sum_fluid |grad_lat(psi_A - psi_B)|^2 against central finite differences
of the oracle's own FP64 runs, for the coupling G, the body force g_x and the
initial density field of component A, with static spheres present; and of the
tangent of the whole final pseudo-potential field, which must reproduce the
loss tangent by the chain rule and match central differences node by node."""
import numpy as np
import pytest

import oracle as O
import synth


def _setup():
    w = synth.Workload("tan", 10, 9, 8, nparticles=2, radius=2.0, particles_fixed=True, seed=31)
    p = O.Params(10, 9, 8, ncomp=2, G=0.65, sc_norm=1.0, g=(1e-6, 0, 0), radius=2.0,
                 particles_fixed=True)
    x = np.array([[2.3, 2.6, 2.2], [7.1, 6.4, 5.3]])
    return p, w.densities(), x


def _loss(p, rho0, x, nsteps):
    o = O.Oracle(p, rho0)
    o.add_particles(x)
    o.step(nsteps)
    return o.loss()


@pytest.mark.parametrize("nsteps", [1, 12])
def test_tangent_matches_central_differences(nsteps):
    p, rho0, x = _setup()
    L, dLdG = O.loss_tangent(p, rho0, nsteps, dG=1.0, x=x)
    assert abs(L - _loss(p, rho0, x, nsteps)) <= 1e-14 * abs(L)
    h = 1e-4 * p.G
    pp = O.Params(**{**p.__dict__, "G": p.G + h})
    pm = O.Params(**{**p.__dict__, "G": p.G - h})
    fd = (_loss(pp, rho0, x, nsteps) - _loss(pm, rho0, x, nsteps)) / (2 * h)
    assert abs(dLdG - fd) <= 1e-6 * abs(fd)

    _, dLdg = O.loss_tangent(p, rho0, nsteps, dg=(1.0, 0, 0), x=x)
    h = 1e-5   # g_x is tiny; a relative step would drown in the cancellation of L
    pp = O.Params(**{**p.__dict__, "g": (p.g[0] + h, 0, 0)})
    pm = O.Params(**{**p.__dict__, "g": (p.g[0] - h, 0, 0)})
    fd = (_loss(pp, rho0, x, nsteps) - _loss(pm, rho0, x, nsteps)) / (2 * h)
    assert abs(dLdg - fd) <= 1e-6 * abs(fd)

    rng = np.random.default_rng(4)
    v = rng.standard_normal(p.N)
    _, dLdv = O.loss_tangent(p, rho0, nsteps, drhoA=v, x=x)
    h = 1e-4
    r_p, r_m = rho0.copy(), rho0.copy()
    r_p[0] += h * v
    r_m[0] -= h * v
    fd = (_loss(p, r_p, x, nsteps) - _loss(p, r_m, x, nsteps)) / (2 * h)
    assert abs(dLdv - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("nsteps", [1, 5])
def test_psi_tangent_matches_differences_and_the_loss_tangent(nsteps):
    p, rho0, x = _setup()
    rng = np.random.default_rng(6)
    v = rng.standard_normal(p.N)
    dg = (0.3, -0.2, 0.1)
    psi, dpsi = O.psi_tangent(p, rho0, nsteps, dG=0.5, dg=dg, drhoA=v, x=x)
    o = O.Oracle(p, rho0)
    o.add_particles(x)
    o.step(nsteps)
    assert np.abs(psi - o.psi()).max() <= 1e-15 * np.abs(psi).max()
    # central differences of psi along the same direction (G, g, rho_A0)
    h = 1e-5

    def psi_at(sgn):
        q = O.Params(**{**p.__dict__, "G": p.G + sgn * h * 0.5,
                        "g": tuple(p.g[a] + sgn * h * dg[a] for a in range(3))})
        r = rho0.copy()
        r[0] += sgn * h * v
        oo = O.Oracle(q, r)
        oo.add_particles(x)
        oo.step(nsteps)
        return oo.psi()
    fd = (psi_at(1) - psi_at(-1)) / (2 * h)
    assert np.abs(dpsi - fd).max() <= 1e-7 * np.abs(fd).max()
    # chain rule: dL = sum over fluid n of 2 grad phi(n) . grad dphi(n)
    c, w = O.lattice()
    own = o.owner()
    nb = _neighbours(p, c)
    phi, dphi = psi[0] - psi[1], dpsi[0] - dpsi[1]
    fluid = np.flatnonzero(own == 0)
    gphi = 3.0 * (phi[nb[fluid]] * w[None, :])[:, :, None] * c[None, :, :]
    gdphi = 3.0 * (dphi[nb[fluid]] * w[None, :])[:, :, None] * c[None, :, :]
    dL_chain = 2.0 * (gphi.sum(1) * gdphi.sum(1)).sum()
    _, dL = O.loss_tangent(p, rho0, nsteps, dG=0.5, dg=dg, drhoA=v, x=x)
    assert abs(dL_chain - dL) <= 1e-12 * abs(dL)


def _neighbours(p, c):
    """[N][19] index of n + c_i (periodic)."""
    n = np.arange(p.N)
    xx, yy, zz = n % p.nx, (n // p.nx) % p.ny, n // (p.nx * p.ny)
    return ((xx[:, None] + c[None, :, 0]) % p.nx
            + p.nx * (((yy[:, None] + c[None, :, 1]) % p.ny)
                      + p.ny * ((zz[:, None] + c[None, :, 2]) % p.nz)))
