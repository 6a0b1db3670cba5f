"""Observables of the HIP path (lb_observables) against the oracle's, field by
field, on a box between moving walls with moving spheres, a body force and
the Shan-Chen coupling: masses, bare and physical momentum (Sec. 2.3 after
Eq. lbsbgk), density extrema, max |u|, the fluid node count, sphere momentum
and kinetic energies, and the link-force magnitude sum.

Tolerances: FP64 1e-12 relative; masses, momenta and energies relative to
their own size or, for a momentum that may cancel, to M max|u| (an upper
bound of |P|); extrema relative to the density, max|u| relative to itself.
FP32 (deviation storage): the observables of a common state agree to 1e-12,
since both sides reduce the same FP32-representable populations in FP64;
the physical momentum to 1e-8, since its force term reads the
pseudo-potential stored in FP32 (2^-24 relative per value, on a Shan-Chen
force sum below 1e-3 of M max|u| here); after one step everything to 1e-5.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import make_pair, requires_gpu, sync_state

pytestmark = [pytest.mark.gpu, requires_gpu]

SHAPE = (24, 20, 18)


def _setup(precision):
    w = synth.Workload("obs", *SHAPE, nparticles=4, radius=3.0, seed=synth.BASE_SEED + 41,
                       walls=True)
    rng = np.random.default_rng(41)
    v = 0.05 * (2 * rng.random((4, 3)) - 1)
    om = 0.02 * (2 * rng.random((4, 3)) - 1)
    kw = dict(ncomp=2, G=0.65, g=(2e-5, -1e-5, 5e-6), walls=True, wall_u_lo=(-0.01, 0, 0),
              wall_u_hi=(0.01, 0.004, 0), radius=3.0, particle_density=1.5,
              zeta=(0.04, -0.04))
    return make_pair(SHAPE, w.densities(), x=w.centres(), v=v, w=om, precision=precision, **kw)


def _errors(ob_o, ob_g):
    """Relative errors of every lb_obs field against the oracle's vector."""
    M = ob_o[0] + ob_o[1]
    pscale = M * max(ob_o[9], 1e-30)
    e = {}
    e["fluid_nodes"] = float(ob_g.fluid_nodes != int(ob_o[10]))
    e["mass"] = float(np.abs(ob_g.mass - ob_o[0:2]).max() / M)
    e["momentum"] = float(np.abs(ob_g.momentum - ob_o[2:5]).max() / pscale)
    e["phys_momentum"] = float(np.abs(ob_g.phys_momentum - ob_o[32:35]).max() / pscale)
    e["rho_min"] = float(np.abs(ob_g.rho_min - ob_o[5:7]).max() / np.abs(ob_o[5:7]).max())
    e["rho_max"] = float(np.abs(ob_g.rho_max - ob_o[7:9]).max() / np.abs(ob_o[7:9]).max())
    e["u_max"] = float(abs(ob_g.u_max - ob_o[9]) / ob_o[9])
    pm = np.abs(ob_o[11:14]).max() + 1e-300
    e["particle_momentum"] = float(np.abs(ob_g.particle_momentum - ob_o[11:14]).max() / pm)
    e["particle_ke"] = float(abs(ob_g.particle_ke - ob_o[14]) / ob_o[14])
    e["particle_ke_rot"] = float(abs(ob_g.particle_ke_rot - ob_o[15]) / ob_o[15])
    if ob_o[35] > 0:
        e["flink_abs"] = float(abs(ob_g.flink_abs - ob_o[35]) / ob_o[35])
    return e


def _gate(e, tol, what):
    print(what, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v <= tol, (what, k, v)


def test_observables_fp64_moving_spheres_and_walls():
    o, lat = _setup("fp64")
    done = 0
    for h in (1, 10, 30):
        o.step(h - done)
        lat.step(h - done)
        done = h
        ob_o = o.observables()
        ob_g = lat.observables()
        assert ob_g.nparticles == 4 and ob_g.step == h and ob_g.flags == 0
        # the physical momentum differs from the bare one by a resolved amount
        assert np.abs(ob_o[32:35] - ob_o[2:5]).max() > 1e-3 * np.abs(ob_o[2:5]).max()
        _gate(_errors(ob_o, ob_g), 1e-12, f"fp64 t={h}")


def test_observables_fp32_common_state_and_one_step():
    o, lat = _setup("fp32")
    lat.step(20)
    sync_state(o, lat)
    ob_o = o.observables()
    e = _errors(ob_o, lat.observables())
    e.pop("flink_abs", None)          # the oracle has not stepped from this state yet
    _gate({"phys_momentum": e.pop("phys_momentum")}, 1e-8, "fp32 common state")
    _gate(e, 1e-12, "fp32 common state")
    o.step(1)
    lat.step(1)
    _gate(_errors(o.observables(), lat.observables()), 1e-5, "fp32 one step")
