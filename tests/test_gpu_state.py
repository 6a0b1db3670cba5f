"""Restart snapshots (lb_get_state / lb_set_state) through the C interface.

A run is snapshotted, continued, and replayed from the snapshot in a fresh
context. The replay must start from a bit-identical state. It then follows
the original to within the order dependence of the FP64 atomic sums of the
sphere forces: about 1e-16 relative per step, which in FP32 storage shows as
an occasional one-unit change in a population (up to ~1e-7 of max|f|).
Mismatched snapshots are rejected, and non-finite populations brought in by a
snapshot are reported by lb_observables.
"""
import numpy as np
import pytest

import synth
from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _params(precision, **over):
    from paper_2004_04080_amd import Params
    kw = dict(ncomp=2, tau=(1.0, 1.0), G=0.65, precision=precision, max_particles=8,
              radius=4.0, particle_density=2.0, hertz_K=1.0)
    kw.update(over)
    return Params(40, 36, 32, **kw)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_snapshot_replay(precision, tol):
    from paper_2004_04080_amd import Lattice
    w = synth.Workload("state", 40, 36, 32, nparticles=6, radius=4.0, seed=synth.BASE_SEED + 51)
    x = w.centres()
    v = np.random.default_rng(3).uniform(-0.01, 0.01, (len(x), 3))
    a = Lattice(_params(precision), w.densities())
    a.add_particles(x, v)
    a.step(15)
    blob = a.state()
    a.step(10)
    fa, pa, ra = a.populations(), a.particles(), a.fields()[0]

    b = Lattice(_params(precision), np.ones((2, w.N)))
    b.set_state(blob)
    assert np.array_equal(b.state(), blob)
    assert b.observables().step == 15 and b.num_particles() == len(x)
    b.step(10)
    fb, pb, rb = b.populations(), b.particles(), b.fields()[0]
    ef = np.abs(fb - fa).max() / np.abs(fa).max()
    er = np.abs(rb - ra).max() / np.abs(ra).max()
    ex = np.abs(pb[:, :13] - pa[:, :13]).max()
    print(f"[state] {precision}: replay eps f {ef:.1e} rho {er:.1e} sphere state {ex:.1e}",
          flush=True)
    assert ef <= tol and er <= tol and ex <= 1e-9
    assert np.array_equal(a.owner(), b.owner())
    a.close()
    b.close()


def test_snapshot_mismatch_and_nonfinite():
    from paper_2004_04080_amd import Lattice, LBError
    w = synth.Workload("state2", 40, 36, 32, seed=synth.BASE_SEED + 52)
    a = Lattice(_params("fp32", max_particles=0), w.densities())
    a.step(2)
    blob = a.state()
    other = Lattice(_params("fp64", max_particles=0), w.densities())
    with pytest.raises(LBError):
        other.set_state(blob)
    other.close()
    with pytest.raises(LBError):
        a.set_state(blob[:100])
    bad = blob.copy()
    # a NaN in the rest population of node 1000 (first plane, after the 72-byte header)
    off = 72 + 4 * 1000
    bad[off:off + 4] = np.frombuffer(np.float32(np.nan).tobytes(), np.uint8)
    a.set_state(bad)
    obs = a.observables(raise_on_flag=False)
    assert obs.flags & 2
    a.close()


def test_set_particles_checks_and_moves_only_before_the_first_step():
    """lb_set_particles: every value must be finite and q non-zero; before the
    first step positions may change (wrapped into the box, checked for overlap
    like lb_add_particles, map rasterised again); after it only v, w, q and
    the previous forces may, and a moved sphere is refused. A refused call
    leaves the state as it was."""
    from paper_2004_04080_amd import Lattice, LBError
    from paper_2004_04080_amd import binding as B
    w = synth.Workload("setp", 40, 36, 32, seed=synth.BASE_SEED + 53)
    lat = Lattice(_params("fp64"), w.densities())
    lat.add_particles(np.array([[10.0, 10.0, 10.0], [30.0, 20.0, 16.0], [20.0, 28.0, 24.0]]))
    rec = lat.particles()
    own0 = lat.owner()

    bad = rec.copy()
    bad[0, B.REC["v"]] = np.nan
    with pytest.raises(LBError) as e:
        lat.set_particles(bad)
    assert e.value.status == B.LB_E_ARG
    bad = rec.copy()
    bad[1, B.REC["q"]:B.REC["q"] + 4] = 0.0
    with pytest.raises(LBError):
        lat.set_particles(bad)
    bad = rec.copy()
    bad[1, 0:3] = bad[0, 0:3] + np.array([5.0, 0.0, 0.0])      # centres 5 < 2R apart
    with pytest.raises(LBError) as e:
        lat.set_particles(bad)
    assert e.value.status == B.LB_E_OVERLAP
    assert np.array_equal(lat.owner(), own0)
    np.testing.assert_array_equal(lat.particles(), rec)

    # before the first step: a move, with a coordinate just below zero
    moved = rec.copy()
    moved[0, 0] = -1e-17          # wraps to x = 0, not to x = 40
    lat.set_particles(moved)
    got = lat.particles()
    assert got[0, 0] == 0.0
    assert not np.array_equal(lat.owner(), own0)
    lat.step(2)

    # after the first step: velocities may change, positions may not
    rec = lat.particles()
    faster = rec.copy()
    faster[:, B.REC["v"]:B.REC["v"] + 3] += 0.001
    lat.set_particles(faster)
    np.testing.assert_array_equal(lat.particles()[:, B.REC["v"]:B.REC["v"] + 3],
                                  faster[:, B.REC["v"]:B.REC["v"] + 3])
    moved = lat.particles()
    moved[0, 0] += 0.25
    with pytest.raises(LBError) as e:
        lat.set_particles(moved)
    assert e.value.status == B.LB_E_STATE
    lat.step(1)
    assert lat.observables().flags == 0
    lat.close()
