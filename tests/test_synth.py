"""The seeded input generators (synth/): the hash is SplitMix64 as published,
values depend only on (seed, stream, counter), and the boxes have the sizes,
value ranges and sphere placements their descriptions state."""
import math

import numpy as np
import pytest

import synth


def test_splitmix64_reference_sequence():
    # outputs of the reference generator (Vigna's splitmix64.c; the generator
    # of Steele, Lea and Flood) started from state 0: state k*gamma -> output k
    gamma = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        states = np.arange(5, dtype=np.uint64) * gamma
    got = [int(v) for v in synth.splitmix64(states)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                   0xF88BB8A8724C81EC, 0x1B39896A51A8749B]


def test_uniform_depends_only_on_seed_stream_and_counter():
    a = synth.uniform(synth.BASE_SEED, 3, 1000)
    assert a.dtype == np.float64 and (a >= 0).all() and (a < 1).all()
    assert np.array_equal(a, synth.uniform(synth.BASE_SEED, 3, 1000))
    # any split of the counter range gives the same values
    assert np.array_equal(a[250:700], synth.uniform(synth.BASE_SEED, 3, 450, start=250))
    # other streams and seeds give other values
    assert not np.array_equal(a, synth.uniform(synth.BASE_SEED, 4, 1000))
    assert not np.array_equal(a, synth.uniform(synth.BASE_SEED + 1, 3, 1000))
    # 53-bit uniforms: mean and variance of 1e5 draws within a few standard errors
    u = synth.uniform(synth.BASE_SEED, 9, 100000)
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 5e-3


def test_noisy_density_range_and_layout():
    r = synth.noisy_density(synth.BASE_SEED, 0, 7, 5, 3)
    assert r.shape == (105,)
    assert (r >= 0.99).all() and (r <= 1.01).all()
    assert np.array_equal(r, 1.0 + 0.01 * (2 * synth.uniform(synth.BASE_SEED, 0, 105) - 1))
    # the two components draw from streams of their own
    assert not np.array_equal(r, synth.noisy_density(synth.BASE_SEED, 1, 7, 5, 3))


@pytest.mark.parametrize("walls", [False, True])
def test_sphere_placement_keeps_its_distances(walls):
    w = synth.Workload("t", 64, 48, 40, nparticles=60, radius=3.0, walls=walls,
                       seed=synth.BASE_SEED + 99)
    x = w.centres()
    assert x.shape == (60, 3)
    L = np.array([64.0, 48.0, 40.0])
    assert (x >= 0).all() and (x < L).all()
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(len(x)) * 1e9
    assert r.min() >= w.hertz_d0                 # no two centres closer than 2R + 1
    if walls:                                    # clear of the wall layers z = 0, nz - 1
        assert (x[:, 2] >= w.radius + 2.0).all() and (x[:, 2] <= 40 - 3.0 - w.radius).all()
    assert np.array_equal(x, w.centres())        # reproducible


def test_named_boxes():
    t = synth.workload("T")
    assert (t.nx, t.ny, t.nz, t.nparticles, t.radius) == (512, 512, 512, 32000, 5.5)
    assert abs(synth.sphere_fraction(t) - 0.166) < 1e-3
    c4 = synth.workload("C4")
    assert c4.walls and (c4.nx, c4.ny, c4.nz, c4.nparticles, c4.radius) == (512, 512, 256, 20000, 4.0)
    b20 = synth.workload("B20")
    assert abs(synth.sphere_fraction(b20) - 0.20) < 1e-3
    for name in ("C1", "C2", "C3", "C5", "MT0", "B0"):
        assert synth.workload(name).name == name
    with pytest.raises(KeyError):
        synth.workload("nope")
