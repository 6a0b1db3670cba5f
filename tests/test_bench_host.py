"""Host logic of bench.py, without a GPU: the refusal of more than one GPU,
the fluid-node and link count of a map against brute force, the roofline's
algorithmic bytes (fluid nodes x 2 x K x 19 x es, plus the pseudo-potential
and the owner map once per node), the hash guard that ties the committed
counter summaries to the sources they were taken on, and the error measure
of the FP32-against-FP64 comparison."""
import os
import subprocess
import sys
import types

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_link_count_matches_brute_force():
    rng = np.random.default_rng(3)
    nx, ny, nz = 7, 6, 5
    owner = (rng.random(nx * ny * nz) < 0.3).astype(np.uint16) * 3
    fluid = links = 0
    for n in range(nx * ny * nz):
        x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
        if owner[n]:
            continue
        fluid += 1
        for cx in (-1, 0, 1):
            for cy in (-1, 0, 1):
                for cz in (-1, 0, 1):
                    if 0 < abs(cx) + abs(cy) + abs(cz) <= 2:
                        m = (x + cx) % nx + nx * (((y + cy) % ny) + ny * ((z + cz) % nz))
                        links += owner[m] != 0
    assert bench.link_count(owner, (nx, ny, nz)) == (fluid, links)


def test_roofline_bytes_and_fraction():
    w = types.SimpleNamespace(name="X", ncomp=2, N=1000, walls=False, nparticles=5)
    res = {"fluid_nodes": 800, "links": 123, "phases": {"collide": (4.0, 8)}}
    rl = bench.roofline(w, res, 4, "fp32")
    want = 800 * 2 * 2 * 19 * 4 + 1000 * 2 * 4 + 1000 * 2
    assert rl["bytes_per_launch"] == want
    assert rl["avg_launch_ms"] == 0.5
    assert abs(rl["achieved"] - want / 0.5e-3 / 1e9) < 0.1
    assert rl["frac"] == round(rl["achieved"] / bench.HBM_PEAK_GBS, 4)
    assert rl["traffic"] is None          # no counters were taken on this workload
    # without walls or spheres the owner map is not read
    w0 = types.SimpleNamespace(name="X", ncomp=2, N=1000, walls=False, nparticles=0)
    assert bench.roofline(w0, res, 8, "fp64")["bytes_per_launch"] == 800 * 2 * 2 * 19 * 8 + 1000 * 2 * 8


def _counter_file(path, sha, value):
    path.write_text("# summary\n\n```counters\nkernel: k\nsource_sha256: %s\n"
                    "traffic_bytes_per_dispatch: %d\n```\n" % (sha, value))


def test_counter_summary_applies_only_to_its_sources(tmp_path, monkeypatch):
    import hashlib
    h = hashlib.sha256()
    for f in bench.COLLIDE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    p, q = tmp_path / "c.md", tmp_path / "c64.md"
    monkeypatch.setattr(bench, "COUNTERS", {"fp32": str(p), "fp64": str(q)})
    _counter_file(p, h.hexdigest(), 123456789)
    assert bench.measured_traffic("T", "fp32") == 123456789
    assert bench.measured_traffic("T", "fp64") is None      # no summary taken in FP64
    _counter_file(q, h.hexdigest(), 987654321)
    assert bench.measured_traffic("T", "fp64") == 987654321
    assert bench.measured_traffic("C4", "fp32") is None
    assert bench.measured_traffic("T", "fp16") is None
    _counter_file(p, "0" * 64, 123456789)
    assert bench.measured_traffic("T", "fp32") is None
    assert bench.measured_traffic("T", "fp64") == 987654321


def test_step_traffic_applies_only_to_its_sources(tmp_path, monkeypatch):
    import hashlib
    h = hashlib.sha256()
    for f in bench.STEP_SOURCES:
        with open(os.path.join(bench.CSRC, f), "rb") as fh:
            h.update(fh.read())
    assert h.hexdigest() == bench.step_sources_sha256()
    p, q = tmp_path / "s.md", tmp_path / "s64.md"
    monkeypatch.setattr(bench, "STEP_COUNTERS", {"fp32": str(p), "fp64": str(q)})
    w = types.SimpleNamespace(name="T", N=512 ** 3)
    p.write_text("```counters\nsource_sha256: %s\ntraffic_bytes_per_step: 75000000000\n```\n"
                 % h.hexdigest())
    st = bench.step_traffic(w, "fp32", 15.0)
    assert st["bytes_per_step"] == 75000000000
    assert abs(st["achieved_GBps"] - 5000.0) < 0.1
    assert st["algorithmic_bytes_per_node"] == 322
    assert bench.step_traffic(w, "fp64", 15.0) is None
    q.write_text("```counters\nsource_sha256: %s\ntraffic_bytes_per_step: 150000000000\n```\n"
                 % h.hexdigest())
    st = bench.step_traffic(w, "fp64", 30.0)
    assert abs(st["achieved_GBps"] - 5000.0) < 0.1
    assert st["algorithmic_bytes_per_node"] == 642
    assert abs(st["algorithmic_GBps"] - 642 * 512 ** 3 / 30e-3 / 1e9) < 0.1
    p.write_text("```counters\nsource_sha256: %s\ntraffic_bytes_per_step: 1\n```\n" % ("f" * 64))
    assert bench.step_traffic(w, "fp32", 15.0) is None


def test_accuracy_is_relative_max_error_on_common_fluid_nodes():
    fa = np.array([True, True, False, True])
    fb = np.array([True, False, True, True])
    ra = np.array([[1.0, 9.0, 9.0, 2.0], [1.0, 9.0, 9.0, 1.0]])
    rb = np.array([[1.0, 0.0, 0.0, 2.5], [1.0, 0.0, 0.0, 1.0]])
    ua = np.zeros((4, 3))
    ub = np.ones((4, 3))
    out = bench.accuracy((fa, ra, ua), (fb, rb, ub), 7)
    assert out["steps"] == 7
    assert out["eps_rho"] == 0.5 / 2.5          # nodes 0 and 3 only
    assert out["eps_u"] == 1.0
    assert abs(out["eps_phi"] - 0.5 / 1.5) < 1e-3    # reported to four digits
