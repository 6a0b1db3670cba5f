#!/usr/bin/env python3
"""Throughput of the two-fluid + colloid D3Q19 step on one MI355X.

Default workload: a 512^3 periodic box, two Shan-Chen components (tau = 1,
G = 0.65, rho_k = 1 + 0.01 (2U - 1) per node) and 32,000 moving spheres of
radius 5.5 placed at random without overlap (16.6% solids), FP32 deviation
storage. Inputs are seeded and synthetic (no dataset is involved).

Prints one JSON line: MLUPS (all nodes counted, paper's Eq. glups) of --steps
steps after --warmup steps, timed with HIP events and no per-phase events;
then a second pass of --steps steps with per-phase HIP events gives the
kernel split and the roofline of the dominant kernel (collide-stream-
bounce-back). The line also carries the same workload timed from step 1000,
the FP64 path (MLUPS, roofline, FP32 error against it), the adjoint leg, the
fluid-only and confined boxes, the streaming probes of the library (the
attainable read, write, copy and collide-pattern rates) and the serial
oracle's MLUPS on a bounded sample of the workload (CPU baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 two-fluid+colloid MLUPS & % HBM peak, FP32 vs FP64 at stated error"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def params_for(w, precision):
    from paper_2004_04080_amd import Params
    return Params(w.nx, w.ny, w.nz, ncomp=w.ncomp, tau=w.tau, G=w.G, precision=precision,
                  walls=w.walls, wall_u_lo=w.wall_u_lo, wall_u_hi=w.wall_u_hi, g=w.g,
                  max_particles=w.nparticles, radius=w.radius,
                  particle_density=w.particle_density, hertz_K=w.hertz_K,
                  particles_fixed=w.particles_fixed)


def link_count(owner: np.ndarray, shape) -> tuple:
    """(fluid nodes, links from a fluid node to a solid neighbour) of a map."""
    nx, ny, nz = shape
    solid = (owner != 0).reshape(nz, ny, nx)
    fluid = ~solid
    links = 0
    for cx in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cz in (-1, 0, 1):
                if (cx, cy, cz) == (0, 0, 0) or abs(cx) + abs(cy) + abs(cz) > 2:
                    continue
                nb = np.roll(solid, shift=(-cz, -cy, -cx), axis=(0, 1, 2))
                links += int(np.count_nonzero(fluid & nb))
    return int(np.count_nonzero(fluid)), links


def _timed(lat, steps):
    """Milliseconds of `steps` steps between HIP events on the library's stream."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def run_gpu(w, rho, x, precision, steps, warmup, want_roofline, want_fields=False,
            late_at=0, fields_at=None):
    """One run of workload w: `warmup` untimed steps, `steps` timed steps
    (the headline, without per-phase events), then `steps` more with per-phase
    HIP events (the kernel split and the roofline). With fields_at the run
    then steps on to that step and reads the fields; with late_at it steps on
    to that step and times `steps` clean steps once more."""
    import torch
    from paper_2004_04080_amd import Lattice
    t0 = time.time()
    lat = Lattice(params_for(w, precision), rho)
    if len(x):
        lat.add_particles(x)
    log(f"[bench] {w.name} {precision}: state on the GPU after {time.time() - t0:.1f}s")
    lat.step(warmup)
    lat.sync()
    log(f"[bench] {w.name} {precision}: {warmup} warm-up steps done")
    ms = _timed(lat, steps) if steps else 0.0
    lat.timing(True)
    ms_ph = _timed(lat, steps)
    phases = lat.timing_read()
    lat.timing(False)
    done = warmup + 2 * steps
    obs = lat.observables(raise_on_flag=False)
    if not steps:
        ms = ms_ph
    log(f"[bench] {w.name} {precision}: {steps} steps in {ms:.1f} ms; with phase events "
        f"{ms_ph:.1f} ms; phases {phases}")
    out = dict(ms_per_step=ms / max(steps, 1), mlups=w.N * steps / (ms * 1e-3) / 1e6 if steps else 0,
               ms_per_step_phase_pass=ms_ph / max(steps, 1), phases=phases, flags=obs.flags,
               mass=obs.mass.tolist())
    if want_roofline:
        lat.domain_size()          # the first call creates the FFT plan
        t = time.time()
        L, _ = lat.domain_size()
        out["domain_size"] = {"L": round(L, 4), "ms": round((time.time() - t) * 1e3, 2)}
        own = lat.owner()
        nfl, nlinks = link_count(own, (w.nx, w.ny, w.nz))
        out["fluid_nodes"] = nfl
        out["links"] = nlinks
        del own
    if fields_at is not None:
        if fields_at > done:
            lat.step(fields_at - done)
            done = fields_at
        own = lat.owner()
        rho_f, u_f = lat.fields()
        out["fields"] = (own == 0, rho_f, u_f)
        out["fields_step"] = done
        del own
    if late_at:
        lat.step(max(late_at - done, 0))
        done = max(late_at, done)
        lat.sync()
        ms_late = _timed(lat, steps)
        obs = lat.observables(raise_on_flag=False)
        out["late"] = {"from_step": done, "steps": steps,
                       "ms_per_step": round(ms_late / steps, 4),
                       "value": round(w.N * steps / (ms_late * 1e-3) / 1e6, 1), "unit": "MLUPS",
                       "flags": obs.flags}
        log(f"[bench] {w.name} {precision}: from step {done}, {steps} steps in {ms_late:.1f} ms")
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


# committed rocprofv3 counter summaries of the 512^3 bench box, per precision
COUNTERS = {pr: os.path.join(ROOT, "profiles", f"k_collide_T512_{pr}_hbm_counters.md")
            for pr in ("fp32", "fp64")}
COLLIDE_SOURCES = ("paper_2004_04080_amd/csrc/lb_fluid.hip", "paper_2004_04080_amd/csrc/lb_device.hpp")


def measured_traffic(workload: str, precision: str):
    """HBM bytes per collide launch from the committed rocprofv3 FETCH_SIZE and
    WRITE_SIZE counters (scaled by the copy calibration), or None when they were
    taken on another workload or the collide sources changed since."""
    if workload != "T" or precision not in COUNTERS:
        return None
    try:
        text = open(COUNTERS[precision]).read()
        block = text.split("```counters", 1)[1].split("```", 1)[0]
        kv = dict(line.split(": ", 1) for line in block.strip().splitlines())
        h = hashlib.sha256()
        for f in COLLIDE_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != kv["source_sha256"]:
            return None
        return int(float(kv["traffic_bytes_per_dispatch"]))
    except (OSError, IndexError, KeyError, ValueError):
        return None


STEP_COUNTERS = {pr: os.path.join(ROOT, "profiles", f"step_T512_{pr}_hbm_traffic.md")
                 for pr in ("fp32", "fp64")}
# the method's minimum HBM bytes per node and step: populations read and
# written once, the pseudo-potential written and read once, the owner map read
MIN_BYTES_PER_NODE = {"fp32": 322, "fp64": 642}
CSRC = os.path.join(ROOT, "paper_2004_04080_amd", "csrc")
# the sources the kernels of lb_step are built from (the adjoint, domain-size,
# allocation-free and probe sources do not run in a step)
STEP_SOURCES = ("lb_api.hip", "lb_device.hpp", "lb_fluid.hip", "lb_internal.hpp",
                "lb_particles.hip")


def step_sources_sha256() -> str:
    """sha256 over the step's sources, in the order of STEP_SOURCES."""
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def step_traffic(w, precision: str, ms_per_step: float):
    """Whole-step HBM traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE over every
    kernel of a step, copy-calibrated, from the committed summary) over the
    step time just measured; None unless the summary's workload and
    precision match and the library's sources are those it was taken on."""
    if w.name != "T" or precision not in STEP_COUNTERS:
        return None
    try:
        text = open(STEP_COUNTERS[precision]).read()
        block = text.split("```counters", 1)[1].split("```", 1)[0]
        kv = dict(line.split(": ", 1) for line in block.strip().splitlines())
        if step_sources_sha256() != kv["source_sha256"]:
            return None
        b = float(kv["traffic_bytes_per_step"])
    except (OSError, IndexError, KeyError, ValueError):
        return None
    gbps = b / (ms_per_step * 1e-3) / 1e9
    m = MIN_BYTES_PER_NODE[precision]
    alg = m * w.N / (ms_per_step * 1e-3) / 1e9
    return {"bytes_per_step": int(b), "bytes_per_node": round(b / w.N, 1),
            "achieved_GBps": round(gbps, 1), "frac_of_peak": round(gbps / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_node": m,
            "algorithmic_GBps": round(alg, 1),
            "algorithmic_frac": round(alg / HBM_PEAK_GBS, 4),
            "source": os.path.relpath(STEP_COUNTERS[precision], ROOT)}


def roofline(w, res, es, precision):
    """Algorithmic bytes of one collide launch over its average duration."""
    K = w.ncomp
    nfl, nlinks, N = res["fluid_nodes"], res["links"], w.N
    bytes_launch = (nfl * 2 * K * 19 * es      # gather + store of the populations
                    + N * K * es               # pseudo-potential field, read once
                    + (N * 2 if w.walls or w.nparticles else 0))   # owner map
    ms, n = res["phases"]["collide"]
    avg_ms = ms / max(n, 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(w.name, precision),
            "kernel": "k_collide", "bytes_per_launch": bytes_launch,
            "avg_launch_ms": round(avg_ms, 4)}


def cpu_baseline():
    """The serial FP64 oracle on a bounded sample of the workload: a 128^3 box
    with the same fluid parameters and sphere volume fraction (500 spheres of
    radius 5.5), timed over 8 steps (about 10 s) on one host thread."""
    import oracle as O
    import synth
    w = synth.workload("C3")
    p = O.Params(w.nx, w.ny, w.nz, ncomp=2, tau=w.tau, G=w.G, radius=w.radius,
                 particle_density=w.particle_density, hertz_K=w.hertz_K)
    o = O.Oracle(p, w.densities())
    o.add_particles(w.centres())
    t = time.time()
    steps = 8
    o.step(steps)
    dt = time.time() - t
    return {"value": round(w.N * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} steps of a 128^3 two-fluid box with 500 spheres R=5.5 "
                      f"(same fluid parameters and volume fraction), {dt:.1f}s serial FP64"}


def accuracy(a, b, steps):
    """eps(X) = max|X_a - X_b| / max|X_b| over the fluid nodes of both runs."""
    fa, ra, ua = a
    fb, rb, ub = b
    m = fa & fb

    def eps(x, y):
        return float(np.abs(x[..., m] - y[..., m]).max() / np.abs(y[..., m]).max())
    out = {"against": "FP64 path from the same initial state (the FP64 path agrees with "
                      "the FP64 oracle to 1e-12 on the parity cases)",
           "steps": steps, "eps_rho": eps(ra, rb), "eps_u": eps(ua.T, ub.T)}
    if ra.shape[0] == 2:
        out["eps_phi"] = eps(ra[0] - ra[1], rb[0] - rb[1])
    return {k: (float(f"{v:.3e}") if isinstance(v, float) else v) for k, v in out.items()}


def adjoint_leg():
    """Reverse sweep on the differentiation box (64^3, 50 fixed spheres R=4,
    g_x = 1e-6, 500 steps, checkpoints every 50), FP64: forward and backward
    wall time, and dL/dG against a central difference of the forward."""
    import torch
    import synth
    from paper_2004_04080_amd import Lattice, Params
    w = synth.workload("C5")
    rho, x = w.densities(), w.centres()

    def make(G, rec):
        p = Params(w.nx, w.ny, w.nz, ncomp=2, tau=w.tau, G=G, g=w.g, precision="fp64",
                   radius=w.radius, max_particles=len(x), particles_fixed=True,
                   checkpoint_every=50 if rec else 0, max_record_steps=w.steps if rec else 0)
        lat = Lattice(p, rho)
        lat.add_particles(x)
        return lat
    lat = make(w.G, True)
    torch.cuda.synchronize()
    t0 = time.time()
    lat.step(w.steps)
    lat.sync()
    t1 = time.time()
    L, sA, sB = lat.loss(seeds=True)
    t2 = time.time()
    _, dG, _ = lat.backward(sA, sB)
    t3 = time.time()
    lat.close()
    h = 1e-4 * w.G
    Ls = []
    for G in (w.G + h, w.G - h):
        lt = make(G, False)
        lt.step(w.steps)
        Ls.append(lt.loss())
        lt.close()
    fd = (Ls[0] - Ls[1]) / (2 * h)
    return {"workload": "C5: 64^3 two fluids + 50 fixed spheres R=4, g_x=1e-6, 500 steps, "
                        "checkpoints every 50, FP64",
            "forward_ms": round((t1 - t0) * 1e3, 2), "loss_ms": round((t2 - t1) * 1e3, 2),
            "backward_ms": round((t3 - t2) * 1e3, 2), "dL_dG": dG, "dL_dG_central_difference": fd,
            "rel_err": float(f"{abs(dG - fd) / abs(fd):.3e}")}


def coarsening(name: str, steps: int, every: int, precision: str = "fp32",
               janus: bool = False) -> dict:
    """Average domain size L(t) (Eq. Cluster_L_eq) along one run of a
    synthetic box, with the wall-clock rate of the run. With janus the spheres
    carry the benchmark's particle model: Janus wetting (108 +- 5 degrees,
    constants 0.1) and lubrication (0.1, 0.67, 0.5)."""
    import dataclasses
    import synth
    from paper_2004_04080_amd import Lattice
    w = synth.workload(name)
    p = params_for(w, precision)
    if janus:
        p = dataclasses.replace(p, janus=True, janus_theta0=108.0, janus_width=10.0,
                                janus_zeta=(0.1, 0.1), lub_mu=0.1, lub_hn=0.67, lub_hcap=0.5)
    lat = Lattice(p, w.densities())
    if w.nparticles:
        lat.add_particles(w.centres())
    series, t0, done = [], time.time(), 0
    while done < steps:
        n = min(every, steps - done)
        lat.step(n)
        done += n
        L, _ = lat.domain_size()
        series.append([done, round(L, 3)])
        log(f"[coarsening] {w.name} {precision}{' janus' if janus else ''} step {done}: L = {L:.3f}")
    dt = time.time() - t0
    obs = lat.observables(raise_on_flag=False)
    lat.close()
    return {"coarsening": series, "workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz}, "
            f"{w.nparticles} spheres R={w.radius} ({100 * synth.sphere_fraction(w):.1f}% solid)"
            + (", Janus wetting 108+-5 deg (0.1, 0.1) and lubrication" if janus else
               ", neutral wetting"),
            "precision": precision, "steps": steps, "seconds": round(dt, 1), "flags": obs.flags}


def copy_probe(gib: float, reps: int = 5) -> dict:
    """The library's hand-written copy kernel (lb_probe_stream, 16-byte chunks)
    over a buffer of known size: the measured copy bandwidth, and the
    reference for scaling the FETCH_SIZE / WRITE_SIZE counters (each launch
    reads and writes `gib` GiB exactly once)."""
    import ctypes as C
    import torch
    from paper_2004_04080_amd import binding as B
    n = int(gib * (1 << 30)) // 16 * 16
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    b = torch.zeros_like(a)
    ms = C.c_double()
    B.check(B.lib().lb_probe_stream(2, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), n,
                                    0, 0, 0, reps,
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    C.byref(ms)), "lb_probe_stream")
    return {"copy_bytes_read": n, "copy_bytes_written": n, "launches": reps + 1,
            "ms": round(ms.value, 4),
            "GBps_read_plus_write": round(2 * n / (ms.value * 1e-3) / 1e9, 1)}


def stream_probes(gib: float = 8.0, box=(512, 512, 512), reps: int = 10,
                  march: bool = False) -> dict:
    """The library's streaming probes (lb_probe_stream): hand-written read,
    write and copy kernels over `gib` GiB, and the fused step's access pattern
    (2 x 19 FP32 planes gathered with the D3Q19 pull offsets and stored in
    place) on a box of the bench's size, and with march=True the same planes
    moved by a z-march that also takes the moments in its sweep (the pattern
    of a step without a separate density pass). GB/s counts the bytes each
    kernel must move (read + written)."""
    import ctypes as C
    import torch
    from paper_2004_04080_amd import binding as B
    lib = B.lib()
    stream = torch.cuda.current_stream()
    out = {}
    n = int(gib * (1 << 30)) // 16 * 16
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    b = torch.zeros_like(a)
    for kind, name, moved in ((0, "read", n), (1, "write", n), (2, "copy", 2 * n)):
        ms = C.c_double()
        B.check(lib.lb_probe_stream(kind, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), n,
                                    0, 0, 0, reps, C.c_void_p(stream.cuda_stream), C.byref(ms)),
                "lb_probe_stream")
        out[name] = {"GBps": round(moved / (ms.value * 1e-3) / 1e9, 1), "bytes": moved,
                     "ms": round(ms.value, 4)}
    del a, b
    torch.cuda.empty_cache()
    N = box[0] * box[1] * box[2]
    nb = 2 * 19 * N * 4
    a = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
    b = torch.zeros_like(a)
    ms = C.c_double()
    B.check(lib.lb_probe_stream(3, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nb,
                                box[0], box[1], box[2], reps, C.c_void_p(stream.cuda_stream),
                                C.byref(ms)), "lb_probe_stream")
    out["collide_pattern"] = {"GBps": round(2 * nb / (ms.value * 1e-3) / 1e9, 1),
                              "bytes": 2 * nb, "ms": round(ms.value, 4),
                              "box": f"{box[0]}x{box[1]}x{box[2]}"}
    if march and box[0] % 128 == 0 and box[1] % 8 == 0:
        # the same planes moved by a z-march that also takes the moments
        ms = C.c_double()
        B.check(lib.lb_probe_stream(4, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nb,
                                    box[0], box[1], box[2], reps,
                                    C.c_void_p(stream.cuda_stream), C.byref(ms)),
                "lb_probe_stream")
        out["march_pattern"] = {"GBps": round(2 * nb / (ms.value * 1e-3) / 1e9, 1),
                                "bytes": 2 * nb, "ms": round(ms.value, 4),
                                "box": f"{box[0]}x{box[1]}x{box[2]}"}
    del a, b
    torch.cuda.empty_cache()
    return out


def other_line(wo, ro, es, precision, steps):
    rl = roofline(wo, ro, es, precision)
    return {"workload": f"{wo.name}: {wo.nx}x{wo.ny}x{wo.nz}, {wo.nparticles} spheres"
                        + (", walls" if wo.walls else ""),
            "precision": precision,
            "value": round(ro["mlups"], 1), "unit": "MLUPS",
            "ms_per_step": round(ro["ms_per_step"], 4),
            "collide_GBps": rl["achieved"], "collide_frac": rl["frac"],
            "phases_ms_per_step": {k: round(v[0] / max(steps, 1), 4)
                                   for k, v in ro["phases"].items()}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="T")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--late", type=int, default=1000,
                    help="also time --steps steps of the main workload from this step (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 run (and with it the FP32 accuracy figure)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--march-probe", action="store_true",
                    help="also time the z-march probe (lb_probe_stream kind 4); not in the "
                         "default run")
    ap.add_argument("--workloads", default="MT0,C4",
                    help="comma-separated further boxes (C2,C3,C4,MT0) timed after the main "
                         "one and reported under other_workloads (same step counts)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run the library's copy kernel over this many GiB and report it")
    ap.add_argument("--coarsening", type=int, default=0,
                    help="only run this many steps of --workload (FP32) and report the "
                         "average domain size every --every steps")
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the reverse-sweep leg (differentiation box) and print it")
    ap.add_argument("--janus", action="store_true",
                    help="coarsening with the benchmark's Janus wetting and lubrication")
    args = ap.parse_args()
    if args.coarsening > 0:
        print(json.dumps(coarsening(args.workload, args.coarsening, args.every, args.precision,
                                    args.janus)), flush=True)
        return
    if args.copy_probe > 0:
        print(json.dumps(copy_probe(args.copy_probe)), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps(adjoint_leg()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the slab decomposition over RCCL is a design, not code). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import synth
    w = synth.workload(args.workload)
    es = 4 if args.precision == "fp32" else 8
    t0 = time.time()
    rho = w.densities()
    x = w.centres()
    log(f"[bench] {w.name}: seeded inputs ready in {time.time() - t0:.1f}s")
    check = not args.no_fp64 and args.precision == "fp32"
    cmp_at = args.warmup + 2 * args.steps
    res = run_gpu(w, rho, x, args.precision, args.steps, args.warmup, want_roofline=True,
                  fields_at=cmp_at if check else None, late_at=args.late)
    fp64 = acc = None
    if check:
        # the FP64 run: its phase pass ends at the step where the FP32 fields were read
        fsteps = max(1, min(args.fp64_steps, cmp_at // 2))
        r64 = run_gpu(w, rho, x, "fp64", fsteps, cmp_at - 2 * fsteps, want_roofline=True,
                      fields_at=cmp_at)
        fp64 = {"value": round(r64["mlups"], 1), "unit": "MLUPS", "steps": fsteps,
                "ms_per_step": round(r64["ms_per_step"], 3),
                "roofline": roofline(w, r64, 8, "fp64"),
                "step_traffic": step_traffic(w, "fp64", r64["ms_per_step"]),
                "phases_ms_per_step": {k: round(v[0] / max(fsteps, 1), 4)
                                       for k, v in r64["phases"].items()}}
        acc = accuracy(res.pop("fields"), r64.pop("fields"), cmp_at)
        log(f"[bench] FP32 against FP64 at step {cmp_at}: {acc}")
    adj = None if args.no_adjoint else adjoint_leg()
    others = []
    for name in [v for v in args.workloads.split(",") if v]:
        wo = synth.workload(name)
        ro = run_gpu(wo, wo.densities(), wo.centres(), args.precision, args.steps, args.warmup,
                     want_roofline=True)
        others.append(other_line(wo, ro, es, args.precision, args.steps))
        log(f"[bench] {others[-1]}")
    probes = None if args.no_probes else stream_probes(box=(w.nx, w.ny, w.nz),
                                                         march=args.march_probe)
    if probes:
        log(f"[bench] streaming probes: {probes}")
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    rl = roofline(w, res, es, args.precision)
    if probes:
        rl["frac_of_collide_pattern_probe"] = round(
            rl["achieved"] / probes["collide_pattern"]["GBps"], 4)
    line = {
        "metric": METRIC,
        "value": round(res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} two-fluid Shan-Chen D3Q19 "
                               f"(tau=1, G=0.65) + {w.nparticles} moving spheres R={w.radius}",
                   "nodes": w.N, "spheres": w.nparticles,
                   "fluid_nodes": res["fluid_nodes"], "links": res["links"]},
        "roofline": rl,
        "step_traffic": step_traffic(w, args.precision, res["ms_per_step"]),
        "cpu_baseline": cpu,
        "fp64": fp64,
        "accuracy": acc,
        "late": res.get("late"),
        "adjoint": adj,
        "other_workloads": others or None,
        "stream_probes": probes,
        "phase_pass": {"ms_per_step": round(res["ms_per_step_phase_pass"], 4),
                       "phases_ms_per_step": {k: round(v[0] / max(args.steps, 1), 4)
                                              for k, v in res["phases"].items()}},
        "domain_size": res.get("domain_size"),
        "flags": res["flags"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
