"""One-step parity of the FP32 path at full size: the bench box (512^3, two
fluids, 32,000 moving spheres of radius 5.5) and the confined box
(512x512x256 between moving walls, 20,000 spheres of radius 4), each built
with the parameters that bench.py uses for it.

The oracle cannot step the whole box, so it steps windows of it. After a few
steps on the GPU (or 200, when the components have begun to separate and the
spheres move, with windows centred on node events), the state (FP32 populations read out as FP64, the map and
the sphere records) of four 80^3 windows is handed to the oracle, which
steps each window once as a periodic box of its own. One step reaches only a
few nodes: streaming, the pseudo-potential stencil, the frontier fill and the
node events each reach one node. A sphere centred up to R + 1 outside a
window is wrapped by the oracle's periodicity onto the far side, where it
reaches up to 2R + 1 into the window. Nodes at least 16 from every window
face are therefore exact copies of the full-box step and are compared: the
map bit for bit, the populations, densities, phi and u to the FP32 bounds of
the other parity tests. Spheres whose whole surface lies in that interior
also have their link, event and Shan-Chen forces and torques compared. Pair
forces are switched off in the oracle windows because they act on the
spheres only after the fluid has been updated.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import perm_gpu_for_oracle, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

W = 80          # window edge
MARGIN = 16     # nodes next to a window face that are not compared
TOL32 = 1e-5
TOL32_U = 5e-5  # derivation in tests/test_gpu_parity.py
TOL64 = 1e-12


def _window_index(origin, shape, win):
    ax = [(origin[d] + np.arange(win[d])) % shape[d] for d in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return (x + shape[0] * (y + shape[1] * z)).reshape(-1).astype(np.int64)


def _eps(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _event_origins(lat, shape, win, per_kind=2):
    """Window origins centred on nodes that the next step creates or destroys:
    the step is taken once from a snapshot to find them, and the snapshot is
    restored."""
    blob = lat.state()
    own_a = lat.owner()
    lat.step(1)
    own_b = lat.owner()
    lat.set_state(blob)
    del blob
    created = np.flatnonzero((own_a > 0) & (own_b == 0))
    destroyed = np.flatnonzero((own_a == 0) & (own_b > 0))
    print(f"[fullsize] next step: {created.size} nodes created, {destroyed.size} destroyed",
          flush=True)
    assert created.size > 0 and destroyed.size > 0
    rng = np.random.default_rng(9)
    origins = []
    for nodes in (created, destroyed):
        for n in rng.choice(nodes, size=min(per_kind, nodes.size), replace=False):
            xyz = (n % shape[0], (n // shape[0]) % shape[1], n // (shape[0] * shape[1]))
            origins.append(tuple(int((xyz[d] - win[d] // 2) % shape[d]) if win[d] < shape[d]
                                 else 0 for d in range(3)))
    return origins


def _window_parity(name, origins, warm=3, precision="fp32", events=False):
    """Step the bench state of workload `name` on the GPU, then one step of
    each window in the oracle; compare the window interiors. With walls a
    window spans the whole z height with the real walls, and only its x and y
    faces are periodic wraps (and excluded from the comparison). With events
    the windows are centred on nodes that the compared step creates or
    destroys, and each window interior must hold node events."""
    import bench
    from paper_2004_04080_amd import Lattice
    w = synth.workload(name)
    shape = (w.nx, w.ny, w.nz)
    win = (W, W, w.nz if w.walls else W)
    tol = TOL32 if precision == "fp32" else TOL64
    tol_u = TOL32_U if precision == "fp32" else TOL64
    print(f"[fullsize] building the {shape} state of {name} ({precision}), {warm} steps",
          flush=True)
    lat = Lattice(bench.params_for(w, precision), w.densities())
    lat.add_particles(w.centres())
    lat.step(warm)
    if events:
        origins = _event_origins(lat, shape, win)
    idx = [_window_index(o, shape, win) for o in origins]
    f = lat.populations()
    f0 = [f[:, :, i] for i in idx]
    del f
    own = lat.owner()
    own0 = [own[i] for i in idx]
    rec0 = lat.particles()
    lat.step(1)
    f = lat.populations()
    f1 = [f[:, :, i] for i in idx]
    del f
    own = lat.owner()
    own1 = [own[i] for i in idx]
    rec1 = lat.particles()
    rho_g, u_g = lat.fields()
    rho1 = [rho_g[:, i] for i in idx]
    u1 = [u_g[i] for i in idx]
    del rho_g, u_g, own
    lat.close()
    print("[fullsize] GPU state read; stepping the oracle windows", flush=True)

    perm = perm_gpu_for_oracle()
    L = np.array(shape, dtype=float)
    R = w.radius
    half = (np.array(win, dtype=float) - 1) / 2.0
    wrapped = np.array([True, True, not w.walls])   # axes where the window is a periodic cut
    REC = O.REC
    inner = np.ones(win[::-1], dtype=bool)           # [z][y][x]
    for a in range(3):
        if wrapped[a]:
            sl = [slice(None)] * 3
            keep = np.zeros(win[a], dtype=bool)
            keep[MARGIN:win[a] - MARGIN] = True
            shape_a = [1, 1, 1]
            shape_a[2 - a] = win[a]
            inner &= keep.reshape(shape_a)
    inner = inner.reshape(-1)
    nspheres_checked = 0
    for k, org in enumerate(origins):
        # spheres that can touch the window, in window coordinates, global order kept
        d = rec0[:, REC["x"]:REC["x"] + 3] - (np.array(org, dtype=float) + half)
        d -= np.where(wrapped, L * np.round(d / L), 0.0)
        sel = np.flatnonzero(np.all(np.abs(d) < half + R + 1.0, axis=1))
        xw = d[sel] + half
        local = np.zeros(len(rec0) + 1, dtype=np.int32)
        local[sel + 1] = np.arange(1, len(sel) + 1, dtype=np.int32)

        def to_local(o):
            return np.where(o > 0, local[np.maximum(o, 0)], o)

        po = O.Params(*win, ncomp=2, tau=w.tau, G=w.G, sc_norm=1.0, g=w.g, radius=R,
                      particle_density=w.particle_density, hertz_K=0.0, walls=w.walls,
                      wall_u_lo=w.wall_u_lo, wall_u_hi=w.wall_u_hi)
        o = O.Oracle(po, np.ones((2, int(np.prod(win)))))
        o.add_particles(xw)
        r = o.particles()
        for key, n in (("v", 3), ("w", 3), ("q", 4), ("Fprev", 3), ("Tprev", 3)):
            r[:, REC[key]:REC[key] + n] = rec0[sel, REC[key]:REC[key] + n]
        r[:, REC["have_prev"]] = rec0[sel, REC["have_prev"]]
        o.set_particle_state(r)
        o.set_owner(to_local(own0[k]))
        o.set_f(f0[k][:, perm, :])
        o.step(1)

        own_o = o.owner()
        own_g = to_local(own1[k])
        assert np.array_equal(own_o[inner], own_g[inner]), f"map, window {org}"
        m = inner & (own_o == 0)
        fo = o.f()[:, :, m]
        fg = f1[k][:, perm, :][:, :, m]
        ro = o.rho()[:, m]
        rg = rho1[k][:, m]
        e = {"f": _eps(fg, fo),
             "rho0": _eps(rg[0], ro[0]), "rho1": _eps(rg[1], ro[1]),
             "phi": _eps(rg[0] - rg[1], ro[0] - ro[1]),
             "u": _eps(u1[k][m], o.u()[m])}
        nev = int(((own0[k] != 0) != (own1[k] != 0))[inner].sum())
        print(f"[fullsize] {name} window {org}: {m.sum()} fluid nodes, {nev} node events, "
              + " ".join(f"{a} {b:.1e}" for a, b in e.items()), flush=True)
        if events:
            assert nev > 0, f"no node event inside window {org}"
        for key in ("f", "rho0", "rho1", "phi"):
            assert e[key] <= tol, (org, key, e[key])
        assert e["u"] <= tol_u, (org, e["u"])

        # spheres whose links and events all fall in the compared interior
        lo = np.where(wrapped, MARGIN + R + 2.0, -np.inf)
        hi = np.where(wrapped, np.array(win) - 1 - MARGIN - R - 2.0, np.inf)
        whole = np.flatnonzero(np.all((xw >= lo) & (xw <= hi), axis=1))
        ro_p = o.particles()
        for j in whole:
            gp = rec1[sel[j]]
            op = ro_p[j]
            scale = op[REC["flabs"]]
            for key in ("Fliq", "Tliq", "FSC", "TSC", "Fd", "Td", "Fc", "Tc"):
                err = np.abs(gp[REC[key]:REC[key] + 3] - op[REC[key]:REC[key] + 3]).max() / scale
                assert err < tol, (org, int(sel[j]), key, err)
        nspheres_checked += len(whole)
    print(f"[fullsize] {name}: spheres compared: {nspheres_checked}", flush=True)
    assert nspheres_checked > 0


def test_full_size_one_step_parity_on_windows():
    """The bench box: 512^3, 32,000 moving spheres of radius 5.5."""
    rng = np.random.default_rng(5)
    origins = [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(4)]
    _window_parity("T", origins)


def test_confined_box_one_step_parity_on_windows():
    """The confined case: 512x512x256 between walls moving at -+0.01 in x,
    20,000 spheres of radius 4. Each window spans the full height."""
    rng = np.random.default_rng(6)
    origins = [(int(rng.integers(0, 512)), int(rng.integers(0, 512)), 0) for _ in range(3)]
    _window_parity("C4", origins)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_demixed_state_with_node_events(precision):
    """The bench box after 200 steps, when the components have started to
    separate and the spheres move: one step compared on four windows centred
    on nodes that the step creates or destroys (two of each), in FP32 at
    1e-5 and in FP64 at 1e-12 against the oracle."""
    _window_parity("T", None, warm=200, precision=precision, events=True)
