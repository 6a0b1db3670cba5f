"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws numbers and lays out boxes. It holds none of the
lattice-Boltzmann arithmetic, so both implementations can take their inputs
from it without sharing any part of the method.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter hash:

    U(seed, stream, n) = (splitmix64(seed ^ splitmix64(stream * 2**40 + n)) >> 11) / 2**53

so a value depends only on (seed, stream, n), never on how work is split.

The workloads stand in for the paper's randomly initialised benchmark boxes
(two fluids of mean density 1 with small noise, spheres of radius 5.5 placed
at random without overlap); no dataset is involved.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

BASE_SEED = 2004040800
STREAM_RHO = (0, 1)      # density noise of component A, B
STREAM_PLACE = 7         # sphere placement

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied to an array of uint64 counters."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """U(seed, stream, n) for n = start .. start+count-1, in [0, 1), float64."""
    n = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = np.uint64(stream) * np.uint64(1 << 40) + n
        h = splitmix64(np.uint64(seed) ^ splitmix64(ctr))
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def noisy_density(seed: int, comp: int, nx: int, ny: int, nz: int,
                  mean: float = 1.0, amp: float = 0.01) -> np.ndarray:
    """rho = mean + amp * (2U - 1) per node, node order n = x + nx*(y + ny*z)."""
    u = uniform(seed, STREAM_RHO[comp], nx * ny * nz)
    return mean + amp * (2.0 * u - 1.0)


def shear_wave_velocity(nx: int, ny: int, nz: int, amp: float = 0.01) -> np.ndarray:
    """u_x = amp * sin(2 pi z / nz), u_y = u_z = 0, as an [N, 3] array."""
    z = np.arange(nx * ny * nz) // (nx * ny)
    u = np.zeros((nx * ny * nz, 3))
    u[:, 0] = amp * np.sin(2.0 * np.pi * z / nz)
    return u


def _min_image(d: np.ndarray, L: np.ndarray) -> np.ndarray:
    return d - L * np.round(d / L)


def place_spheres(seed: int, n: int, box, dmin: float,
                  zrange: Optional[tuple] = None, max_tries: int = 200) -> np.ndarray:
    """Random sequential addition of n centres in a periodic box.

    A candidate centre (three uniform draws from the placement stream) is
    accepted when its minimum-image distance to every accepted centre is at
    least dmin. zrange=(lo, hi) restricts the z coordinate (boxes with walls).
    Raises RuntimeError if the box is too crowded.
    """
    L = np.asarray(box, dtype=np.float64)
    cell = max(dmin, 1.0)
    ncell = np.maximum((L // cell).astype(int), 1)
    grid: dict = {}
    out = np.zeros((n, 3))
    k = 0
    ctr = 0
    tries_left = max_tries * max(n, 1)
    while k < n:
        if tries_left == 0:
            raise RuntimeError(f"could only place {k} of {n} spheres")
        tries_left -= 1
        u = uniform(seed, STREAM_PLACE, 3, start=3 * ctr)
        ctr += 1
        c = u * L
        if zrange is not None:
            c[2] = zrange[0] + u[2] * (zrange[1] - zrange[0])
        ci = (c / L * ncell).astype(int) % ncell
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    key = tuple((ci + (dx, dy, dz)) % ncell)
                    for j in grid.get(key, ()):
                        d = _min_image(out[j] - c, L)
                        if float(d @ d) < dmin * dmin:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            out[k] = c
            grid.setdefault(tuple(ci), []).append(k)
            k += 1
    return out


@dataclass
class Workload:
    """One synthetic box: sizes, physical parameters and initial data."""
    name: str
    nx: int
    ny: int
    nz: int
    ncomp: int = 2
    tau: tuple = (1.0, 1.0)
    G: float = 0.65
    walls: bool = False
    wall_u_lo: tuple = (0.0, 0.0, 0.0)
    wall_u_hi: tuple = (0.0, 0.0, 0.0)
    g: tuple = (0.0, 0.0, 0.0)
    nparticles: int = 0
    radius: float = 5.5
    particle_density: float = 1.0
    hertz_K: float = 20.0
    particles_fixed: bool = False
    steps: int = 100
    seed: int = BASE_SEED
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def hertz_d0(self) -> float:
        return 2.0 * self.radius + 1.0

    @property
    def hertz_rcap(self) -> float:
        return 2.0 * self.radius

    def densities(self) -> np.ndarray:
        """[ncomp, N] initial densities 1 + 0.01 (2U - 1) per node and component."""
        return np.stack([noisy_density(self.seed, k, self.nx, self.ny, self.nz)
                         for k in range(self.ncomp)])

    def centres(self) -> np.ndarray:
        if self.nparticles == 0:
            return np.zeros((0, 3))
        zr = None
        if self.walls:
            zr = (self.radius + 2.0, self.nz - 3.0 - self.radius)
        return place_spheres(self.seed, self.nparticles, (self.nx, self.ny, self.nz),
                             self.hertz_d0, zrange=zr)


def workload(name: str) -> Workload:
    """The named synthetic boxes of the measurement and parity plan."""
    s = BASE_SEED
    if name == "C1":
        return Workload("C1", 32, 32, 32, ncomp=1, tau=(0.8, 0.8), G=0.0, steps=200, seed=s + 1,
                        notes="one component, shear wave u_x = 0.01 sin(2 pi z/32), FP64")
    if name == "C2":
        return Workload("C2", 128, 128, 128, steps=1000, seed=s + 2,
                        notes="two components, spinodal decomposition")
    if name == "C3":
        return Workload("C3", 128, 128, 128, nparticles=500, radius=5.5, steps=2000, seed=s + 3,
                        notes="C2 plus 500 spheres R=5.5")
    if name == "C4":
        return Workload("C4", 512, 512, 256, nparticles=20000, radius=4.0, walls=True,
                        wall_u_lo=(-0.01, 0.0, 0.0), wall_u_hi=(0.01, 0.0, 0.0),
                        steps=5000, seed=s + 4,
                        notes="confined bijel under shear, walls z=0 and z=255")
    if name == "C5":
        return Workload("C5", 64, 64, 64, nparticles=50, radius=4.0, particles_fixed=True,
                        g=(1e-6, 0.0, 0.0), steps=500, seed=s + 5,
                        notes="adjoint box, fixed spheres")
    if name == "T":
        return Workload("T", 512, 512, 512, nparticles=32000, radius=5.5, steps=200, seed=s + 6,
                        notes="512^3 two fluids plus 32,000 spheres R=5.5")
    if name == "B20":
        return Workload("B20", 256, 256, 256, nparticles=4815, radius=5.5, steps=20000,
                        seed=s + 8, notes="256^3 two fluids plus 20% solids (R=5.5), coarsening")
    if name == "B0":
        return Workload("B0", 256, 256, 256, steps=20000, seed=s + 8,
                        notes="256^3 two fluids without spheres, coarsening")
    if name == "MT0":
        return Workload("MT0", 512, 512, 512, steps=200, seed=s + 7,
                        notes="512^3 two fluids, no spheres")
    raise KeyError(name)


def sphere_fraction(w: Workload) -> float:
    return w.nparticles * 4.0 / 3.0 * math.pi * w.radius ** 3 / w.N
