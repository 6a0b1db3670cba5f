"""Independent 50-digit transcription of one LBsoft time step (test helper).

Written directly from Sec. 2 and the eight-step particle sequence of Sec. 3.1
of Bonaccorso et al. (arXiv 2004.04080), with the same readings of the paper
as the oracle, but with its own data structures (dicts keyed by node tuples),
its own direction order and Python's ``decimal`` arithmetic at 50 digits. It
is used only on tiny boxes (4^3 .. 6^3) to pin the oracle: any dropped term,
wrong sign, index or transposed operand in either implementation shows up as
a difference far above double rounding.
"""
from __future__ import annotations

import itertools
from decimal import Decimal as D, getcontext

getcontext().prec = 50

# pi to 60 digits (a mathematical constant, for the sphere mass)
PI = D("3.14159265358979323846264338327950288419716939937510582097494")

# D3Q19 in this helper's own order: lexicographic over {-1,0,1}^3, |c|^2 <= 2
DIRS = [c for c in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in c) <= 2]
assert len(DIRS) == 19
W = {c: (D(1) / 3 if sum(a * a for a in c) == 0 else
         D(1) / 18 if sum(a * a for a in c) == 1 else D(1) / 36) for c in DIRS}
CS2 = D(1) / 3
ZERO3 = (D(0), D(0), D(0))


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def scale(s, a):
    return (s * a[0], s * a[1], s * a[2])


def cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def wrap(x, L):
    """x mod L in [0, L) (Decimal's % keeps the dividend's sign)."""
    L = D(L)
    return x - L * (x / L).to_integral_value(rounding="ROUND_FLOOR")


def equilibrium(c, rho, u):
    """Eq. LEQ: w rho (1 + c.u/cs2 + ((c.u)^2 - cs2 u.u)/(2 cs2^2))."""
    cu = dot(c, u)
    return W[c] * rho * (1 + cu / CS2 + (cu * cu - CS2 * dot(u, u)) / (2 * CS2 * CS2))


class Brute:
    def __init__(self, shape, ncomp, tau, G, sc_norm, g, rho0, u0=None, walls=False,
                 u_lo=(0, 0, 0), u_hi=(0, 0, 0), radius=1.0, pdens=1.0, hertz=(20, 3, 2),
                 zeta=(0, 0), rho_fallback=(1, 1), rotate=True):
        self.L = tuple(shape)
        self.K = ncomp
        self.tau = [D(repr(t)) for t in tau]
        self.G = D(repr(G))
        self.s = D(repr(sc_norm))
        self.g = tuple(D(repr(a)) for a in g)
        self.walls = walls
        self.ulo = tuple(D(repr(a)) for a in u_lo)
        self.uhi = tuple(D(repr(a)) for a in u_hi)
        self.R = D(repr(radius))
        self.mass = D(repr(pdens)) * 4 * PI * self.R ** 3 / 3
        self.inertia = D(2) / 5 * self.mass * self.R * self.R
        self.hK, self.hd0, self.hcap = (D(repr(a)) for a in hertz)
        self.zeta = [D(repr(z)) for z in zeta]
        self.rfb = [D(repr(z)) for z in rho_fallback]
        self.rotate = rotate
        nx, ny, nz = self.L
        self.nodes = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
        self.own = {n: (-1 if self.wall_layer(n) else 0) for n in self.nodes}
        self.parts = []
        self.f = {}
        for idx, n in enumerate(self.nodes):
            if self.own[n]:
                continue
            u = ZERO3 if u0 is None else tuple(D(repr(float(a))) for a in u0[idx])
            for k in range(self.K):
                r = D(repr(float(rho0[k][idx])))
                self.f[(k, n)] = {c: equilibrium(c, r, u) for c in DIRS}

    # geometry ---------------------------------------------------------------
    def wall_layer(self, n):
        return self.walls and n[2] in (0, self.L[2] - 1)

    def nb(self, n, c, sign=1):
        return tuple((n[a] + sign * c[a]) % self.L[a] for a in range(3))

    def mi(self, d, a):
        L = D(self.L[a])
        q = (d / L).to_integral_value(rounding="ROUND_HALF_EVEN")
        return d - L * q

    def sep(self, point, xp):
        return tuple(self.mi(D(point[a]) - xp[a], a) for a in range(3))

    def raster(self):
        M = {n: (-1 if self.wall_layer(n) else 0) for n in self.nodes}
        for p, P in enumerate(self.parts):
            for n in self.nodes:
                if M[n] != 0:
                    continue
                d = self.sep(n, P["x"])
                if dot(d, d) < self.R * self.R:
                    M[n] = p + 1
        return M

    def add_particles(self, xs, vs=None, ws=None):
        for i, x in enumerate(xs):
            self.parts.append(dict(
                x=tuple(wrap(D(repr(float(a))), self.L[k]) for k, a in enumerate(x)),
                v=ZERO3 if vs is None else tuple(D(repr(float(a))) for a in vs[i]),
                w=ZERO3 if ws is None else tuple(D(repr(float(a))) for a in ws[i]),
                q=(D(1), D(0), D(0), D(0)), Fprev=ZERO3, Tprev=ZERO3, have_prev=False))
        M = self.raster()
        for n in self.nodes:
            if M[n] != 0 and self.own[n] == 0:
                for k in range(self.K):
                    del self.f[(k, n)]
        self.own = M

    # one step ---------------------------------------------------------------
    def step(self):
        K, nodes = self.K, self.nodes
        fluid_old = {n for n in nodes if self.own[n] == 0}
        # S1 moments on the old map
        rho, j, u = {}, {}, {}
        for n in fluid_old:
            num, den = ZERO3, D(0)
            for k in range(K):
                fk = self.f[(k, n)]
                rho[(k, n)] = sum(fk.values(), D(0))
                jj = ZERO3
                for c in DIRS:
                    jj = add(jj, scale(fk[c], c))
                j[(k, n)] = jj
                num = add(num, scale(1 / self.tau[k], jj))
                den += rho[(k, n)] / self.tau[k]
            u[n] = scale(1 / den, num)
        acc = {p: {key: ZERO3 for key in ("Fd", "Td", "Fc", "Tc", "FH", "FSC", "TSC",
                                          "Fl", "Tl")} for p in range(len(self.parts))}
        # S2 new map and events
        new = dict(self.own)
        if self.parts:
            new = self.raster()
            for n in nodes:
                o, w_ = self.own[n], new[n]
                if o == 0 and w_ > 0:
                    p = w_ - 1
                    J = ZERO3
                    for k in range(K):
                        J = add(J, j[(k, n)])
                    d = self.sep(n, self.parts[p]["x"])
                    acc[p]["Fd"] = add(acc[p]["Fd"], J)
                    acc[p]["Td"] = add(acc[p]["Td"], cross(d, J))
                    for k in range(K):
                        del self.f[(k, n)]
                        del rho[(k, n)]
                    del u[n]
            for n in nodes:
                o, w_ = self.own[n], new[n]
                if o > 0 and w_ == 0:
                    p = o - 1
                    P = self.parts[p]
                    d = self.sep(n, P["x"])
                    uw = add(P["v"], cross(P["w"], d))
                    both = [c for c in DIRS if c != (0, 0, 0)
                            and self.own[self.nb(n, c)] == 0 and new[self.nb(n, c)] == 0]
                    wsum = sum((W[c] for c in both), D(0))
                    tot = D(0)
                    for k in range(K):
                        rb = (sum((W[c] * rho[(k, self.nb(n, c))] for c in both), D(0)) / wsum
                              if both else self.rfb[k])
                        self.f[(k, n)] = {c: equilibrium(c, rb, uw) for c in DIRS}
                        rho[(k, n)] = rb
                        tot += rb
                    u[n] = uw
                    mom = scale(tot, uw)
                    acc[p]["Fc"] = sub(acc[p]["Fc"], mom)
                    acc[p]["Tc"] = sub(acc[p]["Tc"], cross(d, mom))
            # S3 Hertz contacts (repulsive, onset d0, capped below rcap)
            for p in range(len(self.parts)):
                for q in range(p + 1, len(self.parts)):
                    d = tuple(self.mi(self.parts[q]["x"][a] - self.parts[p]["x"][a], a)
                              for a in range(3))
                    r = dot(d, d).sqrt()
                    if r < self.hd0:
                        h = self.hd0 - max(r, self.hcap)
                        mag = D(5) / 2 * self.hK * h * h.sqrt()
                        e = scale(1 / r, d)
                        acc[p]["FH"] = sub(acc[p]["FH"], scale(mag, e))
                        acc[q]["FH"] = add(acc[q]["FH"], scale(mag, e))
            if self.walls:
                zlo, zhi = D("0.5"), D(self.L[2]) - D("1.5")
                for p, P in enumerate(self.parts):
                    for r, sgn in ((2 * (P["x"][2] - zlo), 1), (2 * (zhi - P["x"][2]), -1)):
                        if r < self.hd0:
                            h = self.hd0 - max(r, self.hcap)
                            mag = D(5) / 2 * self.hK * h * h.sqrt()
                            acc[p]["FH"] = add(acc[p]["FH"], (D(0), D(0), sgn * mag))
        fluid = [n for n in nodes if new[n] == 0]
        fluid_set = set(fluid)
        # S4 pseudo-potential with virtual solid densities, SC forces
        psi = {}
        for n in nodes:
            if new[n] == 0:
                for k in range(K):
                    psi[(k, n)] = rho[(k, n)]
            else:
                fl = [c for c in DIRS if c != (0, 0, 0) and self.nb(n, c) in fluid_set]
                if fl:
                    ws = sum((W[c] for c in fl), D(0))
                    for k in range(K):
                        psi[(k, n)] = (1 + self.zeta[k]) * sum(
                            (W[c] * rho[(k, self.nb(n, c))] for c in fl), D(0)) / ws
        a = {}
        for n in fluid:
            for k in range(K):
                s = ZERO3
                if K == 2:
                    for c in DIRS:
                        if c != (0, 0, 0):
                            s = add(s, scale(W[c] * psi[(1 - k, self.nb(n, c))], c))
                a[(k, n)] = add(scale(-self.G * self.s, s), self.g)
        if K == 2:
            for n in nodes:
                p = new[n] - 1
                if p < 0:
                    continue
                fl = [c for c in DIRS if c != (0, 0, 0) and self.nb(n, c) in fluid_set]
                if not fl:
                    continue
                Fs = ZERO3
                for k in range(2):
                    s = ZERO3
                    for c in fl:
                        s = add(s, scale(W[c] * rho[(1 - k, self.nb(n, c))], c))
                    Fs = add(Fs, scale(-self.G * self.s * psi[(k, n)], s))
                d = self.sep(n, self.parts[p]["x"])
                acc[p]["FSC"] = add(acc[p]["FSC"], Fs)
                acc[p]["TSC"] = add(acc[p]["TSC"], cross(d, Fs))
        # S5 collision
        post = {}
        for n in fluid:
            if K == 1:
                om = 1 / self.tau[0]
            else:
                rt = rho[(0, n)] + rho[(1, n)]
                inv = sum(((rho[(k, n)] / rt) / (CS2 * (self.tau[k] - D("0.5"))) for k in range(2)),
                          D(0))
                om = 2 * CS2 / (2 / inv + CS2)
            for k in range(K):
                r = rho[(k, n)]
                ushift = add(u[n], a[(k, n)])
                post[(k, n)] = {c: equilibrium(c, r, ushift)
                                + (1 - om) * (self.f[(k, n)][c] - equilibrium(c, r, u[n]))
                                for c in DIRS}
        # S6 links
        refl = {}
        for n in fluid:
            for c in DIRS:
                s_ = self.nb(n, c)
                o = new[s_]
                if c == (0, 0, 0) or o == 0:
                    continue
                rw_abs = tuple(D(n[a]) + D(c[a]) / 2 for a in range(3))
                if o < 0:
                    uw = self.ulo if s_[2] == 0 else self.uhi
                    rw = None
                else:
                    P = self.parts[o - 1]
                    rw = tuple(self.mi(rw_abs[a] - P["x"][a], a) for a in range(3))
                    uw = add(P["v"], cross(P["w"], rw))
                Fl = ZERO3
                back = tuple(-a for a in c)
                for k in range(K):
                    corr = 2 * W[c] * rho[(k, n)] * dot(uw, c) / CS2
                    fs = post[(k, n)][c]
                    refl[(k, n, back)] = fs - corr
                    Fl = add(Fl, scale(2 * fs - corr, c))
                if rw is not None:
                    p = o - 1
                    acc[p]["Fl"] = add(acc[p]["Fl"], Fl)
                    acc[p]["Tl"] = add(acc[p]["Tl"], cross(rw, Fl))
        # S7 particles
        report = []
        for p, P in enumerate(self.parts):
            A = acc[p]
            report.append(A)
            if not P["have_prev"]:
                P["Fprev"], P["Tprev"] = A["Fl"], A["Tl"]
            F = add(scale(D("0.5"), add(P["Fprev"], A["Fl"])),
                    add(add(A["Fd"], A["Fc"]), add(A["FH"], A["FSC"])))
            T = add(scale(D("0.5"), add(P["Tprev"], A["Tl"])), add(add(A["Td"], A["Tc"]), A["TSC"]))
            P["v"] = add(P["v"], scale(1 / self.mass, F))
            P["x"] = tuple(wrap(P["x"][k] + P["v"][k], self.L[k]) for k in range(3))
            if self.rotate:
                P["w"] = add(P["w"], scale(1 / self.inertia, T))
                P["q"] = self.rotate_q(P["q"], P["w"])
            P["Fprev"], P["Tprev"], P["have_prev"] = A["Fl"], A["Tl"], True
        # S8 pull streaming on the new map
        fnew = {}
        for n in fluid:
            for k in range(K):
                fnew[(k, n)] = {}
                for c in DIRS:
                    src = self.nb(n, c, -1)
                    fnew[(k, n)][c] = post[(k, src)][c] if new[src] == 0 else refl[(k, n, c)]
        self.f = fnew
        self.own = new
        return report

    @staticmethod
    def qdot(q, w):
        q0, q1, q2, q3 = q
        R = [[q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3, 2 * (q1 * q2 - q0 * q3), 2 * (q1 * q3 + q0 * q2)],
             [2 * (q1 * q2 + q0 * q3), q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3, 2 * (q2 * q3 - q0 * q1)],
             [2 * (q1 * q3 - q0 * q2), 2 * (q2 * q3 + q0 * q1), q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3]]
        wb = [R[0][a] * w[0] + R[1][a] * w[1] + R[2][a] * w[2] for a in range(3)]
        # q (x) (0, w_body), Hamilton product
        s = -(q1 * wb[0] + q2 * wb[1] + q3 * wb[2])
        v = add(scale(q0, tuple(wb)), cross((q1, q2, q3), tuple(wb)))
        return (s / 2, v[0] / 2, v[1] / 2, v[2] / 2)

    def rotate_q(self, q, w):
        qd = self.qdot(q, w)
        for _ in range(50):
            qh = tuple(q[c] + qd[c] / 2 for c in range(4))
            qn = self.qdot(qh, w)
            diff = max(abs(qn[c] - qd[c]) for c in range(4))
            qd = qn
            if diff <= D("1e-14"):
                break
        out = tuple(q[c] + qd[c] for c in range(4))
        nrm = sum((a * a for a in out), D(0)).sqrt()
        return tuple(a / nrm for a in out)

    # views ------------------------------------------------------------------
    def populations(self, dirs_order):
        """float array [K][19][N] in the given direction order (0 on solids)."""
        import numpy as np
        out = np.zeros((self.K, 19, len(self.nodes)))
        for idx, n in enumerate(self.nodes):
            if (0, n) not in self.f:
                continue
            for k in range(self.K):
                for i, c in enumerate(dirs_order):
                    out[k, i, idx] = float(self.f[(k, n)][tuple(int(a) for a in c)])
        return out
