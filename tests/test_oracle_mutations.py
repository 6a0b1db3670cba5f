"""The oracle's pins must fail on plausible mistakes.

Each case plants one mistake (a flipped sign, a swapped cross product, a
transposed rotation matrix, a dropped factor or term, a wrong component or
neighbour index) in a copy of the oracle source, builds it on the CPU into a
temporary directory, and runs the quick pin tests against it in a child
process through LBO_LIB. Every planted mistake must make a pin fail.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbo.cpp")

MUTATIONS = {
    "sc_sign": ("T sc = -(G * P.sc_norm) * s[a];", "T sc = (G * P.sc_norm) * s[a];"),
    "relaxation_dropped": ("feq<T>(i, rk, us) + (1.0 - we) * (F(k, i, n) - feq<T>(i, rk, un));",
                           "feq<T>(i, rk, us) + (F(k, i, n) - feq<T>(i, rk, un));"),
    "surface_velocity_cross": ("cross(pp->w, rw, uw);", "cross(rw, pp->w, uw);"),
    "link_torque_cross": ("cross(rw, Fv, tq);", "cross(Fv, rw, tq);"),
    "hertz_sign": ("parts[p].FH[a] -= mag * d[a] / r;", "parts[p].FH[a] += mag * d[a] / r;"),
    "rotation_not_transposed": (
        "ws[a] = Rm[0][a] * w[0] + Rm[1][a] * w[1] + Rm[2][a] * w[2];",
        "ws[a] = Rm[a][0] * w[0] + Rm[a][1] * w[1] + Rm[a][2] * w[2];"),
    "streaming_direction": ("int64_t src = nb[n * Q + opposite(i)];", "int64_t src = nb[n * Q + i];"),
    "half_step_average_dropped": ("sf.add(0.5 * (pp.Fprev[a] + Fl[a]));", "sf.add(Fl[a]);"),
    "moving_wall_factor": ("T corr = 2.0 * WT[i] * rho[int64_t(k) * N + n] * ucw / CS2;",
                           "T corr = WT[i] * rho[int64_t(k) * N + n] * ucw / CS2;"),
    "wetting_prefactor_dropped": ("rt[int64_t(k) * N + n] = (1.0 + zeta_at(M, n, k)) * s / wsum;",
                                  "rt[int64_t(k) * N + n] = s / wsum;"),
    "creation_momentum_sign": ("pp.Fc[a].add(-Pm[a]);", "pp.Fc[a].add(Pm[a]);"),
    "destruction_torque_cross": ("cross(d, J, tq);", "cross(J, d, tq);"),
    "solid_force_component": (
        "s[a] += WT[i] * val(rho[int64_t(kb) * N + m]) * CV[i][a];",
        "s[a] += WT[i] * val(rho[int64_t(k) * N + m]) * CV[i][a];"),
    "fluid_force_component": ("T r = rt[int64_t(kb) * N + nb[n * Q + i]] * WT[i];",
                              "T r = rt[int64_t(k) * N + nb[n * Q + i]] * WT[i];"),
    "mixture_velocity_weights": ("num[a] += jj[a] / P.tau[k];", "num[a] += jj[a];"),
    "wall_sides_swapped": ("const int face = cz(s) == 0 ? 0 : 1;",
                           "const int face = cz(s) == 0 ? 1 : 0;"),
    "equilibrium_quadrupole": ("return rho * WT[i] * (1.0 + dip + quad * 0.5);",
                               "return rho * WT[i] * (1.0 + dip + quad);"),
    "created_node_neighbours": (
        "if (own[m] == 0 && own_new[m] == 0) s += rho[int64_t(k) * N + m] * WT[i];",
        "if (own_new[m] == 0) s += rho[int64_t(k) * N + m] * WT[i];"),
}

PIN_FILES = ["tests/test_oracle_lattice.py", "tests/test_oracle_fluid.py",
             "tests/test_oracle_particles.py", "tests/test_oracle_bruteforce.py"]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(SRC).read()
    a, b = MUTATIONS[name]
    assert src.count(a) == 1, "mutation anchor not found: the oracle source changed"
    cpp = tmp_path / f"{name}.cpp"
    cpp.write_text(src.replace(a, b))
    so = tmp_path / f"{name}.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                    "-I" + os.path.join(ROOT, "oracle"), "-o", str(so), str(cpp)], check=True)
    env = dict(os.environ, LBO_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow",
                        "-p", "no:cacheprovider"] + PIN_FILES,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
