"""The oracle's pins must fail on plausible mistakes.

Each case plants one mistake (a flipped sign, a swapped cross product, a
transposed rotation matrix, a dropped factor or term, a wrong component or
neighbour index) in a copy of the oracle source, builds it on the CPU into a
temporary directory, and runs the quick pin tests against it in a child
process through LBO_LIB. Every planted mistake must make a pin fail. The
cases cover the core step (S1-S8), the open faces and their extrapolation,
lubrication, Janus wetting, the physical momentum and, in the Python
domain-size module, the shell rounding and averaging. A control run of each
harness without a mistake must pass.
"""
import os
import shutil
import subprocess
import sys

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
    # open faces (Sec. 2.2, Eq. bbp, bbv) and the extrapolation to the face
    "pressure_face_quadratic_coefficient": (
        "(1.0 + uc * uc / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));",
        "(1.0 + uc * uc / (CS2 * CS2) - uu / (2.0 * CS2));"),
    "pressure_face_isotropic_term_dropped": (
        "(1.0 + uc * uc / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));",
        "(1.0 + uc * uc / (2.0 * CS2 * CS2));"),
    "face_velocity_extrapolation_sign": (
        "uw[a] = ok ? u[n * 3 + a] + 0.5 * (u[n * 3 + a] - u[inner * 3 + a]) : u[n * 3 + a];",
        "uw[a] = ok ? u[n * 3 + a] - 0.5 * (u[n * 3 + a] - u[inner * 3 + a]) : u[n * 3 + a];"),
    "face_density_extrapolation_sign": (
        "const T rw = ok ? rn + 0.5 * (rn - rho[int64_t(k) * N + inner]) : rn;",
        "const T rw = ok ? rn - 0.5 * (rn - rho[int64_t(k) * N + inner]) : rn;"),
    # lubrication (Eq. libric) and Janus wetting
    "lubrication_prefactor": (
        "const double fl = -6.0 * M_PI * P.lub_mu * 0.25 * P.radius * P.radius *",
        "const double fl = -6.0 * M_PI * P.lub_mu * 0.5 * P.radius * P.radius *"),
    "lubrication_relative_velocity_sign": (
        "vn += (parts[p].v[a] - parts[q].v[a]) * d[a] / r;",
        "vn += (parts[q].v[a] - parts[p].v[a]) * d[a] / r;"),
    "lubrication_along_the_wrong_axis": (
        "parts[p].FH[a] += fl * d[a] / r;",
        "parts[p].FH[a] += fl * d[(a + 1) % 3] / r;"),
    "janus_switch_sign": (
        "return k == 0 ? P.janus_zeta[0] * S : -P.janus_zeta[1] * S;",
        "return k == 0 ? -P.janus_zeta[0] * S : P.janus_zeta[1] * S;"),
    "janus_axis_from_a_row": (
        "2 * (q[1] * q[2] + q[0] * q[3]), 2 * (q[1] * q[3] - q[0] * q[2])};",
        "2 * (q[1] * q[2] - q[0] * q[3]), 2 * (q[1] * q[3] + q[0] * q[2])};"),
    # physical momentum (Sec. 2.3 after Eq. lbsbgk)
    "physical_momentum_full_force": (
        "ph[a].add(0.5 * (-(S->G * S->P.sc_norm) * rk * s[a] + rk * S->g[a]));",
        "ph[a].add(-(S->G * S->P.sc_norm) * rk * s[a] + rk * S->g[a]);"),
}

PIN_FILES = ["tests/test_oracle_lattice.py", "tests/test_oracle_fluid.py",
             "tests/test_oracle_particles.py", "tests/test_oracle_bruteforce.py",
             "tests/test_oracle_open.py", "tests/test_oracle_f1.py"]

# Mistakes in the domain-size measure (oracle/domain.py, Eq. Cluster_L_eq).
DOMAIN_MUTATIONS = {
    "shell_ties_rounded_down": (
        "down = (so > 0) & ((2 * so - 1) ** 2 * (A * A) > rhs)",
        "down = (so > 0) & ((2 * so - 1) ** 2 * (A * A) >= rhs)"),
    "shell_width_from_the_largest_side": (
        "return so.astype(np.int64), 2 * np.pi / Lmin, Lmin // 2",
        "return so.astype(np.int64), 2 * np.pi / max(shape), Lmin // 2"),
    "shell_mean_not_divided": (
        "mean = np.where(counts > 0, sums / np.maximum(counts, 1), 0.0)",
        "mean = np.where(counts > 0, sums, 0.0)"),
    "mean_not_removed": (
        "out[fluid] = phi[fluid] - phi[fluid].mean()",
        "out[fluid] = phi[fluid]"),
}


def _run_pins(tmp_path, name):
    """Build a copy of the oracle source carrying mutation `name` (None:
    unchanged) and run the pin files against it; returns the exit code."""
    src = open(SRC).read()
    if name is not None:
        a, b = MUTATIONS[name]
        assert src.count(a) == 1, "mutation anchor not found: the oracle source changed"
        src = src.replace(a, b)
    tag = name or "control"
    cpp = tmp_path / f"{tag}.cpp"
    cpp.write_text(src)
    so = tmp_path / f"{tag}.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                    "-I" + os.path.join(ROOT, "oracle"), "-o", str(so), str(cpp)], check=True)
    env = dict(os.environ, LBO_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow",
                        "-p", "no:cacheprovider"] + PIN_FILES,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout


@pytest.mark.slow
def test_harness_passes_without_a_mistake(tmp_path):
    """Control: the copied, rebuilt oracle passes every pin file."""
    rc, out = _run_pins(tmp_path, None)
    assert rc == 0, out[-2000:]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    rc, out = _run_pins(tmp_path, name)
    assert rc != 0, f"planted mistake {name} passed every pin:\n{out[-2000:]}"


def _run_domain_pins(tmp_path, name):
    """Run the domain pins against a copy of the oracle package whose
    domain.py carries mutation `name` (None: unchanged); returns the exit code."""
    src_dir = os.path.join(ROOT, "oracle")
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "domain.py"):
        shutil.copy(os.path.join(src_dir, f), pkg / f)
    (tmp_path / "tests").mkdir()
    for f in ("conftest.py", "test_oracle_domain.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), tmp_path / "tests" / f)
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp_path / "pytest.ini")
    if name is not None:
        text = (pkg / "domain.py").read_text()
        a, b = DOMAIN_MUTATIONS[name]
        assert text.count(a) == 1, "mutation anchor not found: the domain module changed"
        (pkg / "domain.py").write_text(text.replace(a, b))
    env = dict(os.environ, LBO_LIB=os.path.join(src_dir, "liblbo.so"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle_domain.py"],
                       cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout


@pytest.mark.slow
def test_domain_harness_passes_without_a_mistake(tmp_path):
    """Control: the copied package and pin file pass as they are, so a failure
    under a mutation comes from the mutation."""
    rc, out = _run_domain_pins(tmp_path, None)
    assert rc == 0, out[-2000:]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(DOMAIN_MUTATIONS))
def test_planted_domain_mistake_is_caught(name, tmp_path):
    """The domain-size module is Python: the mutated copy goes into a copy of
    the oracle package next to a copy of its pin file, run from there."""
    rc, out = _run_domain_pins(tmp_path, name)
    assert rc != 0, f"planted mistake {name} passed every pin:\n{out[-2000:]}"
