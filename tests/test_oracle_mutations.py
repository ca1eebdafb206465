"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle.c (a dropped term, a wrong
sign or constant, a transposed index, a wrong comparison), builds it with gcc
and runs the CPU pin suite against it in a subprocess; the suite must fail.
The cases are independent, so their subprocesses run side by side (one per
CPU, at most 8); each case is still its own test.  Nothing here touches the
GPU.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "drop_self_image_quadratic": ("+ 0.5 * dWd);", "+ 0.0 * dWd);"),
    "dipole_tensor_sign": ("D[0] = (1.0 - 3.0 * rx * rx / r2) / r3;", "D[0] = (1.0 + 3.0 * rx * rx / r2) / r3;"),
    "transposed_separation": ("long rho = imod(yi - yj, L) * L + imod(xi - xj, L);",
                              "long rho = imod(xi - xj, L) * L + imod(yi - yj, L);"),
    "weyl_constant": ("k0 += 0x9E3779B9u;", "k0 += 0x9E3779B8u;"),
    "philox_word_swap": ("uint32_t y1 = lo1;", "uint32_t y1 = lo0;"),
    "metropolis_direction": ("return u < exp(-dE / T);", "return u > exp(-dE / T);"),
    "exchange_sign_in_dE": ("double dex = -p->J *", "double dex = p->J *"),
    "quartic_anisotropy_sign": ("- p->K4 * (z1 * z1 * z1 * z1 - z0 * z0 * z0 * z0);",
                                "+ p->K4 * (z1 * z1 * z1 * z1 - z0 * z0 * z0 * z0);"),
    "box_edge_weight": ("if (twice == edge) return 0.5;", "if (twice == edge) return 1.0;"),
    "incremental_field_sign": ("h[2 * N + m] += Wzz[rho] * d[2];", "h[2 * N + m] -= Wzz[rho] * d[2];"),
    "vertical_walls_along_x": ("nv += 1 - sgn(s[c * N + i]) * sgn(s[c * N + iy]);",
                               "nv += 1 - sgn(s[c * N + i]) * sgn(s[c * N + ix]);"),
    "cone_angle_offset": ("double dth = acos(z) - 0.5 * PI;", "double dth = acos(z) - 0.25 * PI;"),
    "direction_axes": ("S[0] = rxy * cos(phi);\n    S[1] = rxy * sin(phi);",
                       "S[0] = rxy * sin(phi);\n    S[1] = rxy * cos(phi);"),
    "all_images_self_term_dropped": ("xx -= self;", "xx -= 0.0 * self;"),
    "all_images_reciprocal_sign": ("xx += f * kx * kx;", "xx -= f * kx * kx;"),
    "all_images_gaussian_term": ("+ 3.0 * gs / r2 + 2.0 * a * a * gs;", "+ 3.0 * gs / r2 + 1.0 * a * a * gs;"),
    "coset_membership_axes": ("if ((int)(k % L) % l != cx || (int)(k / L) % l != cy) continue;",
                              "if ((int)(k % L) % l != cy || (int)(k / L) % l != cx) continue;"),
    "coset_error_partner_weight": ("eps += 2.0 / (r2 * sqrt(r2));", "eps += 1.0 / (r2 * sqrt(r2));"),
    "ising_trial_not_reversed": ("S[0] = -s[k]; S[1] = -s[N + k]; S[2] = -s[2 * N + k];",
                                 "S[0] = -s[k]; S[1] = -s[N + k]; S[2] = s[2 * N + k];"),
    "stripe_axis": ("mh += ((i / L) % 2 == 0) ? z : -z;", "mh += ((i % L) % 2 == 0) ? z : -z;"),
    "exchange_rule_sign": ("const double delta = (1.0 / p[r].T - 1.0 / p[r + 1].T) * (E[r] - E[r + 1]);",
                           "const double delta = (1.0 / p[r].T - 1.0 / p[r + 1].T) * (E[r + 1] - E[r]);"),
    "variance_without_mean": ("const double d = obs[k * ORC_NOBS + slot[q]] - mean;",
                              "const double d = obs[k * ORC_NOBS + slot[q]] - 0.0 * mean;"),
    "state_cone_angle_scale": ("eta_state += sqrt((2.0 / PI) * (2.0 / PI) * dth * dth);",
                               "eta_state += sqrt((2.0 / PI) * dth * dth);"),
    "susceptibility_square_of_mean": ("return (double)L * (double)L / T * (m2 - m1 * m1);",
                                      "return (double)L * (double)L / T * (m2 - m1);"),
    "checkerboard_moves_applied_late": ("if ((int)((x + y) % 2) != color) continue;\n                if (!orc_metropolis_accept",
                                        "if ((int)((x + y) % 2) == color) continue;\n                if (!orc_metropolis_accept"),
}


def _run_pins(text):
    """Build `text` as the oracle and run the CPU pin suite against it."""
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "oracle.c")
        open(src, "w").write(text)
        so = os.path.join(td, "liboracle_mut.so")
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-I", os.path.join(ROOT, "oracle"), "-o", so, src, "-lm"])
        env = dict(os.environ, ORACLE_LIB=so)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_rng.py"),
                            os.path.join(ROOT, "tests", "test_oracle_model.py"),
                            os.path.join(ROOT, "tests", "test_oracle_sampler.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r


CONTROL = "__unmodified__"


@pytest.fixture(scope="module")
def pin_runs():
    """Every case's pin-suite run (the unmodified copy under CONTROL; None
    for a mutation whose anchor is not found exactly once)."""
    text = open(SRC).read()
    jobs = {CONTROL: text}
    for name, (old, new) in MUTATIONS.items():
        jobs[name] = text.replace(old, new) if text.count(old) == 1 else None
    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        futs = {k: ex.submit(_run_pins, v) for k, v in jobs.items() if v is not None}
        return {k: (futs[k].result() if k in futs else None) for k in jobs}


def test_control_copy_passes(pin_runs):
    """The unmodified source, built and loaded the same way, passes the pins."""
    r = pin_runs[CONTROL]
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, pin_runs):
    r = pin_runs[name]
    assert r is not None, "mutation anchor not found uniquely: %s" % name
    assert r.returncode != 0, "pins did not catch mutation %s:\n%s" % (name, r.stdout[-2000:])
