"""Mutation check of the oracle's pins: copies of the oracle source, each
with one plausible mistake planted (a dropped term, a wrong sign, index or
coefficient, a step in the wrong order), are built on the CPU and loaded in
place of the oracle; for every copy some pin must fail.  The pins run in a
child process that loads the mutated library through ORACLE_LIB."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "nbody_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_symplectic.py",
        "tests/test_oracle_field.py", "tests/test_golden.py"]

# (what is wrong, original text, mutated text); each original occurs once
MUTANTS = [
    ("jerk coefficient 2 instead of 3",
     "const double alpha = 3.0 * rv * rinv2;", "const double alpha = 2.0 * rv * rinv2;"),
    ("jerk sign", "nsum_add(&sj[0], mr3 * (wx - alpha * rx));",
     "nsum_add(&sj[0], mr3 * (wx + alpha * rx));"),
    ("softening dropped", "const double s = rx * rx + ry * ry + rz * rz + eps2;",
     "const double s = rx * rx + ry * ry + rz * rz;"),
    ("r^-2 instead of r^-3", "const double mr3 = m[j] * rinv * rinv2;",
     "const double mr3 = m[j] * rinv2;"),
    ("y difference against the wrong axis", "const double ry = x[3 * j + 1] - xi[1];",
     "const double ry = x[3 * j + 1] - xi[0];"),
    ("self slot not skipped", "    if (j == self) continue;\n", "\n"),
    ("potential falls as 1/r^2", "nsum_add(&sp, -m[j] * rinv);", "nsum_add(&sp, -m[j] * rinv2);"),
    ("pair potential halved", "for (int64_t i = 0; i < n; ++i) nsum_add(&w, wi[i]);",
     "for (int64_t i = 0; i < n; ++i) nsum_add(&w, 0.5 * wi[i]);"),
    ("angular momentum z sign", "nsum_add(&L[2], m[i] * (xi[0] * vi[1] - xi[1] * vi[0]));",
     "nsum_add(&L[2], m[i] * (xi[1] * vi[0] - xi[0] * vi[1]));"),
    ("predictor drops the jerk's 1/2", "vp[c] = v[c] + dt * (a[c] + dt * (0.5 * j[c]));",
     "vp[c] = v[c] + dt * (a[c] + dt * (j[c]));"),
    ("corrector jerks swapped", "h * (4.0 * j0[c] + 2.0 * j1[c])", "h * (2.0 * j0[c] + 4.0 * j1[c])"),
    ("corrector 1/12 for 1/24", "x1[c] = xp[c] + a2 * (h2 * h2 / 24.0)",
     "x1[c] = xp[c] + a2 * (h2 * h2 / 12.0)"),
    ("Aarseth numerator |j| for |j|^2", "const double num = na * n2 + nj * nj;",
     "const double num = na * n2 + nj;"),
    ("doubling ignores commensurability", "if (t_tick % two_dt_ticks == 0) --level;", "--level;"),
    ("initial step |j|/|a|", "eta_s * na / nj;", "eta_s * nj / na;"),
    ("sixth-order weight sign", "const double w1 = -1.17767998417887;",
     "const double w1 = 1.17767998417887;"),
    ("leapfrog drift before the first half kick",
     "      for (int64_t q = 0; q < 3 * n; ++q) v[q] += 0.5 * c * a[q];\n"
     "      for (int64_t q = 0; q < 3 * n; ++q) x[q] += c * v[q];",
     "      for (int64_t q = 0; q < 3 * n; ++q) x[q] += c * v[q];\n"
     "      for (int64_t q = 0; q < 3 * n; ++q) v[q] += 0.5 * c * a[q];"),
    ("bulge jerk coefficient", "sph_add(g, -3.0 * g / d2, x, v, acc, jerk);",
     "sph_add(g, -2.0 * g / d2, x, v, acc, jerk);"),
    ("disk radial scale on z instead of zeta", "const double u = f->disk_a + zeta;",
     "const double u = f->disk_a + z;"),
    ("disk jerk drops the b^2 term",
     "v[2] * (u * b * b / (zeta * zeta * zeta) + z * z / (zeta * zeta))",
     "v[2] * (z * z / (zeta * zeta))"),
    ("halo enclosed mass one power short", "Mr = Mh * s * sg / (1.0 + sg);",
     "Mr = Mh * sg / (1.0 + sg);"),
    ("halo potential exterior constant", "phi -= Mc / r;", "phi -= Mc / f->halo_rc;"),
    ("field taken at the old position in block steps",
     "    add_field(p->field, na, act, xp, vp, a1, j1);",
     "    add_field(p->field, na, act, x, v, a1, j1);"),
    ("field energy halved", "    nsum_add(&we, m[i] * phi);", "    nsum_add(&we, 0.5 * m[i] * phi);"),
]


def _run_pins(source: str, tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    c = tmp_path / "copy.c"
    c.write_text(source)
    lib = oracle_build.build(src=str(c), out=str(tmp_path / "libcopy.so"))
    env = dict(os.environ, ORACLE_LIB=lib)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           *PINS], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=600)


def test_unmodified_copy_passes(tmp_path):
    # the harness itself: the same source built and loaded the same way
    r = _run_pins(open(SRC).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("what,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(what, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found once: {what}"
    r = _run_pins(src.replace(old, new), tmp_path)
    # 1: a pin failed; negative: the mutant crashed the process
    assert r.returncode == 1 or r.returncode < 0, f"no pin caught: {what}\n{r.stdout[-2000:]}"
