"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of ``oracle/oracle.c`` -- a sign, a
coefficient, a dropped factor, an off-by-one, a wrong knot offset or
coefficient placement, a transposed operand or index, a clipped support or
pixel box -- builds it with the oracle's own compiler flags into a
temporary directory and runs the oracle's pin modules against it in a
subprocess: at least one pin must fail.  An unmodified copy built the same
way must pass them all, so a broken harness cannot make the mutants look
caught.  The oracle itself is never modified.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = [os.path.join(ROOT, "tests", f) for f in
        ("test_oracle_bspline.py", "test_oracle_footprint.py", "test_oracle_operator.py")]

# (name, exact text in oracle.c, replacement): each is a one-token mistake
MUTATIONS = [
    ("cubic B-spline sign", "if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;",
     "if (a < 1.0) return 2.0 / 3.0 - a * a - 0.5 * a * a * a;"),
    ("quadratic B-spline coefficient", "if (a < 0.5) return 0.75 - a * a;",
     "if (a < 0.5) return 0.75 - 0.5 * a * a;"),
    ("Gauss-Legendre weight drops a factor", "weights[m - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);",
     "weights[m - 1 - i] = 2.0 / ((1.0 - x * x) * dp);"),
    ("footprint segment without its half-length", "ks_add(&acc, half * s);", "ks_add(&acc, s);"),
    ("footprint misses the last interior knot", "        for (int j = 1; j <= n; ++j) {\n            double t = (-h + j - x[i]) / w[i];",
     "        for (int j = 1; j < n; ++j) {\n            double t = (-h + j - x[i]) / w[i];"),
    ("footprint chord with the offset's sign flipped", "double ta = (-h - x[i]) / w[i], tb = (h - x[i]) / w[i];",
     "double ta = (-h + x[i]) / w[i], tb = (h + x[i]) / w[i];"),
    ("knot planes of even degree at integers", "double kap = (n & 1) ? 0.0 : 0.5;   /* knot planes sit at o + kap + integer */",
     "double kap = 0.0;   /* knot planes sit at o + kap + integer */"),
    ("coefficient placement off by half a step", "        o[i] = -0.5 * (double)(N[i] - 1);\n        lo[i] = o[i] - h;",
     "        o[i] = -0.5 * (double)N[i];\n        lo[i] = o[i] - h;"),
    ("pixel centre with rows and columns transposed",
     "double ci = (double)i - 0.5 * (g->C - 1), cj = (double)j - 0.5 * (g->R - 1);",
     "double ci = (double)i - 0.5 * (g->R - 1), cj = (double)j - 0.5 * (g->C - 1);"),
    ("adjoint coefficient index transposed", "int64_t q1 = q % N[0], q2 = (q / N[0]) % N[1], q3 = q / (N[0] * N[1]);",
     "int64_t q3 = q % N[0], q2 = (q / N[0]) % N[1], q1 = q / (N[0] * N[1]);"),
    # (floor + 1 would still be the tight bound ceil for a non-integer edge;
    # floor + 2 drops the first column whose centre can lie in the shadow)
    ("adjoint pixel box clipped", "*i0 = (int64_t)floor(umin + ci) - 1;", "*i0 = (int64_t)floor(umin + ci) + 2;"),
]


def _run_pins(tmpdir, name, text):
    d = os.path.join(tmpdir, name.replace(" ", "_").replace("'", ""))
    os.makedirs(d, exist_ok=True)
    src = os.path.join(d, "oracle.c")
    with open(src, "w") as fh:
        fh.write(text)
    env = dict(os.environ, ORACLE_SRC=src, ORACLE_LIB=os.path.join(d, "liboracle.so"), OMP_NUM_THREADS="2")
    # the wrapper builds the copy on first use with the oracle's own flags
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-800:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed to build the oracle copies")
def test_every_planted_mistake_fails_a_pin(tmp_path):
    original = open(SRC).read()
    jobs = [("unmodified", original)]
    for name, old, new in MUTATIONS:
        assert original.count(old) >= 1, f"mutation target not found: {name}"
        jobs.append((name, original.replace(old, new, 1)))
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda j: (j[0],) + _run_pins(str(tmp_path), *j), jobs))
    control = results[0]
    assert control[1] == 0, f"unmodified oracle copy fails its pins:\n{control[2]}"
    survivors = [name for name, rc, _ in results[1:] if rc == 0]
    assert not survivors, f"mistakes no pin catches: {survivors}"
