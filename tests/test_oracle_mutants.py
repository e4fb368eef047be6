"""The oracle's pins catch plausible mistakes (CPU only).

Each case copies the oracle's C source, plants one mistake of the kind a
reader could make (a wrong sign, a swapped function, an off-by-one
neighbour, a max where the paper takes a min), builds the copy, and runs
the pins of the affected function against it in a child process: the pins
must fail.  Nothing here touches the real oracle library.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "amy_oracle.c")

# (name, text in the source, replacement, pin tests that must fail)
MUTANTS = [
    ("adversary maximises", "if (qw < q) q = qw;", "if (qw > q || q == INFINITY) q = qw;",
     "tests/test_oracle_disturbance.py"),
    ("disturbance ignored after the first point", "for (int64_t w = 0; w < C->nw; ++w) {",
     "for (int64_t w = 0; w < 1; ++w) {", "tests/test_oracle_disturbance.py"),
    ("disturbance sign flipped", "d = d + D[i * p->p + l] * w[l];", "d = d - D[i * p->p + l] * w[l];",
     "tests/test_oracle_disturbance.py"),
    ("robot heading: sin and cos swapped", "mu[0] = x[0] + a * cos(u[1]);", "mu[0] = x[0] + a * sin(u[1]);",
     "tests/test_oracle_disturbance.py"),
    ("unicycle: sin and cos swapped", "mu[0] = x[0] + a * cos(x[2]);", "mu[0] = x[0] + a * sin(x[2]);",
     "tests/test_oracle_dynamics_pins.py"),
    ("room: right neighbour off by one", "right = x[(i + 1) % n];", "right = x[(i + 2) % n];",
     "tests/test_oracle_dynamics_pins.py"),
    ("room: heater exchange sign", "double g = ga * (Th - x[i]);", "double g = ga * (x[i] - Th);",
     "tests/test_oracle_dynamics_pins.py"),
    ("vehicle: slow branch heading", "f1 = x4 * cos(x5);", "f1 = x4 * sin(x5);",
     "tests/test_oracle_dynamics_pins.py"),
    ("normal mass: straddling branch", "return 0.5 * (erf(b * INV_SQRT2) - erf(a * INV_SQRT2));",
     "return 0.5 * (erf(b * INV_SQRT2) + erf(a * INV_SQRT2));", "tests/test_oracle_pins.py"),
    ("window: interval shrunk", "else keep = (centre(p, i, j) - mu[i] >= zl) && (centre(p, i, j) - mu[i] <= zh);",
     "else keep = (centre(p, i, j) - mu[i] >= 0.9 * zl) && (centre(p, i, j) - mu[i] <= 0.9 * zh);",
     "tests/test_oracle_pins.py"),
    ("uniform: support start taken from its end",
     "double fa = clampd((ta - p->na[i]) / w, 0.0, 1.0), fb = clampd((tb - p->na[i]) / w, 0.0, 1.0);",
     "double fa = clampd((ta - p->nb[i]) / w, 0.0, 1.0), fb = clampd((tb - p->nb[i]) / w, 0.0, 1.0);",
     "tests/test_oracle_noise.py"),
    ("exponential: rate read as a scale", "double sa = ta <= 0.0 ? 1.0 : exp(-p->na[i] * ta);",
     "double sa = ta <= 0.0 ? 1.0 : exp(-ta / p->na[i]);", "tests/test_oracle_noise.py"),
    ("exponential: cut not divided by the rate", "*zh = (p->cutoff > 0) ? log(p->na[i] / p->cutoff) / p->na[i] : INFINITY;",
     "*zh = (p->cutoff > 0) ? log(p->na[i] / p->cutoff) : INFINITY;", "tests/test_oracle_noise.py"),
    ("beta: shapes swapped",
     "return beta_mass((ta - p->na[i]) / w, (tb - p->na[i]) / w, p->nalpha[i], p->nbeta[i]);",
     "return beta_mass((ta - p->na[i]) / w, (tb - p->na[i]) / w, p->nbeta[i], p->nalpha[i]);",
     "tests/test_oracle_noise.py"),
    ("multiplicative: scale by the signed coordinate", "s = s * fabs(xi);", "s = s * xi;",
     "tests/test_oracle_noise.py"),
    ("intersect rule: centres tested instead", "if (intersect) keep = (edge(p, i, j + 1) - mu[i] > zl) && (edge(p, i, j) - mu[i] < zh);",
     "if (intersect) keep = (centre(p, i, j) - mu[i] >= zl) && (centre(p, i, j) - mu[i] <= zh);",
     "tests/test_oracle_noise.py"),
    ("reach: target mass dropped", "return safety ? q : q + t0;", "return q;", "tests/test_oracle_pins.py"),
    ("argmax: highest index on ties", "if (q > best) {", "if (q >= best) {", "tests/test_oracle_pins.py"),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_its_pins(tmp_path, name, old, new, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: anchor not found once in the oracle source"
    bad = tmp_path / "amy_oracle.c"
    bad.write_text(src.replace(old, new))
    (tmp_path / "amy_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "amy_oracle.h")).read())
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-o", str(lib), str(bad), "-lm"])
    env = dict(os.environ, AMY_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, pins)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"{name}: the pins in {pins} pass on an oracle with this mistake"
