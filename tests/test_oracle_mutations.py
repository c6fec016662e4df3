"""The oracle's pins catch plausible mistakes: each case plants one mistake in
a copy of the C oracle (on the CPU), builds it, and runs the pin tests of
tests/test_oracle_pins.py against it; at least one pin must fail.  The
unchanged oracle passes the same pins in the ordinary run of the suite."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hisq_oracle.c")

# (name, text replaced, replacement[, function]): the first occurrence in the
# file (the operator helpers, then oracle_dslash), or the first one after the
# named function's definition
MUTATIONS = [
    ("backward hop sign", "add_mdag_v(acc, link_at(F, b1, mu), in + b1 * 3, -1.0);",
     "add_mdag_v(acc, link_at(F, b1, mu), in + b1 * 3, +1.0);"),
    ("backward link read at the output site", "add_mdag_v(acc, link_at(F, b1, mu), in + b1 * 3, -1.0);",
     "add_mdag_v(acc, link_at(F, s, mu), in + b1 * 3, -1.0);"),
    ("Naik hop of two sites", "long f3 = neighbour(L, s, mu, +3), b3 = neighbour(L, s, mu, -3);",
     "long f3 = neighbour(L, s, mu, +2), b3 = neighbour(L, s, mu, -2);"),
    ("backward Naik term dropped", "add_mdag_v(acc, link_at(N, b3, mu), in + b3 * 3, -1.0);", ""),
    ("adjoint without conjugation", "t += conj(M[b * 3 + a]) * v[b];", "t += M[b * 3 + a] * v[b];"),
    ("transposed link in the forward hop", "for (int b = 0; b < 3; ++b) t += M[a * 3 + b] * v[b];",
     "for (int b = 0; b < 3; ++b) t += M[b * 3 + a] * v[b];"),
    ("mass term 2 m^2", "const double diag = 4.0 * mass * mass + sigma;",
     "const double diag = 2.0 * mass * mass + sigma;"),
    ("staggered phase of the wrong direction", "for (int nu = 0; nu < mu; ++nu) e += c[nu];",
     "for (int nu = 0; nu <= mu; ++nu) e += c[nu];"),
    # the sampled-site evaluation that judges the full-size GPU parity
    ("sites: backward Naik link read at the output site", "add_mdag_v(acc, link_at(N, b3, mu), in + b3 * 3, -1.0);",
     "add_mdag_v(acc, link_at(N, s, mu), in + b3 * 3, -1.0);", "oracle_dslash_sites"),
    ("sites: forward fat hop of three sites", "add_mv(acc, link_at(F, s, mu), in + f1 * 3, +1.0);",
     "add_mv(acc, link_at(F, s, mu), in + f3 * 3, +1.0);", "oracle_dslash_sites"),
    ("sites: backward fat term dropped", "add_mdag_v(acc, link_at(F, b1, mu), in + b1 * 3, -1.0);", "",
     "oracle_dslash_sites"),
]


def mutate(src, old, new, function=None):
    """src with the first `old` (after the definition of `function`) replaced by `new`."""
    start = src.index(f"void {function}(") if function else 0
    at = src.index(old, start)
    return src[:at] + new + src[at + len(old):]


def run_pins(tmp_path, source):
    """Build `source` as the oracle library and run the pin tests against it."""
    mutant = tmp_path / "mutant.c"
    mutant.write_text(source)
    lib = tmp_path / "mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-w", "-o", str(lib), str(mutant),
                    "-lm"], check=True, capture_output=True)
    env = dict(os.environ, HISQ_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    return subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-x",
                           "-q", "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=600)


def test_unchanged_copy_passes(tmp_path):
    """Control: the harness itself (a copy built the same way) passes every pin."""
    r = run_pins(tmp_path, open(SRC).read())
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("mut", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, mut):
    name, old, new = mut[:3]
    src = open(SRC).read()
    r = run_pins(tmp_path, mutate(src, old, new, *mut[3:]))
    # a failed pin, not a crash or an import error
    assert r.returncode == 1 and " failed" in r.stdout, f"no pin caught: {name}\n{r.stdout[-2000:]}"
