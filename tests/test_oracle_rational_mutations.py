"""The rational-function pins catch plausible mistakes in the oracle's own
construction: each case plants one mistake in a copy of oracle/rational.py
(on the CPU), and runs the oracle-only tests of tests/test_rational.py
against it from a scratch tree; at least one must fail.  The unchanged copy
passes them (control)."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rational.py")

MUTATIONS = [
    ("nodes not squared", "lower = sn ** 2 / cn ** 2", "lower = sn / cn"),
    ("elliptic argument over 2n", "sn, cn, _, _ = ellipj(np.arange(1, n + 1) * K / (2 * n + 1), m)",
     "sn, cn, _, _ = ellipj(np.arange(1, n + 1) * K / (2 * n), m)"),
    ("poles at the even nodes", "    p = c[0::2]\n    num = c[1::2]", "    p = c[1::2]\n    num = c[0::2]"),
    ("residues without the constant", "res[l] = D * (num[-1] - p[l])", "res[l] = (num[-1] - p[l])"),
    ("shift applied with the wrong sign", "sigma=float(s))", "sigma=-float(s))"),
    ("rescaling by lmin instead of sqrt(lmin)", "    s = np.sqrt(lmin)\n    return D / s", "    s = lmin\n    return D / s"),
]


def run_pins(tmp_path, source):
    """Run the oracle-only rational tests against `source` as oracle/rational.py."""
    tree = tmp_path / "tree"
    (tree / "tests").mkdir(parents=True)
    shutil.copytree(os.path.join(ROOT, "oracle"), tree / "oracle", ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "synth"), tree / "synth", ignore=shutil.ignore_patterns("__pycache__"))
    for f in ("conftest.py", "test_rational.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), tree / "tests" / f)
    (tree / "oracle" / "rational.py").write_text(source)
    env = dict(os.environ, OMP_NUM_THREADS="4", HISQ_ORACLE_LIB=os.path.join(ROOT, "oracle", "_hisq_oracle.so"))
    return subprocess.run([sys.executable, "-m", "pytest", "tests/test_rational.py", "-q", "-p", "no:cacheprovider",
                           "-k", "test_oracle_ and not heatbath"], cwd=tree, env=env, capture_output=True, text=True,
                          timeout=600)


def test_unchanged_copy_passes(tmp_path):
    r = run_pins(tmp_path, open(SRC).read())
    assert r.returncode == 0, r.stdout[-2000:]
    assert " passed" in r.stdout


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, name
    r = run_pins(tmp_path, src.replace(old, new, 1))
    assert r.returncode == 1 and " failed" in r.stdout, f"no pin caught: {name}\n{r.stdout[-2000:]}"
