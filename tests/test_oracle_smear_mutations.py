"""The smearing pins catch plausible mistakes in the oracle's construction:
each case plants one mistake in a copy of oracle/smear.py (on the CPU) and
runs tests/test_oracle_smear.py against it from a scratch tree; at least one
pin must fail.  The unchanged copy passes them (control)."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "smear.py")

MUTATIONS = [
    ("upper transport without adjoint", "fwd = up @ _roll(dims, A, nu, dist) @ _dag(_roll(dims, up, mu, 1))",
     "fwd = up @ _roll(dims, A, nu, dist) @ _roll(dims, up, mu, 1)"),
    ("backward staple read at x", "down = _roll(dims, up, nu, -dist)", "down = up"),
    ("backward staple not shifted along mu", "bwd = _dag(down) @ _roll(dims, A, nu, -dist) @ _roll(dims, down, mu, 1)",
     "bwd = _dag(down) @ _roll(dims, A, nu, -dist) @ down"),
    ("Lepage coefficient of one smearing", "LEVEL2 = dict(c1=1.0, c3=1 / 16, c5=1 / 64, c7=1 / 384, cL=-1 / 8)",
     "LEVEL2 = dict(c1=1.0, c3=1 / 16, c5=1 / 64, c7=1 / 384, cL=-1 / 16)"),
    ("five-link path along one direction twice", "                if rho == nu:\n                    continue\n",
     ""),
    ("seven-link and five-link weights swapped", "LEVEL1 = dict(c1=1 / 8, c3=1 / 16, c5=1 / 64, c7=1 / 384, cL=0.0)",
     "LEVEL1 = dict(c1=1 / 8, c3=1 / 16, c5=1 / 384, c7=1 / 64, cL=0.0)"),
    ("projection with (V^+ V)^-1", "return V @ (E * (1.0 / np.sqrt(w))[..., None, :]) @ _dag(E)",
     "return V @ (E * (1.0 / w)[..., None, :]) @ _dag(E)"),
    ("Naik hop of two sites", "_roll(dims, W[:, mu], mu, 1) @ _roll(dims, W[:, mu], mu, 2)",
     "_roll(dims, W[:, mu], mu, 1) @ _roll(dims, W[:, mu], mu, 1)"),
    ("Naik boundary sign at t + 1", "sl[:, 3] *= np.where(c[:, 3] + 3 >= Lt, -1.0, 1.0)",
     "sl[:, 3] *= np.where(c[:, 3] + 1 >= Lt, -1.0, 1.0)"),
    ("Lepage two-step transport read once", "up = Tn @ _roll(dims, Tn, nu, 1)", "up = Tn @ Tn"),
]


def run_pins(tmp_path, source, stop_first=False):
    tree = tmp_path / "tree"
    (tree / "tests").mkdir(parents=True)
    shutil.copytree(os.path.join(ROOT, "oracle"), tree / "oracle", ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "synth"), tree / "synth", ignore=shutil.ignore_patterns("__pycache__"))
    for f in ("conftest.py", "test_oracle_smear.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), tree / "tests" / f)
    (tree / "oracle" / "smear.py").write_text(source)
    env = dict(os.environ, OMP_NUM_THREADS="4", HISQ_ORACLE_LIB=os.path.join(ROOT, "oracle", "_hisq_oracle.so"))
    # a mutant needs one failing pin: stop there
    return subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_smear.py", "-q", "-p",
                           "no:cacheprovider"] + (["-x"] if stop_first else []), cwd=tree, env=env,
                          capture_output=True, text=True, timeout=600)


def test_unchanged_copy_passes(tmp_path):
    r = run_pins(tmp_path, open(SRC).read())
    assert r.returncode == 0, r.stdout[-2000:]
    assert " passed" in r.stdout


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, name
    r = run_pins(tmp_path, src.replace(old, new, 1), stop_first=True)
    assert r.returncode == 1 and " failed" in r.stdout, f"no pin caught: {name}\n{r.stdout[-2000:]}"
