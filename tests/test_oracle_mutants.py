"""The pins catch plausible mistakes in the oracle.

Each case writes a copy of ``oracle/sweep_oracle.c`` with one planted
mistake (the substitutions listed in ``tests/oracle_mutants.py``; the oracle
source itself holds none), builds it with gcc, and runs the oracle pin tests
against it in a subprocess (``ORACLE_LIB`` selects the build).  Every planted
mistake must make at least one pin fail; the same harness on the unmodified
source must pass.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

from oracle import build as obuild
from tests.oracle_mutants import MUTANTS, mutate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_bspline.py", "tests/test_oracle_frame.py", "tests/test_oracle_grad.py",
             "tests/test_oracle_rational.py", "tests/test_oracle_frenet_laws.py",
             "tests/test_oracle_arclength_mesh.py", "tests/test_oracle_kappa.py"]
IDS = sorted(MUTANTS)


def _run_pins(lib_path: str) -> subprocess.CompletedProcess:
    env = dict(os.environ, ORACLE_LIB=lib_path, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_FILES],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")
    with open(obuild.SRC) as f:
        clean = f.read()

    def one(k):
        src = d / f"sweep_oracle_m{k}.c"
        src.write_text(clean if k == 0 else mutate(clean, k))
        lib = obuild.build(out=str(d / f"liboracle_m{k}.so"), src=str(src))
        return k, _run_pins(lib)

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        return dict(ex.map(one, [0] + IDS))


def test_oracle_source_holds_no_planted_mistake():
    with open(obuild.SRC) as f:
        clean = f.read()
    for k, (_, original, mutated) in MUTANTS.items():
        assert clean.count(original) == 1, k
        assert mutated not in clean, k


def test_unmodified_build_passes_the_pins(results):
    r = results[0]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("k", IDS)
def test_planted_mistake_is_caught(results, k):
    r = results[k]
    assert r.returncode != 0, f"mistake {k} ({MUTANTS[k][0]}) passed every pin:\n{r.stdout[-1500:]}"
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    print(f"mistake {k}: caught by {failed[:1]}")
