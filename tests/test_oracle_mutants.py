"""The pins catch plausible mistakes in the oracle.

Each case builds ``sweep_oracle.c`` with one planted mistake
(``-DOR_MUTANT=k``; the switch is compiled out of the normal build) and runs
the oracle pin tests against it in a subprocess (``ORACLE_LIB`` selects the
build).  Every planted mistake must make at least one pin fail; the same
harness on the unmodified source must pass.  Mistakes planted:

  1  Cox-de Boor: wrong factor (u - U_{k+1}) in the right-hand term
  2  basis derivative: the factor q dropped
  3  sample parameter i/n_s instead of i/(n_s - 1)
  4  periodic wrap off by one control point
  5  double reflection: second reflection skipped
  6  double reflection: chord x_{i+1} + x_i instead of the difference
  7  axis rule: argmax instead of argmin
  8  surface: sign of the S_x a term in X_u
  9  normal: X_u x X_v (orientation flipped)
 10  rational C'': the Leibniz factor 2 dropped
 11  surface: the S_z t' term of X_u dropped
 12  clamped knots k/(n-p+1)
 13  frame: s = r x t (left-handed)
 14  finite differences divided by h instead of 2h
 15  frame derivative: sign of the omega term in r'
 16  twist law: sign of sigma theta' in the derivative of the profile point
 17  Frenet torsion rate doubled
 18  arc-length targets i/n_s instead of i/(n_s - 1)
 19  first triangle of each quad wound clockwise
 20  normal term of the loss: the cross product not normalised
 21  adaptive sampling density: lam |C' x C''| / |C'|^3 (kappa without |C'|)
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_bspline.py", "tests/test_oracle_frame.py", "tests/test_oracle_grad.py",
             "tests/test_oracle_rational.py", "tests/test_oracle_frenet_laws.py",
             "tests/test_oracle_arclength_mesh.py"]
MUTANTS = list(range(1, 22))


def _run_pins(lib_path: str) -> subprocess.CompletedProcess:
    env = dict(os.environ, ORACLE_LIB=lib_path, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_FILES],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")

    def one(k):
        lib = obuild.build([f"-DOR_MUTANT={k}"], out=str(d / f"liboracle_m{k}.so"))
        return k, _run_pins(lib)

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        return dict(ex.map(one, [0] + MUTANTS))


def test_unmodified_build_passes_the_pins(results):
    r = results[0]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("k", MUTANTS)
def test_planted_mistake_is_caught(results, k):
    r = results[k]
    assert r.returncode != 0, f"mistake {k} passed every pin:\n{r.stdout[-1500:]}"
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    print(f"mistake {k}: caught by {failed[:1]}")
