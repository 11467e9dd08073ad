"""Build the FP64 CPU oracle shared library (test infrastructure only).

``python -m oracle.build`` or ``oracle.build.build()`` compiles
``sweep_oracle.c`` with gcc into ``liboracle_sweep.so`` next to it.
FP contraction is disabled so the oracle rounds every operation where the
source writes it.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sweep_oracle.c")
LIB = os.path.join(HERE, "liboracle_sweep.so")

CFLAGS = ["-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(extra_flags=None, out=LIB, quiet=True, src=SRC) -> str:
    """Compile the oracle (or another copy of its source, ``src``); returns
    the path of the shared library."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), src, "-o", tmp, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    if not quiet and res.stderr:
        sys.stderr.write(res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(quiet=False))
