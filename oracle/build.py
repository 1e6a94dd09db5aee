"""Build the FP64 oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure: compiling the checker is not using it.  ``mutant``
plants one numbered mistake (see fft_oracle.c) for the test that shows the
pins catch it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fft_oracle.c")


def build(out: str | None = None, mutant: int = 0) -> str:
    out = out or os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
           "-fno-fast-math", "-ffp-contract=off", f"-DORACLE_MUTANT={int(mutant)}",
           SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(mutant=int(sys.argv[1]) if len(sys.argv) > 1 else 0))
