"""Compile the oracle's C parts (oracle/*.c) with gcc into oracle/lib<name>.so.

Test and baseline infrastructure only; called by the repository's build step.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> list:
    out = []
    for f in sorted(os.listdir(HERE)):
        if not f.endswith(".c"):
            continue
        lib = os.path.join(HERE, "lib" + f[:-2] + ".so")
        cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-o", lib, os.path.join(HERE, f)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        out.append(lib)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
