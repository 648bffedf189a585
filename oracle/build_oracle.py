"""Build the oracle's C helper (test infrastructure only).

Compiles oracle/csrc/*.c with gcc into oracle/liboracle_fma.so. Plain C with
-ffp-contract=off, so the only fused operations are the explicit fma() calls.
"""
from __future__ import annotations

import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
LIB = HERE / "liboracle_fma.so"


def build(force: bool = True) -> pathlib.Path:
    if LIB.exists() and not force:
        return LIB
    src = sorted(str(p) for p in (HERE / "csrc").glob("*.c"))
    tmp = LIB.with_suffix(".so.tmp")
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                    "-shared", "-fPIC", "-o", str(tmp), *src, "-lm"], check=True)
    tmp.replace(LIB)
    return LIB


if __name__ == "__main__":
    print(build())
