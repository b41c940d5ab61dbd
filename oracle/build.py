"""Builds the CPU reference library (test infrastructure only).

The reference is plain C, compiled with gcc at -O3 without FMA contraction
and with OpenMP over block rows.  ``build(mutant=n)`` produces a copy with one
deliberate mistake planted (see the header of ``bsmm_oracle.c``); the test
suite uses those copies to show that its pins catch such mistakes.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bsmm_oracle.c")


def lib_path(mutant: int = 0) -> str:
    name = "liborc.so" if mutant == 0 else f"liborc_mutant{mutant}.so"
    return os.path.join(HERE, name)


def build(mutant: int = 0, out: str = None) -> str:
    out = out or lib_path(mutant)
    cmd = [
        "gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-Wextra",
        f"-DORC_MUTANT={int(mutant)}", "-o", out + ".tmp", SRC, "-lm",
    ]
    if mutant == 0:
        cmd.insert(1, "-Werror")
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
