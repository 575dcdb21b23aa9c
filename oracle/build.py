"""Compile the host oracle (plain C, OpenMP) into ``oracle/liboracle.so``.

Test infrastructure: the product library never links or loads this.
``mutant`` > 0 builds a variant with one planted mistake (see the header of
apsp_oracle.c) into ``oracle/liboracle_mutant<m>.so``; the test suite uses
those variants to show that its pins catch such mistakes.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "apsp_oracle.c")


def lib_path(mutant: int = 0) -> str:
    name = "liboracle.so" if mutant == 0 else f"liboracle_mutant{mutant}.so"
    return os.path.join(HERE, name)


def build(mutant: int = 0, force: bool = False) -> str:
    out = lib_path(mutant)
    if (not force and os.path.exists(out)
            and os.path.getmtime(out) >= os.path.getmtime(SRC)):
        return out
    # x86-64-v3 (AVX2) rather than -march=native: the library built here also
    # runs on other hosts.
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wextra", "-Wno-unused-parameter",
           f"-DORC_MUTANT={int(mutant)}", SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(force=True))
