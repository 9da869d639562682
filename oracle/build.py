"""Compile the C oracle (test infrastructure): ``oracle/liborc.so``, serial,
and ``oracle/liborc_omp.so``, the same source with OpenMP over the lines of
each sweep (the all-core CPU timing baseline)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "asd_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
LIB_OMP = os.path.join(HERE, "liborc_omp.so")
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def _build_one(out, extra):
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, *extra, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True, omp: bool = None) -> str:
    """Build the oracle libraries with gcc (omp None: both); returns the
    serial library's path."""
    for path, extra, want in ((LIB, [], omp in (None, False)), (LIB_OMP, ["-fopenmp"], omp in (None, True))):
        if not want:
            continue
        if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(SRC):
            continue
        _build_one(path, extra)
    return LIB


if __name__ == "__main__":
    print(build())
