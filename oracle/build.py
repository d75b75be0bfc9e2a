"""Builds the FP64 CPU oracle (test infrastructure) with gcc: plain -O2, no FMA
contraction, no fast-math.  Two builds of the same source: liboracle.so single-threaded
(the parity reference), liboracle_omp.so with -fopenmp (the all-cores CPU baseline and the
oracle of the largest parity cases)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall", "-fPIC", "-shared"]


def _build_one(out, extra, force):
    src = os.path.join(HERE, "pml_oracle.c")
    hdr = os.path.join(HERE, "pml_oracle.h")
    if (not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src)
            and os.path.getmtime(out) >= os.path.getmtime(hdr)):
        return out
    tmp = out + ".tmp"
    subprocess.run(["gcc"] + FLAGS + extra + ["-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    out = _build_one(os.path.join(HERE, "liboracle.so"), ["-Wno-unknown-pragmas"], force)
    _build_one(os.path.join(HERE, "liboracle_omp.so"), ["-fopenmp"], force)
    return out


if __name__ == "__main__":
    print(build())
