"""Builds the FP64 CPU oracle (test infrastructure) with gcc: plain -O2, no FMA
contraction, no fast-math, single-threaded."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(force: bool = True) -> str:
    out = os.path.join(HERE, "liboracle.so")
    src = os.path.join(HERE, "pml_oracle.c")
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall",
           "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
