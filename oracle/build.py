"""Compile the CPU oracle into ``oracle/liboracle.so`` (test infrastructure).

Flags: ``-ffp-contract=off`` so that the compiler never fuses a multiply and
an add the source did not write as ``fma``, and no fast-math (no
reassociation), so the optimisation level and target changes no result;
OpenMP over trajectories.  The in-tree library targets x86-64-v3 (AVX2 and
FMA: every current server CPU), so that one build serves any host; the
CPU-baseline timing builds a copy for the host it runs on
(``build_native``, ``-march=native``).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
OUT = os.path.join(HERE, "liboracle.so")

FLAGS = ["-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
         "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wno-unused-function"]
PORTABLE = ["-march=x86-64-v3"]
NATIVE = ["-march=native"]


def _compile(out, arch, verbose):
    tmp = out + ".tmp"
    cmd = ["g++", *FLAGS, *arch, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    return _compile(OUT, PORTABLE, verbose)


def build_native(out: str, verbose: bool = False) -> str:
    """A copy tuned for the host that builds it (for timing on that host)."""
    return _compile(out, NATIVE, verbose)


def flags(native: bool = False) -> str:
    return " ".join(["g++", *FLAGS, *(NATIVE if native else PORTABLE)])


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
