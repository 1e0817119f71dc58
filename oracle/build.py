"""Build the oracle's C part (``liboracle.so``) with gcc. Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "dijkstra.c")
    tmp = LIB + ".tmp"
    # binary32 sums must be single IEEE additions: no contraction into fused
    # multiply-adds, no wider intermediates (x86-64 SSE arithmetic)
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fexcess-precision=standard", "-fPIC", "-shared",
           "-pthread", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
