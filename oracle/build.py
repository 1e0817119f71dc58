"""Build the oracle's C part (``liboracle.so``) with gcc. Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


# binary32 sums must be single IEEE additions: no contraction into fused
# multiply-adds, no wider intermediates (x86-64 SSE arithmetic)
FLAGS = ["-std=c11", "-ffp-contract=off", "-fexcess-precision=standard", "-fPIC", "-shared", "-pthread"]


def build(verbose: bool = False) -> str:
    """The in-tree library, for any x86-64 host (it travels with the tree)."""
    src = os.path.join(HERE, "dijkstra.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3"] + FLAGS + ["-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_for_this_host(out_dir: str, verbose: bool = False) -> str:
    """The same source tuned for the CPU it is built on (-O3 -march=native),
    written to out_dir: for timing the oracle as a CPU baseline on the machine
    that runs it. Same arithmetic (no contraction, no excess precision)."""
    src = os.path.join(HERE, "dijkstra.c")
    out = os.path.join(out_dir, "liboracle_native.so")
    cmd = ["gcc", "-O3", "-march=native"] + FLAGS + ["-o", out, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
