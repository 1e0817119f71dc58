"""Loader for the hand-worked fixtures in tests/golden/."""
import glob
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
INF = 0xFFFFFFFF


def load(path):
    n = s = None
    src, dst, w = [], [], []
    dist = None
    overflow = False
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            tag = line[0]
            if tag == "n":
                n = int(line[1])
            elif tag == "s":
                s = int(line[1])
            elif tag == "e":
                src.append(int(line[1]))
                dst.append(int(line[2]))
                w.append(int(line[3]))
            elif tag == "d":
                dist = np.array([INF if t == "INF" else int(t) for t in line[1:]], dtype=np.uint64)
            elif tag == "x" and line[1] == "overflow":
                overflow = True
    return {
        "name": os.path.basename(path),
        "n": n,
        "s": s,
        "src": np.array(src, dtype=np.int32),
        "dst": np.array(dst, dtype=np.int32),
        "w": np.array(w, dtype=np.uint64).astype(np.uint32),
        "dist": None if dist is None else dist.astype(np.uint32),
        "overflow": overflow,
    }


def all_fixtures():
    return [load(p) for p in sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))]
