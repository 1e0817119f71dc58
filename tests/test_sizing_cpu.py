"""The heavy-chunk list capacity (csrc/sizing.h) against the chunks a tick can
emit. The capacity is compiled from the library's own header into a scratch
shared object (no GPU), and compared with an exact count of what the round
batch emits -- ceil(size / 256) chunks for every range longer than the split
threshold -- over worst-case and random ticks: every vertex an item of at most
two segments, each range inside its row."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_2506_19349_amd", "csrc")
CHUNK = 256          # kHeavyChunk
MIN_SPLIT = 64       # kDefaultHeavy: the least split the library allows


@pytest.fixture(scope="module")
def capacity(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("sizing")
    src = d / "cap.cpp"
    src.write_text('#include "sizing.h"\n'
                   'extern "C" long long cap(long long nnz, long long heavy_rows, long long chunk) {\n'
                   '  return (long long)sssp::heavy_list_capacity(nnz, heavy_rows, chunk);\n}\n')
    so = d / "libcap.so"
    subprocess.run([cxx, "-O1", "-shared", "-fPIC", "-I" + HEADER_DIR, str(src), "-o", str(so)], check=True)
    lib = ctypes.CDLL(str(so))
    lib.cap.restype = ctypes.c_longlong
    lib.cap.argtypes = [ctypes.c_longlong] * 3
    return lambda deg: lib.cap(int(deg.sum()), int((deg > MIN_SPLIT).sum()), CHUNK)


def chunks(sizes, split):
    s = np.asarray(sizes, np.int64)
    s = s[s > split]
    return int(((s + CHUNK - 1) // CHUNK).sum())


def test_worst_tick_fits(capacity):
    """Every vertex twice, whole rows, at the least split: the largest count."""
    rng = np.random.default_rng(1)
    degs = [np.full(1000, 65), np.full(1000, 257), np.full(300, 513), rng.integers(0, 300, size=5000),
            np.concatenate([np.full(3, 400000), np.full(20000, 1)]), np.zeros(10, np.int64),
            graphgen.to_csr(graphgen.rmat(12, seed=5)).degrees(),
            graphgen.to_csr(graphgen.gnm(1 << 12, 50 << 12, 4, seed=6)).degrees()]
    for deg in degs:
        deg = np.asarray(deg, np.int64)
        cap = capacity(deg)
        for split in (MIN_SPLIT, 65, 100, 255, 256, 1000):
            worst = 2 * chunks(deg, split)
            assert worst <= cap, (split, worst, cap)
    # the bound is not loose by more than the rounding of each row: rows of
    # 65 entries each take one chunk per appearance
    deg = np.full(1000, 65)
    assert capacity(deg) <= 2 * chunks(deg, MIN_SPLIT) + 2 * ((65000 + 255) // 256) + 16


def test_random_ticks_fit(capacity):
    rng = np.random.default_rng(2)
    for trial in range(200):
        n = int(rng.integers(1, 3000))
        deg = rng.integers(0, int(rng.choice([80, 300, 3000])), size=n).astype(np.int64)
        cap = capacity(deg)
        split = int(rng.choice([64, 100, 256, 1024]))
        # each vertex appears 0, 1 or 2 times with a range inside its row
        times = rng.integers(0, 3, size=n)
        sizes = []
        for v in np.nonzero(times)[0]:
            for _ in range(int(times[v])):
                lo = int(rng.integers(0, deg[v] + 1))
                hi = int(rng.integers(lo, deg[v] + 1))
                sizes.append(hi - lo)
        assert chunks(sizes, split) <= cap, trial


def test_old_rule_was_not_a_bound():
    """nnz / 128 + 4096 (the earlier sizing) is exceeded by a first round of a
    graph whose rows hold 65..256 entries: one chunk per range."""
    deg = np.full(200000, 100, np.int64)
    assert 2 * chunks(deg, MIN_SPLIT) > int(deg.sum()) // 128 + 4096
