"""Host build of the eigenvalue ranking that orders the small SVD's output
(Section 2.1, step 6: singular values sorted descending).

The finishing kernel inverts these ranks into an index table and then reads
eigenvector columns through it, so the ranks must be a permutation for every
input, including NaN eigenvalues (a non-finite input matrix) and ties.  The
routine is compiled for the host with g++ from the same header the kernel
includes and checked here against a plain Python sort.
"""

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rank_bin(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("rank") / "rank_check")
    subprocess.run([gxx, "-O1", "-std=c++17", os.path.join(HERE, "rank_check.cpp"), "-o", out],
                   check=True)
    return out


def run(rank_bin, rows):
    text = "\n".join(f"{len(r)} " + " ".join(repr(float(x)) for x in r) for r in rows) + "\n"
    res = subprocess.run([rank_bin], input=text, capture_output=True, text=True, check=True)
    return [list(map(int, ln.split())) for ln in res.stdout.strip().split("\n")]


def expected(vals):
    # descending, NaN as -inf, ties by index
    key = [(-(v if not math.isnan(v) else -math.inf), i) for i, v in enumerate(vals)]
    order = sorted(range(len(vals)), key=lambda i: key[i])
    rank = [0] * len(vals)
    for r, i in enumerate(order):
        rank[i] = r
    return rank


CASES = [
    [3.0, 1.0, 2.0],
    [1.0, 1.0, 1.0, 1.0],
    [float("nan"), 2.0, 1.0],
    [float("nan"), float("nan"), 0.5, float("nan")],
    [float("inf"), float("nan"), -float("inf"), 0.0, -0.0, 0.0],
    [2.0, float("nan"), 2.0, -1.0, float("nan"), 2.0],
    [0.0],
]


def test_ranks_are_a_permutation_with_nan_and_ties(rank_bin):
    rng = np.random.default_rng(5)
    rows = [list(c) for c in CASES]
    for _ in range(40):
        l = int(rng.integers(1, 40))
        v = rng.choice([0.0, 1.0, 2.0, float("nan"), float("inf"), -1.0], size=l)
        rows.append(list(v))
    got = run(rank_bin, rows)
    for vals, r in zip(rows, got):
        assert sorted(r) == list(range(len(vals))), (vals, r)
        assert r == expected(vals), (vals, r)


def test_plain_count_rank_is_not_a_permutation_with_nan():
    # the rank without the NaN mapping (count strictly larger values, ties by
    # index) collides once a NaN is present: the failure the mapping removes
    vals = [float("nan"), 2.0, 1.0]
    rank = [sum((vj > vi) or (vj == vi and j < i) for j, vj in enumerate(vals))
            for i, vi in enumerate(vals)]
    assert sorted(rank) != list(range(len(vals)))
