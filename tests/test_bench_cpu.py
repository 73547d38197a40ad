"""Host-side checks of the benchmark's bookkeeping (no GPU): the interior-pixel count and the enumeration count
that its algorithmic-bytes and ALU-roofline figures rest on, against brute force over the oracle's partition, and
the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import dope as od  # noqa: E402


def brute_interior_axis(N, B, o, r):
    """Coordinates x whose window [x - r, x + r] (clipped to the axis) lies in exactly one block, the same one
    for every coordinate of the window."""
    iv = od.partition_axis(N, B, o)
    member = [frozenset(t for t, (a, b) in enumerate(iv) if a <= y < b) for y in range(N)]
    count = 0
    for x in range(N):
        win = {member[y] for y in range(max(0, x - r), min(N, x + r + 1))}
        if len(win) == 1 and len(next(iter(win))) == 1:
            count += 1
    return count


@pytest.mark.parametrize("dims,block,overlap,r", [
    ((512, 512, 1), (32, 32, 1), (2, 2, 0), 1),
    ((257, 131, 1), (32, 16, 1), (3, 1, 0), 1),
    ((128, 128, 64), (16, 16, 16), (1, 1, 1), 1),
    ((512, 512, 1), (32, 32, 1), (2, 2, 0), 2),
    ((200, 150, 1), (16, 16, 1), (3, 3, 0), 3),
    ((131, 97, 1), (16, 16, 1), (4, 4, 0), 4),
    ((512, 512, 1), (66, 66, 1), (2, 2, 0), 1),     # 64 even blocks
    ((40, 7, 1), (64, 8, 1), (2, 2, 0), 1),         # one block along x, one pixel narrower than B along y
])
def test_interior_count_matches_brute_force(dims, block, overlap, r):
    expect = 1
    for N, B, o in zip(dims, block, overlap):
        expect *= brute_interior_axis(N, B if B < N else N, o if B < N else 0, r)
    assert bench.interior_count(dims, block, overlap, r) == expect


@pytest.mark.parametrize("dims,block,overlap", [
    ((256, 256, 1), (4, 4, 1), (1, 1, 0)),
    ((37, 29, 1), (4, 4, 1), (1, 1, 0)),
    ((12, 10, 1), (4, 3, 1), (2, 1, 0)),
])
def test_exhaustive_codes_match_block_sizes(dims, block, overlap):
    blocks = od.make_blocks(dims, block, overlap)
    assert bench.exhaustive_codes(dims, block, overlap) == sum(2 ** len(b.idx) for b in blocks)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode != 0
    assert "one GPU" in out.stdout
