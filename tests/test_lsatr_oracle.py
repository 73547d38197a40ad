"""Pins of the oracle's LSA-TR block solver (oracle/lsatr.py), on the CPU.

Independent checks: the solver never ends above its start or below the exhaustive minimum of the block problem;
on submodular blocks its first step (lam = 0, nothing to linearise) is the minimal minimum cut, so it returns the
max-flow solver's labelling; the first step's linearised unaries of a two-pixel problem worked by hand; and the
acceptance rule against the reductions it reports."""
import numpy as np
import pytest

from oracle import dope as od
from oracle import lsatr


def _grid_edges(W, H):
    ea, eb = [], []
    for y in range(H):
        for x in range(W):
            i = x + W * y
            if x + 1 < W:
                ea.append(i); eb.append(i + 1)
            if y + 1 < H:
                ea.append(i); eb.append(i + W)
    return np.array(ea, np.int32), np.array(eb, np.int32)


def _random_block(rng, W, H, neg_frac):
    ea, eb = _grid_edges(W, H)
    cap = rng.integers(50, 500, size=len(ea)).astype(np.int64)
    cap = np.where(rng.random(len(ea)) < neg_frac, -cap, cap) * (1 << 14)
    U = rng.integers(-1000, 1000, size=W * H).astype(np.int64) * (1 << 14)
    return U, ea, eb, cap


@pytest.mark.parametrize("seed", range(40))
def test_between_start_and_exhaustive_minimum(seed):
    rng = np.random.default_rng(seed)
    U, ea, eb, cap = _random_block(rng, 4, 3, 0.35)
    x = lsatr.lsatr(U, ea, eb, cap)
    xe, _ = od.solve_subproblem(U, ea, eb, cap, "exhaustive")
    e = lsatr.block_energy(U, ea, eb, cap, x)
    assert lsatr.block_energy(U, ea, eb, cap, xe) <= e <= lsatr.block_energy(U, ea, eb, cap, (U < 0).astype(int))


def test_usually_finds_the_block_minimum():
    rng = np.random.default_rng(123)
    hits = 0
    for _ in range(100):
        U, ea, eb, cap = _random_block(rng, 4, 4, 0.3)
        x = lsatr.lsatr(U, ea, eb, cap)
        xe, _ = od.solve_subproblem(U, ea, eb, cap, "exhaustive")
        hits += lsatr.block_energy(U, ea, eb, cap, x) == lsatr.block_energy(U, ea, eb, cap, xe)
    assert hits >= 70


@pytest.mark.parametrize("seed", range(10))
def test_submodular_blocks_give_the_minimal_minimum_cut(seed):
    rng = np.random.default_rng(1000 + seed)
    U, ea, eb, cap = _random_block(rng, 8, 6, 0.0)
    x = lsatr.lsatr(U, ea, eb, cap)
    xm, _ = od.solve_subproblem(U, ea, eb, cap, "maxflow")
    assert np.array_equal(x, xm)


def test_two_pixel_linearisation_by_hand():
    """E(x) = 3 x0 - 5 x1 + c |x0 - x1| with c = -4 (repulsive).  Start x~ = [U < 0] = (0, 1), E = -5 + (-4) = -9.
    Linearised at x~: U0 += c (1 - 2 x~1) = +4 -> 7, U1 += c (1 - 2 x~0) = -4 -> -9; no positive edge, so the
    step's minimiser is (0, 1) = x~ and the search stops there.  The exact minimum is also (0, 1): E(0,0) = 0,
    E(1,0) = -1, E(1,1) = -2, E(0,1) = -9."""
    U = np.array([3, -5], np.int64)
    ea, eb = np.array([0], np.int32), np.array([1], np.int32)
    cap = np.array([-4], np.int64)
    rec = []
    x = lsatr.lsatr(U, ea, eb, cap, record=rec)
    assert list(x) == [0, 1] and rec == [(-1, False)]
    # a start that linearisation improves: U = (-3, -5), c = -10: x~ = (1, 1), E = -8; linearised U0 = -3 + 10 = 7,
    # U1 = -5 + 10 = 5 -> minimiser (0, 0): actual E = 0 (R = -8 < 0, rejected) -> lam = 2^14 level 0 with trust
    # term lam (1 - 2 x~_i) = -2^14 on both: U' = (7 - 16384, 5 - 16384) -> (1, 1) = x~: stop
    rec = []
    x = lsatr.lsatr(np.array([-3, -5], np.int64), ea, eb, np.array([-10], np.int64), record=rec)
    assert list(x) == [1, 1] and rec == [(-1, False), (0, False)]


def test_acceptance_rule_matches_the_reductions():
    """Replaying every recorded step: an accepted step lowered the energy."""
    rng = np.random.default_rng(77)
    for _ in range(30):
        U, ea, eb, cap = _random_block(rng, 5, 4, 0.4)
        rec = []
        x = lsatr.lsatr(U, ea, eb, cap, record=rec)
        assert len(rec) <= lsatr.MAX_STEPS
        levels = [lv for lv, _ in rec]
        assert all(-1 <= lv <= lsatr.LEVEL_MAX + 1 for lv in levels)
        assert lsatr.block_energy(U, ea, eb, cap, x) <= lsatr.block_energy(U, ea, eb, cap, (U < 0).astype(int))
