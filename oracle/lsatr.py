"""ORACLE — test infrastructure only (same rules as oracle/dope.py).

Block sub-problem solver for non-submodular blocks of any size: the trust-region local submodular approximation
(LSA-TR) of Gorelick, Schmidt, Boykov, Delong and Ward (CVPR 2014), the serial non-submodular optimiser whose
computations the paper distributes with DOPE in its curvature experiment (Sec. 3.3, Table 1).

The block problem is Eq. (8) scaled by 2^14:  E(x) = sum_i U_i x_i + sum_{(i,j)} c_ij |x_i - x_j|,  x in {0,1}^m,
with capacities c_ij of either sign (c < 0 on repulsive edges makes the term supermodular:
c |x_i - x_j| = c x_i + c x_j - 2 c x_i x_j with -2c > 0).

One LSA-TR step at the current labelling x~:
  * the supermodular terms are replaced by their linearisation at x~ (x_i x_j ~ x~_j x_i + x~_i x_j - x~_i x~_j),
    which adds c_ij (1 - 2 x~_j) to U_i and c_ij (1 - 2 x~_i) to U_j for every edge with c_ij < 0; the result is
    the approximation A(x) = sum_i U'_i x_i + sum_{c_ij > 0} c_ij |x_i - x_j| (+ a constant, exact at x~);
  * the trust region adds lam |x_i - x~_i| = lam (1 - 2 x~_i) x_i + lam x~_i;
  * x* = the minimal minimiser of A + trust (a submodular problem: one max-flow, canonical minimal cut);
  * actual reduction R = E(x~) - E(x*), predicted reduction P = A(x~) - A(x*);
    accept x* when R > 0 and R >= P / 4; when also R >= 3 P / 4 the region grows (lam level down), and a rejected
    step shrinks it (lam level up); a step whose x* is x~ ends the search (no better labelling in the region).

Integer reading of the step-size schedule (the paper's optimiser uses real factors): lam = 0 at level -1 and
lam = 2^14 10^k at level k >= 0 (2^14 is one unit of the input energy in the block problem's scale); the search
also stops when the level passes 4 (lam > 2^28) or after 32 steps.  Start: x~_i = [U_i < 0] (the unary-only minimiser).
"""
from __future__ import annotations

import numpy as np

from . import dope as od

LAMBDA_UNIT = 1 << 14
LEVEL_MAX = 4
MAX_STEPS = 32


def block_energy(U, ea, eb, cap, x) -> int:
    x = np.asarray(x, dtype=np.int64)
    return int(np.asarray(U, dtype=np.int64) @ x + np.asarray(cap, dtype=np.int64) @ np.abs(x[ea] - x[eb]))


def lam_of(level: int) -> int:
    return 0 if level < 0 else LAMBDA_UNIT * 10 ** level


def lsatr(U, ea, eb, cap, record=None):
    """LSA-TR on one block problem; returns the labelling (uint8).  record, if a list, receives (level, accepted)
    per step."""
    U = np.asarray(U, dtype=np.int64)
    ea = np.asarray(ea, dtype=np.int64)
    eb = np.asarray(eb, dtype=np.int64)
    cap = np.asarray(cap, dtype=np.int64)
    m = len(U)
    x = (U < 0).astype(np.int64)
    E = block_energy(U, ea, eb, cap, x)
    neg = cap < 0
    pos = cap > 0
    level = -1
    for _ in range(MAX_STEPS):
        U1 = U.copy()
        np.add.at(U1, ea[neg], cap[neg] * (1 - 2 * x[eb[neg]]))
        np.add.at(U1, eb[neg], cap[neg] * (1 - 2 * x[ea[neg]]))
        lam = lam_of(level)
        U2 = U1 + lam * (1 - 2 * x)
        xs, _ = od.solve_subproblem(U2, ea[pos].astype(np.int32), eb[pos].astype(np.int32), cap[pos], "maxflow")
        xs = np.asarray(xs, dtype=np.int64)
        if np.array_equal(xs, x):
            if record is not None:
                record.append((level, False))
            break
        A_x = int(U1 @ x + cap[pos] @ np.abs(x[ea[pos]] - x[eb[pos]]))
        A_s = int(U1 @ xs + cap[pos] @ np.abs(xs[ea[pos]] - xs[eb[pos]]))
        Es = block_energy(U, ea, eb, cap, xs)
        R, P = E - Es, A_x - A_s
        accepted = R > 0 and 4 * R >= P
        if record is not None:
            record.append((level, accepted))
        if accepted:
            x, E = xs, Es
            if 4 * R >= 3 * P and level >= 0:
                level -= 1
        else:
            level += 1
            if level > LEVEL_MAX:
                break
    assert len(x) == m
    return x.astype(np.uint8)
