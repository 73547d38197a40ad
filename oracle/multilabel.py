"""ORACLE — test infrastructure only (same rules as oracle/dope.py: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it; the product library never does).

Multi-label Potts segmentation by alpha-expansion with DOPE solving every expansion move.  The paper's energy is
binary (Eq. 1); its introduction notes that multi-region problems reduce to sequences of binary ones, and its
conclusion names multi-label energies as the next step.  The outer loop here is the expansion-move algorithm of
Boykov, Veksler and Zabih (2001): for each label a in turn, every pixel may switch to a or keep its label, which is
a binary problem that is submodular for Potts interactions.

Energy (integers; lambda folded into the edge weights by the caller):

    E(L) = sum_i D[L_i, i] + sum_{edges (i,j)} V_ij [L_i != L_j],      L_i in {0, .., nl - 1},  V_ij >= 0,

with V on the half-stencil layout of the binary energy (V[o, i] weights the edge i <-> i + offset o).

Expansion move of label a from L: y_i = 1 moves pixel i to a.  Writing l_i(0) = L_i, l_i(1) = a, each edge term
[l_i(y_i) != l_j(y_j)] takes four values; doubled, it is affine in y plus a multiple of |y_i - y_j|:
  * L_i = L_j != a:             2 |y_i - y_j|
  * L_i = L_j = a:              0
  * L_i != L_j, neither is a:   2 - y_i - y_j + |y_i - y_j|
  * L_i = a != L_j:             2 - 2 y_j          (and symmetrically)
so  2 E(move(L, y, a)) = 2 E(L) + sum_i u_i y_i + sum_{edges} W_ij |y_i - y_j|  with
  u_i  = 2 (D[a, i] - D[L_i, i]) - sum_{j ~ i : L_j != L_i, L_i != a} V_ij (1 + [L_j = a]),
  W_ij = 2 V_ij if L_i = L_j != a;  V_ij if L_i != L_j and neither is a;  0 otherwise.
This binary energy is the one DOPE takes (Eq. 1 with lambda = 1, i.e. lambda_q8 = 256, and w = W >= 0).

Loop (deterministic): labels start at argmin_l D[l, i] (smallest l on ties); a cycle visits a = 0 .. nl - 1; a
move's labelling (DOPE's labels after its solve) is accepted only when it lowers E strictly; the loop stops after
a cycle without an accepted move or after max_cycles cycles.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

from . import dope as od


def _edges(dims, ndim, conn):
    """(o, i, j, valid) per half-stencil offset: arrays of pixel indices of every on-grid edge i <-> j."""
    W_, H_, D_ = dims
    n = W_ * H_ * D_
    idx = np.arange(n, dtype=np.int64)
    x, y, z = idx % W_, (idx // W_) % H_, idx // (W_ * H_)
    out = []
    for o, (dx, dy, dz) in enumerate(od.neighbour_offsets(ndim, conn)):
        ok = (x + dx >= 0) & (x + dx < W_) & (y + dy >= 0) & (y + dy < H_) & (z + dz >= 0) & (z + dz < D_)
        i = idx[ok]
        out.append((o, i, i + dx + W_ * (dy + H_ * dz)))
    return out


def energy(D: np.ndarray, V: np.ndarray, L: np.ndarray, dims, ndim, conn) -> int:
    """E(L) = sum_i D[L_i, i] + sum_edges V_ij [L_i != L_j] (exact int64)."""
    L = np.asarray(L, dtype=np.int64)
    n = L.size
    e = int(np.asarray(D, dtype=np.int64)[L, np.arange(n)].sum())
    for o, i, j in _edges(dims, ndim, conn):
        e += int(np.asarray(V[o], dtype=np.int64)[i][L[i] != L[j]].sum())
    return e


def expansion_energy(D, V, L, a, dims, ndim, conn) -> Tuple[np.ndarray, np.ndarray]:
    """The binary energy of the expansion move of label a from L: (u int64[n], W int64[h, n]) as in the module
    docstring (2 E(move) = 2 E(L) + u.y + sum W |y_i - y_j|)."""
    D = np.asarray(D, dtype=np.int64)
    L = np.asarray(L, dtype=np.int64)
    n = L.size
    ar = np.arange(n)
    u = 2 * (D[a, ar] - D[L, ar])
    Wb = np.zeros((len(od.neighbour_offsets(ndim, conn)), n), dtype=np.int64)
    for o, i, j in _edges(dims, ndim, conn):
        v = np.asarray(V[o], dtype=np.int64)[i]
        li, lj = L[i], L[j]
        same = li == lj
        Wb[o, i] = np.where(same, np.where(li != a, 2 * v, 0), np.where((li != a) & (lj != a), v, 0))
        diff = ~same
        # pixel i's share: its label differs from j's and is not a
        si = diff & (li != a)
        np.subtract.at(u, i[si], v[si] * (1 + (lj[si] == a)))
        sj = diff & (lj != a)
        np.subtract.at(u, j[sj], v[sj] * (1 + (li[sj] == a)))
    return u, Wb


@dataclasses.dataclass
class MoveRecord:
    label: int
    accepted: bool
    energy: int                  # E after the move (the old energy when rejected)
    binary_iterations: int       # DOPE iterations of the move's solve
    labels: np.ndarray           # labels after the move


def initial_labels(D: np.ndarray) -> np.ndarray:
    """argmin_l D[l, i], smallest l on ties."""
    return np.argmin(np.asarray(D, dtype=np.int64), axis=0).astype(np.uint8)


def binary_problem(template, u, Wb):
    """The expansion move as a DOPE problem on the template's grid, partition and schedule (lambda_q8 = 256)."""
    return dataclasses.replace(template, u=np.asarray(u, dtype=np.int64).astype(np.int32),
                               w=np.asarray(Wb, dtype=np.int64).astype(np.int32), lam_q8=256, solver="maxflow")


def alpha_expansion(template, D, V, max_cycles: int = 5, threads: Optional[int] = None,
                    move_solver=None) -> Tuple[np.ndarray, int, List[MoveRecord]]:
    """Alpha-expansion with DOPE (Algorithm 1, solved to its stopping rule or max_iter) for every move.
    template: a Problem carrying dims, stencil, block partition and ADMM schedule.  move_solver, if given,
    replaces DOPE: a function (problem) -> (binary labels, iterations)."""
    dims, ndim, conn = template.dims, template.ndim, template.conn
    nl = int(np.asarray(D).shape[0])
    L = initial_labels(D)
    E = energy(D, V, L, dims, ndim, conn)
    recs: List[MoveRecord] = []
    for _ in range(max_cycles):
        changed = False
        for a in range(nl):
            u, Wb = expansion_energy(D, V, L, a, dims, ndim, conn)
            prob = binary_problem(template, u, Wb)
            if move_solver is None:
                st, infos, _, _ = od.run(prob, threads=threads)
                y, iters = od.labels(st.Y), len(infos)
            else:
                y, iters = move_solver(prob)
            Ln = np.where(np.asarray(y) != 0, a, L).astype(np.uint8)
            En = energy(D, V, Ln, dims, ndim, conn)
            acc = En < E
            if acc:
                L, E, changed = Ln, En, True
            recs.append(MoveRecord(a, bool(acc), E, iters, L.copy()))
        if not changed:
            break
    return L, E, recs


def exact_move_solver(prob):
    """A move solved exactly: the global minimal min cut of the binary energy (for the pins)."""
    x, _ = od.global_mincut(prob)
    return x, 0
