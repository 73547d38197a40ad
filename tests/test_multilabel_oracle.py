"""Pins of the multi-label oracle (alpha-expansion around DOPE, oracle/multilabel.py), on the CPU.

What fixes the oracle independently of itself: the expansion-move energy identity checked against the definition
of E by brute force over every move labelling; Boykov-Veksler-Zabih's bound (exact expansion moves end within a
factor 2 of the optimum of a Potts energy with nonnegative data terms) and local optimality against brute force;
and, with a one-block partition (where DOPE's first iteration is the global minimal min cut and it stops there),
the DOPE-driven loop equals the loop with exact moves."""
import itertools

import numpy as np
import pytest

from oracle import dope as od
from oracle import multilabel as ml
from synth.multilabel import multilabel_image


def _edges_loop(dims, ndim, conn):
    W_, H_, D_ = dims
    out = []
    for o, (dx, dy, dz) in enumerate(od.neighbour_offsets(ndim, conn)):
        for z in range(D_):
            for y in range(H_):
                for x in range(W_):
                    if 0 <= x + dx < W_ and 0 <= y + dy < H_ and 0 <= z + dz < D_:
                        out.append((o, x + W_ * (y + H_ * z), x + dx + W_ * (y + dy + H_ * (z + dz))))
    return out


def _energy_loop(D, V, L, dims, ndim, conn):
    e = sum(int(D[L[i], i]) for i in range(len(L)))
    for o, i, j in _edges_loop(dims, ndim, conn):
        if L[i] != L[j]:
            e += int(V[o, i])
    return e


def _tiny(seed, dims, ndim, conn, nl, d_max=50, v_max=30):
    rng = np.random.default_rng(seed)
    n = dims[0] * dims[1] * dims[2]
    D = rng.integers(0, d_max + 1, size=(nl, n)).astype(np.int32)
    h = len(od.neighbour_offsets(ndim, conn))
    V = np.zeros((h, n), dtype=np.int32)
    for o, i, j in _edges_loop(dims, ndim, conn):
        V[o, i] = rng.integers(0, v_max + 1)
    return D, V


CASES = [((3, 3, 1), 2, 4), ((4, 3, 1), 2, 8), ((2, 2, 3), 3, 6), ((5, 5, 1), 2, 24)]


@pytest.mark.parametrize("dims,ndim,conn", CASES)
def test_energy_is_the_potts_definition(dims, ndim, conn):
    D, V = _tiny(1, dims, ndim, conn, 3)
    rng = np.random.default_rng(2)
    for _ in range(5):
        L = rng.integers(0, 3, size=D.shape[1]).astype(np.uint8)
        assert ml.energy(D, V, L, dims, ndim, conn) == _energy_loop(D, V, L, dims, ndim, conn)


@pytest.mark.parametrize("dims,ndim,conn", CASES[:3])
def test_expansion_energy_identity_by_brute_force(dims, ndim, conn):
    """2 E(move(L, y, a)) = 2 E(L) + u.y + sum W |y_i - y_j| for every move labelling y."""
    nl = 3
    D, V = _tiny(3, dims, ndim, conn, nl)
    n = D.shape[1]
    rng = np.random.default_rng(4)
    edges = _edges_loop(dims, ndim, conn)
    for _ in range(4):
        L = rng.integers(0, nl, size=n).astype(np.uint8)
        E0 = _energy_loop(D, V, L, dims, ndim, conn)
        for a in range(nl):
            u, Wb = ml.expansion_energy(D, V, L, a, dims, ndim, conn)
            assert np.all(Wb >= 0)
            for bits in range(1 << n):
                y = [(bits >> i) & 1 for i in range(n)]
                Lm = [a if y[i] else L[i] for i in range(n)]
                rhs = 2 * E0 + sum(int(u[i]) * y[i] for i in range(n))
                rhs += sum(int(Wb[o, i]) * abs(y[i] - y[j]) for o, i, j in edges)
                assert 2 * _energy_loop(D, V, Lm, dims, ndim, conn) == rhs


def _brute_min(D, V, dims, ndim, conn, nl):
    n = D.shape[1]
    best = None
    for L in itertools.product(range(nl), repeat=n):
        e = _energy_loop(D, V, np.array(L), dims, ndim, conn)
        best = e if best is None or e < best else best
    return best


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_exact_moves_within_factor_two_and_locally_optimal(seed):
    dims, ndim, conn, nl = (3, 3, 1), 2, 8, 3
    D, V = _tiny(10 + seed, dims, ndim, conn, nl, d_max=40, v_max=40)
    tmpl = multilabel_image(seed=0, W=3, H=3, n_labels=nl, conn=conn, block=(3, 3), overlap=(0, 0)).template
    L, E, recs = ml.alpha_expansion(tmpl, D, V, max_cycles=10, move_solver=ml.exact_move_solver)
    Emin = _brute_min(D, V, dims, ndim, conn, nl)
    assert Emin <= E <= 2 * Emin
    energies = [r.energy for r in recs]
    assert all(b <= a for a, b in zip(energies, energies[1:]))
    n = D.shape[1]
    for a in range(nl):
        for bits in range(1 << n):
            Lm = np.array([a if (bits >> i) & 1 else L[i] for i in range(n)])
            assert _energy_loop(D, V, Lm, dims, ndim, conn) >= E


def test_one_block_dope_moves_equal_exact_moves():
    """One block: DOPE's first iteration is the global minimal min cut of each move, so the two loops agree move
    by move."""
    p = multilabel_image(seed=5, W=20, H=16, n_labels=3, conn=8, block=(32, 32), overlap=(0, 0))
    L1, E1, r1 = ml.alpha_expansion(p.template, p.D, p.V, max_cycles=4)
    L2, E2, r2 = ml.alpha_expansion(p.template, p.D, p.V, max_cycles=4, move_solver=ml.exact_move_solver)
    assert E1 == E2 and np.array_equal(L1, L2)
    assert [(r.label, r.accepted, r.energy) for r in r1] == [(r.label, r.accepted, r.energy) for r in r2]
    assert all(r.binary_iterations == 1 for r in r1)


def test_dope_moves_lower_the_energy_and_track_exact_moves():
    p = multilabel_image(seed=6, W=48, H=40, n_labels=4, conn=8, block=(16, 16), overlap=(2, 2))
    L0 = ml.initial_labels(p.D)
    E0 = ml.energy(p.D, p.V, L0, p.template.dims, 2, 8)
    L, E, recs = ml.alpha_expansion(p.template, p.D, p.V, max_cycles=4)
    _, Eex, _ = ml.alpha_expansion(p.template, p.D, p.V, max_cycles=4, move_solver=ml.exact_move_solver)
    energies = [E0] + [r.energy for r in recs]
    assert all(b <= a for a, b in zip(energies, energies[1:]))
    assert E < E0
    assert E <= Eex * 1.01   # DOPE moves are approximate; on this image they end within 1 % of exact moves
