"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each test names the passage it checks.  None of them re-types the oracle's own formula: they use exact
rational identities from the proof of Theorem 1, closed forms derived by hand from the matrix definitions,
a generic least-squares solve for Eq. (10), brute-force enumeration for the block solver, and special cases
whose answer is known in closed form.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import dope

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# --------------------------------------------------------------------------------------------------------
# helpers written independently of the oracle's matrix code
# --------------------------------------------------------------------------------------------------------

def neighbours(problem):
    """dict i -> list of (j, w_ij) from the half-stencil arrays directly (full stencil)."""
    W_, H_, D_ = problem.dims
    nb = {i: [] for i in range(problem.n)}
    for o, (dx, dy, dz) in enumerate(synth.half_stencil(problem.ndim, problem.conn)):
        for i in range(problem.n):
            wv = int(problem.w[o][i])
            if wv == 0:
                continue
            x, y, z = i % W_, (i // W_) % H_, i // (W_ * H_)
            j = (x + dx) + W_ * ((y + dy) + H_ * (z + dz))
            nb[i].append((j, wv))
            nb[j].append((i, wv))
    return nb


def block_sets(problem):
    blocks = dope.make_blocks(problem.dims, problem.block, problem.overlap)
    return [list(map(int, b.idx)) for b in blocks]


def multiplicities(problem, bsets):
    q = [0] * problem.n
    for b in bsets:
        for i in b:
            q[i] += 1
    return q


def tiny_problem(seed, dims, conn, block, overlap, neg_frac=0.0):
    return synth.random_problem(seed, dims, conn, block, overlap, lam_q8=384, u_range=(-900, 900),
                                w_range=(0, 700), neg_frac=neg_frac)


TINY = [
    ((5, 7, 1), 4, (3, 3, 1), (1, 1, 0)),
    ((7, 5, 1), 8, (3, 4, 1), (1, 1, 0)),
    ((6, 6, 1), 4, (4, 4, 1), (0, 0, 0)),
    ((9, 7, 1), 8, (5, 5, 1), (2, 2, 0)),
    ((4, 4, 4), 6, (3, 3, 3), (1, 1, 1)),
    ((5, 4, 3), 6, (3, 2, 2), (1, 0, 0)),
    ((7, 7, 1), 24, (4, 4, 1), (1, 1, 0)),     # 5x5 neighbourhood, stride 3 >= radius 2
    ((8, 7, 1), 48, (5, 5, 1), (2, 2, 0)),     # 7x7 neighbourhood, stride 3 = radius 3
    ((5, 4, 4), 32, (3, 3, 3), (1, 1, 1)),     # 3D ball of radius 2, stride 2 = radius
    ((9, 8, 1), 80, (6, 6, 1), (2, 2, 0)),     # 9x9 neighbourhood, stride 4 = radius 4
    ((6, 5, 5), 122, (4, 4, 4), (1, 1, 1)),    # 3D ball of radius 3, stride 3 = radius
    ((7, 6, 6), 256, (5, 5, 5), (1, 1, 1)),    # 3D ball of radius 4, stride 4 = radius
]


@pytest.mark.parametrize("conn,r", [(24, 2), (48, 3), (80, 4)])
def test_square_neighbourhood_offsets(conn, r):
    """The larger neighbourhoods of the experiments (square kernels of size 5 and 7): the half-stencil and its
    negation partition the (2r+1)^2 square without its centre, so every undirected edge appears exactly once."""
    half = dope.neighbour_offsets(2, conn)
    full = half + [(-dx, -dy, -dz) for dx, dy, dz in half]
    square = [(dx, dy, 0) for dy in range(-r, r + 1) for dx in range(-r, r + 1) if (dx, dy) != (0, 0)]
    assert len(half) == len(set(half)) == (len(square)) // 2
    assert sorted(full) == sorted(square)


@pytest.mark.parametrize("conn,r,count", [(32, 2, 32), (122, 3, 122), (256, 4, 256)])
def test_ball_neighbourhood_offsets(conn, r, count):
    """The spherical kernels of size 5, 7 and 9 in 3D: the half-stencil and its negation partition the lattice
    points of the radius-r ball without its centre."""
    half = dope.neighbour_offsets(3, conn)
    full = half + [(-dx, -dy, -dz) for dx, dy, dz in half]
    ball = [(x, y, z) for x in range(-r, r + 1) for y in range(-r, r + 1) for z in range(-r, r + 1)
            if 0 < x * x + y * y + z * z <= r * r]
    assert len(ball) == count and len(half) == len(set(half)) == count // 2
    assert sorted(full) == sorted(ball)


# --------------------------------------------------------------------------------------------------------
# block partition and Proposition 1
# --------------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("N,B,o,count", [(64, 16, 1, 5), (512, 32, 2, 17), (128, 16, 1, 9), (64, 16, 1, 5),
                                          (256, 4, 1, 85), (10, 16, 2, 1), (16, 16, 3, 1), (17, 16, 3, 2)])
def test_partition_counts(N, B, o, count):
    iv = dope.partition_axis(N, B, o)
    assert len(iv) == count
    assert iv[0][0] == 0 and iv[-1][1] == N
    for (a0, a1), (b0, b1) in zip(iv, iv[1:]):
        assert a1 - b0 == o                      # consecutive blocks share exactly o pixels
        assert a1 - a0 == B
    assert iv[-1][1] - iv[-1][0] > o or len(iv) == 1


def test_partition_block_counts_of_workloads():
    for dims, B, o, K in [((64, 64, 1), (16, 16, 1), (1, 1, 0), 25), ((512, 512, 1), (32, 32, 1), (2, 2, 0), 289),
                          ((128, 128, 64), (16, 16, 16), (1, 1, 1), 405), ((256, 256, 1), (4, 4, 1), (1, 1, 0), 7225)]:
        blocks = dope.make_blocks(dims, B, o)
        assert len(blocks) == K
    blocks = dope.make_blocks((64, 64, 1), (16, 16, 1), (1, 1, 0))
    assert sum(len(b.idx) for b in blocks) == 4624


@pytest.mark.parametrize("case", TINY)
def test_q_counts_blocks(case):
    """Q = sum_k S_k^T S_k is diagonal with q_ii = number of blocks containing pixel i (Prop. 1)."""
    dims, conn, block, overlap = case
    p = tiny_problem(1, dims, conn, block, overlap)
    dec = dope.decompose(p)
    bsets = block_sets(p)
    assert list(dec.q) == multiplicities(p, bsets)
    assert set(np.unique(dec.q)) <= {1, 2, 4, 8}


# --------------------------------------------------------------------------------------------------------
# Theorem 1: exact identity of the reformulation at a consistent point
# --------------------------------------------------------------------------------------------------------

def _dense_frac(m, scale=64):
    d = m.toarray()
    return [[Fraction(int(v), scale) for v in row] for row in d]


@pytest.mark.parametrize("case", TINY)
@pytest.mark.parametrize("neg", [0.0, 0.3])
def test_theorem1_identity_exact(case, neg):
    """With y^_k = S_k y, sum_k (u^_k + lam (C_k + R_k S_k) y)^T y^_k + lam sum_k y^_k^T L^_k y^_k equals
    u^T y + lam y^T L y (Eq. 3), for binary y and for real y (Theorem 1, proof in the appendix)."""
    dims, conn, block, overlap = case
    p = tiny_problem(2, dims, conn, block, overlap, neg_frac=neg)
    dec = dope.decompose(p)
    nb = neighbours(p)
    lam = Fraction(p.lam_q8, 256)
    rng = np.random.default_rng(3)
    for trial in range(3):
        if trial == 0:
            y = [Fraction(int(v)) for v in rng.integers(0, 2, p.n)]
        else:
            y = [Fraction(int(v), 7) for v in rng.integers(-7, 15, p.n)]
        # right-hand side: Eq. (3) written from the edge list
        rhs = sum(Fraction(int(p.u[i])) * y[i] for i in range(p.n))
        for i in range(p.n):
            for j, wv in nb[i]:
                if i < j:
                    rhs += lam * wv * (y[i] - y[j]) ** 2
        lhs = Fraction(0)
        for k, blk in enumerate(dec.blocks):
            idx = list(map(int, blk.idx))
            yk = [y[i] for i in idx]
            M = _dense_frac(dec.M64[k])
            What = _dense_frac(dec.W64[k])
            for a, i in enumerate(idx):
                uh = Fraction(int(p.u[i]), int(dec.q[i]))
                g = sum(M[a][j] * y[j] for j in range(p.n) if M[a][j] != 0)
                lhs += (uh + lam * g) * yk[a]
            # y^T L^ y = sum_{a<b} W^_ab (y_a - y_b)^2
            m = len(idx)
            for a in range(m):
                for b in range(a + 1, m):
                    if What[a][b] != 0:
                        lhs += lam * What[a][b] * (yk[a] - yk[b]) ** 2
        assert lhs == rhs


@pytest.mark.parametrize("case", TINY)
def test_coupling_matches_hand_closed_form(case):
    """[(C_k + R_k S_k) y]_i = sum_{j in N(i)} w_ij (q_j - [j in k]) / (q_i q_j) (y_i - y_j), and the transpose
    [(C_k + R_k S_k)^T y^]_m = [m in k] y^_m sum_j w_mj (q_j - [j in k])/(q_m q_j)
                               - (q_m - [m in k]) sum_{i in k, i in N(m)} w_im y^_i / (q_i q_m),
    both derived by hand from the definitions of C_k and R_k in Theorem 1."""
    dims, conn, block, overlap = case
    p = tiny_problem(4, dims, conn, block, overlap, neg_frac=0.2)
    dec = dope.decompose(p)
    nb = neighbours(p)
    bsets = block_sets(p)
    q = multiplicities(p, bsets)
    rng = np.random.default_rng(5)
    y = rng.integers(-50000, 120000, p.n)
    for k, idx in enumerate(bsets):
        ink = set(idx)
        # forward
        got = dec.M64[k] @ y
        for a, i in enumerate(idx):
            exp = Fraction(0)
            for j, wv in nb[i]:
                exp += Fraction(wv * (q[j] - (j in ink)), q[i] * q[j]) * int(y[i] - y[j])
            assert Fraction(int(got[a]), 64) == exp
        # transpose
        yh = rng.integers(0, 2, len(idx))
        got_t = dec.M64[k].T @ yh
        pos = {i: a for a, i in enumerate(idx)}
        for m in range(p.n):
            exp = Fraction(0)
            if m in ink:
                exp += int(yh[pos[m]]) * sum(Fraction(wv * (q[j] - (j in ink)), q[m] * q[j]) for j, wv in nb[m])
            exp -= (q[m] - (m in ink)) * sum(Fraction(wv * int(yh[pos[i]]), q[i] * q[m])
                                              for i, wv in nb[m] if i in ink)
            assert Fraction(int(got_t[m]), 64) == exp


def test_chain_micro_example():
    """Chain 1-2-3 (weights 5 and 7), blocks {1,2} and {2,3}, q = (1, 2, 1):
    g_{1,1} = (w12/2)(y1 - y2), g_{1,2} = (w23/2)(y2 - y3), g_{2,2} = (w12/2)(y2 - y1), g_{2,3} = (w23/2)(y3 - y2)."""
    p = synth.Problem("chain3", (3, 1, 1), 2, 4, np.zeros(3, np.int32),
                      np.array([[5, 7, 0], [0, 0, 0]], np.int32), 256, (2, 1, 1), (1, 0, 0), 1000)
    dec = dope.decompose(p)
    assert list(dec.q) == [1, 2, 1]
    y = np.array([3, 11, 2], dtype=np.int64)
    g1 = dec.M64[0] @ y
    g2 = dec.M64[1] @ y
    assert [Fraction(int(v), 64) for v in g1] == [Fraction(5, 2) * (3 - 11), Fraction(7, 2) * (11 - 2)]
    assert [Fraction(int(v), 64) for v in g2] == [Fraction(5, 2) * (11 - 3), Fraction(7, 2) * (2 - 11)]


# --------------------------------------------------------------------------------------------------------
# Eq. (10) is the minimiser of Eq. (9); Eq. (11) update
# --------------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("case", TINY[:4])
def test_eq10_is_least_squares_minimiser(case):
    """Minimise lam sum_k y^_k^T M_k y + mu/2 sum_k ||S_k y - (y^_k + a_k)||^2 with a generic least-squares
    solver (the objective is written as an augmented least-squares system); the oracle's Q16.16 update must
    equal floor(2^16 y*) up to the solver's rounding."""
    dims, conn, block, overlap = case
    p = tiny_problem(6, dims, conn, block, overlap)
    dec = dope.decompose(p)
    rng = np.random.default_rng(7)
    tot = int(dec.offsets[-1])
    yhat = rng.integers(0, 2, tot).astype(np.uint8)
    A = rng.integers(-40000, 40000, tot).astype(np.int64)
    M = 1234
    lam = p.lam_q8 / 256.0
    # stack rows sqrt(mu/2) (S_k y - b_k) and fold the linear term into the least-squares target:
    # lam g^T y + mu/2 ||S y - b||^2 = mu/2 ||S y - (b - lam/mu Q^-1-free correction)||^2 is not separable,
    # so solve the normal equations of the full quadratic with lstsq on [sqrt(mu) S] and target.
    rows, tgt = [], []
    lin = np.zeros(p.n)
    for k, Sk in enumerate(dec.S):
        a, b = dec.offsets[k], dec.offsets[k + 1]
        Sd = Sk.toarray().astype(float)
        rows.append(np.sqrt(M) * Sd)
        tgt.append(np.sqrt(M) * (yhat[a:b] + A[a:b] / 65536.0))
        lin += lam * (dec.M64[k].T @ yhat[a:b].astype(np.int64)) / 64.0
    Amat = np.vstack(rows)
    # gradient: Amat^T Amat y - Amat^T t + lin = 0  ->  least squares with shifted target
    t = np.concatenate(tgt)
    shift = np.linalg.lstsq(Amat.T, lin, rcond=None)[0]    # Amat^T shift = lin
    ystar = np.linalg.lstsq(Amat, t - shift, rcond=None)[0]
    got = dope.consensus(dec, yhat, A, M)
    assert np.all(np.abs(got - np.floor(ystar * 65536.0)) <= 1)


def test_iteration_applies_eq11():
    p = tiny_problem(8, (9, 7, 1), 8, (5, 5, 1), (2, 2, 0))
    dec = dope.decompose(p)
    st = dope.initial_state(dec, 1500)
    new, _ = dope.iterate(dec, st, threads=1)
    for k, Sk in enumerate(dec.S):
        a, b = dec.offsets[k], dec.offsets[k + 1]
        assert np.array_equal(new.A[a:b], st.A[a:b] + 65536 * new.yhat[a:b].astype(np.int64) - Sk @ new.Y)
    assert new.M == 1500 * 21 // 20


# --------------------------------------------------------------------------------------------------------
# block sub-problem solvers against brute force and duality
# --------------------------------------------------------------------------------------------------------

def brute_minimisers(un, edges):
    n = len(un)
    best, sols = None, []
    for code in range(1 << n):
        x = [(code >> i) & 1 for i in range(n)]
        e = sum(un[i] * x[i] for i in range(n)) + sum(c * abs(x[a] - x[b]) for a, b, c in edges)
        if best is None or e < best:
            best, sols = e, [code]
        elif e == best:
            sols.append(code)
    return best, sols


def random_subproblem(rng, n, allow_neg=False, tie_prone=False):
    scale = 3 if tie_prone else 1000
    un = rng.integers(-scale, scale + 1, n)
    edges = []
    for a in range(n):
        for b in range(a + 1, n):
            if rng.random() < 0.35:
                c = int(rng.integers(0, scale + 1))
                if allow_neg and rng.random() < 0.3:
                    c = -c
                edges.append((a, b, c))
    return un, edges


@pytest.mark.parametrize("seed", range(60))
def test_mincut_is_minimal_minimiser(seed):
    """Max-flow labels = the intersection of all minimisers = the smallest-code minimiser; and
    max-flow value - sum_{un<0} |un| = minimum energy (max-flow / min-cut duality)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 12))
    un, edges = random_subproblem(rng, n, tie_prone=(seed % 2 == 0))
    ea = np.array([e[0] for e in edges], np.int32)
    eb = np.array([e[1] for e in edges], np.int32)
    cap = np.array([e[2] for e in edges], np.int64)
    x, flow = dope.solve_subproblem(un, ea, eb, cap, "maxflow")
    best, sols = brute_minimisers(list(map(int, un)), edges)
    inter = (1 << n) - 1
    for s in sols:
        inter &= s
    code = sum(int(x[i]) << i for i in range(n))
    assert code == inter == min(sols)
    assert flow - int(np.sum(np.maximum(-un, 0))) == best


@pytest.mark.parametrize("seed", range(30))
def test_enumeration_smallest_code(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 11))
    un, edges = random_subproblem(rng, n, allow_neg=True, tie_prone=(seed % 3 == 0))
    ea = np.array([e[0] for e in edges], np.int32)
    eb = np.array([e[1] for e in edges], np.int32)
    cap = np.array([e[2] for e in edges], np.int64)
    x, emin = dope.solve_subproblem(un, ea, eb, cap, "exhaustive")
    best, sols = brute_minimisers(list(map(int, un)), edges)
    assert emin == best
    assert sum(int(x[i]) << i for i in range(n)) == min(sols)


def test_maxflow_rejects_non_submodular():
    """Footnote of Sec. 1: a negative pairwise weight breaks submodularity; the graph-cut solver refuses it."""
    with pytest.raises(ValueError):
        dope.solve_subproblem(np.array([1, -1]), np.array([0], np.int32), np.array([1], np.int32),
                              np.array([-5], np.int64), "maxflow")


# --------------------------------------------------------------------------------------------------------
# energy, global min cut
# --------------------------------------------------------------------------------------------------------

def test_energy_definition_eq1():
    p = tiny_problem(9, (6, 5, 1), 8, (3, 3, 1), (1, 1, 0), neg_frac=0.3)
    nb = neighbours(p)
    rng = np.random.default_rng(1)
    for _ in range(5):
        l = rng.integers(0, 2, p.n).astype(np.uint8)
        exp = 256 * sum(int(p.u[i]) * int(l[i]) for i in range(p.n))
        exp += p.lam_q8 * sum(wv * abs(int(l[i]) - int(l[j])) for i in range(p.n) for j, wv in nb[i] if i < j)
        assert dope.energy_q(p, l) == exp


@pytest.mark.parametrize("seed", range(8))
def test_global_mincut_vs_bruteforce(seed):
    p = tiny_problem(20 + seed, (4, 3, 1), [4, 8, 24, 48][seed % 4], (2, 2, 1), (0, 0, 0))
    x, e = dope.global_mincut(p)
    best, sols = None, []
    for code in range(1 << p.n):
        l = np.array([(code >> i) & 1 for i in range(p.n)], np.uint8)
        v = dope.energy_q(p, l)
        if best is None or v < best:
            best, sols = v, [code]
        elif v == best:
            sols.append(code)
    assert e == best
    assert sum(int(x[i]) << i for i in range(p.n)) == min(sols)


# --------------------------------------------------------------------------------------------------------
# special cases of Algorithm 1
# --------------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("conn,dims", [(4, (7, 6, 1)), (8, (6, 6, 1)), (6, (4, 3, 3)), (24, (6, 5, 1)),
                                       (48, (6, 6, 1)), (32, (4, 4, 3)), (80, (6, 5, 1)), (122, (4, 4, 4)),
                                       (256, (4, 4, 4))])
def test_single_block_is_global_cut(conn, dims):
    """K = 1: C = R = 0, so iteration 1 solves Eq. (3) exactly; y = y^ and the residual is 0 (stop at t = 1)."""
    p = tiny_problem(30, dims, conn, (0, 0, 0), (0, 0, 0))
    st, infos, _, dec = dope.run(p)
    assert len(infos) == 1 and infos[0].converged
    x, _ = dope.global_mincut(p)
    assert np.array_equal(st.yhat, x)
    assert np.array_equal(st.Y, 65536 * x.astype(np.int64))
    assert np.all(st.A == 0)


def test_zero_pairwise_gives_unary_sign():
    """w = 0: every block problem is separable; labels = [u < 0] (ties at u = 0 -> 0), converged at t = 1."""
    p = tiny_problem(31, (9, 8, 1), 8, (4, 4, 1), (1, 1, 0))
    p.w[:] = 0
    p.u[::7] = 0
    st, infos, _, dec = dope.run(p)
    assert len(infos) == 1 and infos[0].converged
    assert np.array_equal(dope.labels(st.Y), (p.u < 0).astype(np.uint8))


@pytest.mark.parametrize("case", TINY)
def test_first_iteration_blocks_are_independent(case):
    """At y = 1/2, a = 0 (Alg. 1 initialisation) the coupling and the mu-term vanish: block k solves
    min sum_i 2^14 u_i/q_i y_i + sum_{(i,j) in k} lambda_q 64 w_ij/(q_i q_j) |y_i - y_j| (built here by loops)."""
    dims, conn, block, overlap = case
    p = tiny_problem(32, dims, conn, block, overlap)
    dec = dope.decompose(p)
    st = dope.initial_state(dec, 777)
    new, _ = dope.iterate(dec, st, threads=1)
    nb = neighbours(p)
    bsets = block_sets(p)
    q = multiplicities(p, bsets)
    for k, idx in enumerate(bsets):
        pos = {i: a for a, i in enumerate(idx)}
        un = np.array([(1 << 14) * int(p.u[i]) // q[i] for i in idx], np.int64)
        ea, eb, cap = [], [], []
        for i in idx:
            for j, wv in nb[i]:
                if i < j and j in pos:
                    ea.append(pos[i]); eb.append(pos[j]); cap.append(p.lam_q8 * wv * 64 // (q[i] * q[j]))
        x, _ = dope.solve_subproblem(un, np.array(ea, np.int32), np.array(eb, np.int32), np.array(cap, np.int64))
        assert np.array_equal(new.yhat[dec.offsets[k]:dec.offsets[k + 1]], x)


def test_overflow_detected_with_tiny_mu():
    """A tiny mu makes the lambda/mu term of Eq. (10) blow up: the run stops with an overflow flag and clamped state."""
    p = synth.config1(mu0=1)
    st, infos, _, _ = dope.run(p, n_iter=10)
    assert infos[-1].overflow
    assert np.max(np.abs(st.Y)) <= 1 << 22 and np.max(np.abs(st.A)) <= 1 << 22


def test_mu_schedule():
    M, seq = 1000, []
    for _ in range(5):
        M = dope.next_mu(M)
        seq.append(M)
    assert seq == [1050, 1102, 1157, 1214, 1274]
    assert dope.next_mu((1 << 24) - 1) == (1 << 24) - 1


# --------------------------------------------------------------------------------------------------------
# fixed-point loop against a real-valued float64 implementation written from Eq. (8), (10), (11)
# --------------------------------------------------------------------------------------------------------

def float_dope(p, iters):
    """Real-valued Algorithm 1 using the hand closed forms of the coupling terms (independent of the oracle)."""
    nb = neighbours(p)
    bsets = block_sets(p)
    q = multiplicities(p, bsets)
    lam = p.lam_q8 / 256.0
    mu = float(p.mu0)
    y = np.full(p.n, 0.5)
    a = [np.zeros(len(b)) for b in bsets]
    hist = []
    for _ in range(iters):
        yh = []
        for k, idx in enumerate(bsets):
            ink = set(idx)
            pos = {i: t for t, i in enumerate(idx)}
            un = np.zeros(len(idx))
            ea, eb, cap = [], [], []
            for t, i in enumerate(idx):
                g = sum(wv * (q[j] - (j in ink)) / (q[i] * q[j]) * (y[i] - y[j]) for j, wv in nb[i])
                un[t] = p.u[i] / q[i] + lam * g + mu * (a[k][t] - y[i] + 0.5)
                for j, wv in nb[i]:
                    if i < j and j in pos:
                        ea.append(t); eb.append(pos[j]); cap.append(lam * wv / (q[i] * q[j]))
            # solve with the oracle's integer solver after a fine scaling (labels only)
            x, _ = dope.solve_subproblem(np.round(un * 2 ** 20).astype(np.int64), np.array(ea, np.int32),
                                         np.array(eb, np.int32), np.round(np.array(cap) * 2 ** 20).astype(np.int64))
            yh.append(x.astype(float))
        num = np.zeros(p.n)
        for k, idx in enumerate(bsets):
            ink = set(idx)
            pos = {i: t for t, i in enumerate(idx)}
            for t, i in enumerate(idx):
                num[i] += mu * (yh[k][t] + a[k][t])
            for m in range(p.n):
                h = 0.0
                if m in ink:
                    h += yh[k][pos[m]] * sum(wv * (q[j] - (j in ink)) / (q[m] * q[j]) for j, wv in nb[m])
                h -= (q[m] - (m in ink)) * sum(wv * yh[k][pos[i]] / (q[i] * q[m]) for i, wv in nb[m] if i in ink)
                num[m] -= lam * h
        y = num / (mu * np.array(q))
        for k, idx in enumerate(bsets):
            a[k] = a[k] + yh[k] - y[idx]
        mu = mu * 1.05
        hist.append((np.concatenate(yh), y.copy()))
    return hist


def test_fixed_point_tracks_real_valued_loop():
    p = synth.config1(size=24, mu0=1000)
    p.block, p.overlap = (8, 8, 1), (1, 1, 0)
    st, infos, states, dec = dope.run(p, n_iter=3, record=True)
    hist = float_dope(p, 3)
    for t in range(3):
        yh_f, y_f = hist[t]
        assert np.array_equal(states[t].yhat, yh_f.astype(np.uint8))
        assert np.max(np.abs(states[t].Y / 65536.0 - y_f)) < 1e-3


def test_energy_gap_invariant_and_quality():
    """E_dope >= E_GC (the global cut is optimal); the paper reports Dice > 0.99 and small Delta E in 2D."""
    p = synth.config1()
    st, infos, _, dec = dope.run(p, n_iter=10)
    l = dope.labels(st.Y)
    x, egc = dope.global_mincut(p)
    e = dope.energy_q(dec, l)
    assert e >= egc
    assert (e - egc) / abs(egc) < 0.01
    assert 2 * np.sum(l & x) / (np.sum(l) + np.sum(x)) > 0.99


# --------------------------------------------------------------------------------------------------------
# the stopping rule of Algorithm 1 (its while-condition on the per-block residuals)
# --------------------------------------------------------------------------------------------------------

def _no_pairwise_problem():
    """8x8 grid, 4-connected, w = 0, 4x4 blocks with 1-pixel overlap (2 x 2 blocks); with w = 0 Eq. (10) is the
    plain average of the copies: Y_m = floor(sum_k (2^16 yhat_k,m + A_k,m) / q_m)."""
    p = tiny_problem(41, (8, 8, 1), 4, (5, 5, 1), (2, 2, 0))
    p.w[:] = 0
    return p


def _copy_index(dec, k, pixel):
    return int(dec.offsets[k] + list(dec.blocks[k].idx).index(pixel))


@pytest.mark.parametrize("vals", [(5,), (3, 4), (6, 0, 8)])
def test_stopping_threshold_is_eps_squared(vals):
    """Block 0 gets multipliers v on pixels that lie in it alone (q = 1); with yhat = 0 and w = 0 the new Y of
    those pixels is v (Eq. 10), every other copy is consistent, so r_0 = sum v^2 and r_k = 0 elsewhere.  The loop
    stops iff max_k r_k <= eps^2: eps = sqrt(sum v^2) stops (equality included), one less does not."""
    p = _no_pairwise_problem()
    dec = dope.decompose(p)
    st = dope.initial_state(dec, 1000)
    st.Y[:] = 0
    interior = [i for i in dec.blocks[0].idx if dec.q[i] == 1]
    for v, pix in zip(vals, interior):
        st.A[_copy_index(dec, 0, int(pix))] = v
    yz = np.zeros_like(st.yhat)
    R = sum(v * v for v in vals)
    eps = int(round(R ** 0.5))
    assert eps * eps == R
    new, info = dope.iterate(dec, st, yhat_override=yz, eps_q16=eps)
    assert info.resid2[0] == R and np.all(info.resid2[1:] == 0)
    assert info.converged
    _, info = dope.iterate(dec, st, yhat_override=yz, eps_q16=eps - 1)
    assert not info.converged
    if R > 1:
        # a threshold of eps instead of eps^2 would not stop here
        assert R > eps


def test_residual_of_shared_pixel_counts_in_every_block():
    """A pixel in two blocks (q = 2) with multipliers 6 and 10 gets Y = floor(16 / 2) = 8 (Eq. 10 with w = 0); both
    blocks' residuals hold (0 - 8)^2 = 64 and the multipliers become 6 - 8 and 10 - 8 (Eq. 11)."""
    p = _no_pairwise_problem()
    dec = dope.decompose(p)
    st = dope.initial_state(dec, 1000)
    st.Y[:] = 0
    shared = [i for i in dec.blocks[0].idx if dec.q[i] == 2 and i in set(dec.blocks[1].idx)][0]
    c0, c1 = _copy_index(dec, 0, int(shared)), _copy_index(dec, 1, int(shared))
    st.A[c0], st.A[c1] = 6, 10
    new, info = dope.iterate(dec, st, yhat_override=np.zeros_like(st.yhat), eps_q16=7)
    assert new.Y[shared] == 8
    assert info.resid2[0] == 64 and info.resid2[1] == 64 and np.all(info.resid2[2:] == 0)
    assert new.A[c0] == -2 and new.A[c1] == 2
    assert not info.converged          # 64 > 7^2
    _, info = dope.iterate(dec, st, yhat_override=np.zeros_like(st.yhat), eps_q16=8)
    assert info.converged              # 64 <= 8^2


@pytest.mark.parametrize("case", TINY[:6])
def test_block_residuals_by_hand(case):
    """After two iterations of a random problem, r_k = sum over the pixels of block k of (2^16 yhat_k,i - Y_i)^2,
    summed here by plain loops over the block's pixel list."""
    dims, conn, block, overlap = case
    p = tiny_problem(43, dims, conn, block, overlap)
    dec = dope.decompose(p)
    st = dope.initial_state(dec, 900)
    st, _ = dope.iterate(dec, st, threads=1)
    new, info = dope.iterate(dec, st, threads=1, eps_q16=6554)
    for k, idx in enumerate(block_sets(p)):
        a = int(dec.offsets[k])
        r = 0
        for t, i in enumerate(idx):
            d = 65536 * int(new.yhat[a + t]) - int(new.Y[i])
            r += d * d
        assert info.resid2[k] == r
    assert info.converged == (max(int(x) for x in info.resid2) <= 6554 * 6554)


# --------------------------------------------------------------------------------------------------------
# non-convergence on the 64x64 disk is the method's: a real-valued Algorithm 1 settles in the same 2-cycle
# --------------------------------------------------------------------------------------------------------

def float_dope_vectorised(p, iters):
    """Real-valued (float64) Algorithm 1 on sparse matrices built from the hand closed forms of Theorem 1's
    coupling term: g_k(y) = G_k y with G_k[i, i] += c, G_k[i, j] -= c, c = w_ij (q_j - [j in k]) / (q_i q_j);
    Eq. (10) uses G_k^T yhat_k.  Block problems are solved with real unaries and capacities scaled by 2^20 and
    rounded (labels only).  Returns per iteration (block labels, y, per-block residuals ||yhat_k - S_k y||^2)."""
    import scipy.sparse as sps
    nb = neighbours(p)
    bsets = block_sets(p)
    q = np.array(multiplicities(p, bsets), float)
    lam = p.lam_q8 / 256.0
    G, S, edges = [], [], []
    for idx in bsets:
        ink = set(idx)
        pos = {i: t for t, i in enumerate(idx)}
        rows, cols, vals = [], [], []
        ea, eb, cap = [], [], []
        for t, i in enumerate(idx):
            for j, wv in nb[i]:
                c = wv * (q[j] - (j in ink)) / (q[i] * q[j])
                rows += [t, t]
                cols += [i, j]
                vals += [c, -c]
                if i < j and j in pos:
                    ea.append(t); eb.append(pos[j]); cap.append(lam * wv / (q[i] * q[j]))
        G.append(sps.csr_matrix((vals, (rows, cols)), shape=(len(idx), p.n)))
        S.append(sps.csr_matrix((np.ones(len(idx)), (np.arange(len(idx)), idx)), shape=(len(idx), p.n)))
        edges.append((np.array(ea, np.int32), np.array(eb, np.int32),
                      np.round(np.array(cap) * 2 ** 20).astype(np.int64)))
    u = np.asarray(p.u, float)
    mu = float(p.mu0)
    y = np.full(p.n, 0.5)
    a = [np.zeros(len(b)) for b in bsets]
    hist = []
    for _ in range(iters):
        yh = []
        for k, idx in enumerate(bsets):
            un = u[idx] / q[idx] + lam * (G[k] @ y) + mu * (a[k] - y[idx] + 0.5)
            x, _ = dope.solve_subproblem(np.round(un * 2 ** 20).astype(np.int64), *edges[k])
            yh.append(x.astype(float))
        num = np.zeros(p.n)
        for k in range(len(bsets)):
            num += S[k].T @ (mu * (yh[k] + a[k])) - lam * (G[k].T @ yh[k])
        y = num / (mu * q)
        r = []
        for k, idx in enumerate(bsets):
            a[k] = a[k] + yh[k] - y[idx]
            r.append(float(np.sum((yh[k] - y[idx]) ** 2)))
        mu *= 1.05
        hist.append((np.concatenate(yh).astype(np.uint8), y.copy(), np.array(r)))
    return hist


def test_disk_two_cycle_is_the_methods():
    """On the 64x64 disk (16x16 blocks, o = 1, mu0 = 1000) the fixed-point loop never meets eps = 0.1: from
    iteration 7 the same few overlap copies flip every iteration (block labels repeat with period 2) and
    sqrt(max_k r_k) stays near 0.71.  A real-valued float64 Algorithm 1 settles into the same 2-cycle with the
    same residual, so the stall belongs to Algorithm 1 on this input, not to the Q16.16 reading."""
    p = synth.config1()
    n_it = 40
    _, infos, states, _ = dope.run(p, n_iter=n_it, record=True)
    hist = float_dope_vectorised(p, n_it)
    for t in range(20, n_it):
        fx_res = np.sqrt(np.max(infos[t].resid2)) / 65536.0
        fl_res = np.sqrt(np.max(hist[t][2]))
        assert 0.6 < fx_res < 0.8 and 0.6 < fl_res < 0.8, (t, fx_res, fl_res)
        assert abs(fx_res - fl_res) < 0.01
        # period 2, and a real flip each iteration
        assert np.array_equal(states[t].yhat, states[t - 2].yhat)
        assert not np.array_equal(states[t].yhat, states[t - 1].yhat)
        assert np.array_equal(hist[t][0], hist[t - 2][0])
        assert not np.array_equal(hist[t][0], hist[t - 1][0])
    # the two loops flip the same copies
    assert np.array_equal(states[n_it - 1].yhat, hist[n_it - 1][0])
