"""ORACLE — test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg import this module.  The product
library never imports, links or calls it, and it shares no code with the GPU path: the two meet only in the
seeded input generators of the ``synth`` package.

A plain, slow, obviously-correct CPU implementation of the DOPE iteration (Algorithm 1), written in the
paper's own notation.  The per-block parameters of Theorem 1 are formed literally as the sparse matrix
products that define them:

    Q      = sum_k S_k^T S_k                                       (Proposition 1, Eq. 4)
    u^_k   = S_k Q^-1 u                                            (Theorem 1)
    W^_k   = S_k Q^-1 W Q^-1 S_k^T,  D^_k = diag(row sums of W^_k),  L^_k = D^_k - W^_k
    C_k    = S_k Q^-1 L (I - Q^-1 S_k^T S_k)
    R_k    = S_k Q^-1 D Q^-1 S_k^T - D^_k

and the loop takes the steps of Algorithm 1 in order: block solves of Eq. (8), the y update of Eq. (10),
the multiplier update of Eq. (11), mu <- mu * mu_fact.

Fixed-point reading (the paper is real-valued; these constants make every step an exact integer operation):
  * y and a are held as Q16.16 integers Y = 2^16 y, A = 2^16 a; mu is an integer M in input-energy units;
    lambda = lambda_q / 256.
  * Since q_i in {1, 2, 4, 8}, 64 * C_k, 64 * R_k and 64 * W^_k are integer matrices; the code builds them as
    S_k (8Q^-1) L (8I - 8Q^-1 S_k^T S_k) and so on.
  * Block problem = 2^14 x (Eq. 8) with only the unary floored:
        U~_k = 2^14 u^_k + floor( (lambda_q * (64 M_k) Y + 2^14 M (A_k - S_k Y + 2^15)) / 2^16 ),
        pairwise capacities lambda_q * (64 W^_k)_ij,        where M_k = C_k + R_k S_k.
    The returned block labelling is the unique minimal minimiser (label 1 = source side of the minimal
    minimum cut) for max-flow blocks, and the smallest-code minimiser for enumerated blocks.
  * Y <- floor( 2^16 x (Eq. 10) ) = floor( (M * sum_k S_k^T (2^16 y^_k + A_k) - 4 lambda_q sum_k (64 M_k)^T y^_k)
                                            / (M q) ).
  * A_k <- A_k + 2^16 y^_k - S_k Y                          (Eq. 11, exact).
  * Stop when max_k sum_{i in block k} (2^16 y^_k,i - Y_i)^2 <= eps_q^2 (the while-condition of Algorithm 1,
    tested after each full iteration).  Overflow when any |Y| or |A| >= 2^22 (values are then stored clamped
    to +-2^22 and the run stops).
  * M <- min(floor(M * num / den), 2^24 - 1)                 (mu_fact = num / den, default 21/20).
  * Output labels l_i = [Y_i > 2^15]; energy E_q = 256 u^T l + lambda_q l^T L l = 2^8 x (Eq. 1 / Eq. 3).

Block partition (the paper leaves the grow direction and clipping unstated): per axis of length N, block edge
B and overlap 0 <= o <= B/2: stride s = B - o, count 1 + max(0, ceil((N - B) / s)), block t covers
[t s, min(t s + B, N)).  Blocks are Cartesian products of these intervals, ordered x-fastest.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import concurrent.futures as cf
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
Y_ONE = 1 << 16
Y_HALF = 1 << 15
STATE_LIMIT = 1 << 22
MU_MAX = (1 << 24) - 1

_lib = None


def _solvers():
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "_solvers.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        for name in ("oracle_mincut", "oracle_enumerate"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i32p, i32p, i64p, u8p, i64p]
            f.restype = ctypes.c_int
        lib.oracle_objective.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i32p, i32p, i64p, u8p]
        lib.oracle_objective.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ----------------------------------------------------------------------------------------------------------
# Binary sub-problem solvers (the role the BK algorithm plays in the paper, Sec. 2 after Eq. 8)
# ----------------------------------------------------------------------------------------------------------

def solve_subproblem(un: np.ndarray, ea: np.ndarray, eb: np.ndarray, cap: np.ndarray,
                     method: str = "maxflow") -> Tuple[np.ndarray, int]:
    """Minimise sum un_i x_i + sum_e cap_e |x_a - x_b|.  Returns (x uint8, flow or min energy)."""
    un = np.ascontiguousarray(un, dtype=np.int64)
    ea = np.ascontiguousarray(ea, dtype=np.int32)
    eb = np.ascontiguousarray(eb, dtype=np.int32)
    cap = np.ascontiguousarray(cap, dtype=np.int64)
    x = np.zeros(len(un), dtype=np.uint8)
    val = ctypes.c_int64(0)
    lib = _solvers()
    f = lib.oracle_mincut if method == "maxflow" else lib.oracle_enumerate
    rc = f(len(un), _ptr(un, ctypes.c_int64), len(ea), _ptr(ea, ctypes.c_int32), _ptr(eb, ctypes.c_int32),
           _ptr(cap, ctypes.c_int64), _ptr(x, ctypes.c_uint8), ctypes.byref(val))
    if rc == -4:
        raise ValueError("negative pairwise capacity: the max-flow solver needs a submodular block")
    if rc != 0:
        raise RuntimeError(f"oracle solver failed rc={rc}")
    return x, int(val.value)


def subproblem_objective(un, ea, eb, cap, x) -> int:
    un = np.ascontiguousarray(un, dtype=np.int64)
    ea = np.ascontiguousarray(ea, dtype=np.int32)
    eb = np.ascontiguousarray(eb, dtype=np.int32)
    cap = np.ascontiguousarray(cap, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.uint8)
    return int(_solvers().oracle_objective(len(un), _ptr(un, ctypes.c_int64), len(ea), _ptr(ea, ctypes.c_int32),
                                            _ptr(eb, ctypes.c_int32), _ptr(cap, ctypes.c_int64),
                                            _ptr(x, ctypes.c_uint8)))


# ----------------------------------------------------------------------------------------------------------
# Problem structure: W, L = D - W (Eq. 3), blocks Omega_k and selectors S_k (Sec. 2), Q (Eq. 4)
# ----------------------------------------------------------------------------------------------------------

def neighbour_offsets(ndim: int, conn: int):
    """Half-stencil offsets: each undirected edge i <-> i + offset once (the neighbourhood of Sec. 1's grid
    graphs; the experiments' square kernels of size 3, 5, 7 and 9 in 2D are conn 8, 24, 48 and 80)."""
    if ndim == 2 and conn == 4:
        return [(1, 0, 0), (0, 1, 0)]
    if ndim == 2 and conn == 8:
        return [(1, 0, 0), (0, 1, 0), (1, 1, 0), (-1, 1, 0)]
    if ndim == 2 and conn in (24, 48, 80):
        r = {24: 2, 48: 3, 80: 4}[conn]
        # every offset of the (2r+1)^2 square whose first nonzero coordinate, taken from y down to x, is positive
        return [(dx, 0, 0) for dx in range(1, r + 1)] + \
               [(dx, dy, 0) for dy in range(1, r + 1) for dx in range(-r, r + 1)]
    if ndim == 3 and conn == 6:
        return [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    if ndim == 3 and conn in (32, 122, 256):
        # the spherical kernels of size 5, 7 and 9: lattice offsets of length at most r = 2, 3 or 4, each
        # undirected edge once (first nonzero coordinate taken from z down to x positive), z slowest and x fastest
        r = {32: 2, 122: 3, 256: 4}[conn]
        ball = [(dx, dy, dz) for dz in range(r + 1) for dy in range(-r, r + 1) for dx in range(-r, r + 1)
                if 0 < dx * dx + dy * dy + dz * dz <= r * r]
        return [v for v in ball if v[2] > 0 or (v[2] == 0 and (v[1] > 0 or (v[1] == 0 and v[0] > 0)))]
    raise ValueError("unsupported stencil")


def pairwise_matrix(dims, ndim, conn, w) -> sp.csr_matrix:
    """Symmetric W with W_ij = w_ij for each stencil edge i <-> j (each undirected edge once in w)."""
    W_, H_, D_ = dims
    n = W_ * H_ * D_
    idx = np.arange(n, dtype=np.int64)
    x = idx % W_
    y = (idx // W_) % H_
    z = idx // (W_ * H_)
    rows, cols, vals = [], [], []
    for o, (dx, dy, dz) in enumerate(neighbour_offsets(ndim, conn)):
        wv = np.asarray(w[o], dtype=np.int64)
        ok = ((x + dx >= 0) & (x + dx < W_) & (y + dy >= 0) & (y + dy < H_) & (z + dz >= 0) & (z + dz < D_))
        if np.any(wv[~ok] != 0):
            raise ValueError("nonzero weight on an off-grid edge")
        sel = ok & (wv != 0)
        i = idx[sel]
        j = i + dx + W_ * (dy + H_ * dz)
        rows += [i, j]
        cols += [j, i]
        vals += [wv[sel], wv[sel]]
    if rows:
        r = np.concatenate(rows); c = np.concatenate(cols); v = np.concatenate(vals)
    else:
        r = c = v = np.zeros(0, dtype=np.int64)
    return sp.csr_matrix((v, (r, c)), shape=(n, n), dtype=np.int64)


def partition_axis(N: int, B: int, o: int) -> List[Tuple[int, int]]:
    if B <= 0 or B >= N:
        return [(0, N)]
    if not (0 <= o and 2 * o <= B):
        raise ValueError("overlap must satisfy 0 <= o <= B/2")
    s = B - o
    count = 1 + max(0, -(-(N - B) // s))
    return [(t * s, min(t * s + B, N)) for t in range(count)]


@dataclasses.dataclass
class Block:
    origin: Tuple[int, int, int]
    extent: Tuple[int, int, int]
    idx: np.ndarray   # global pixel index of each block pixel, local raster order (x fastest)


def make_blocks(dims, block, overlap) -> List[Block]:
    W_, H_, D_ = dims
    ax = [partition_axis(N, B, o) for N, B, o in zip(dims, block, overlap)]
    out = []
    for (z0, z1) in ax[2]:
        for (y0, y1) in ax[1]:
            for (x0, x1) in ax[0]:
                zz, yy, xx = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
                idx = (xx + W_ * (yy + H_ * zz)).reshape(-1).astype(np.int64)
                out.append(Block((x0, y0, z0), (x1 - x0, y1 - y0, z1 - z0), idx))
    return out


def selector(blk: Block, n: int) -> sp.csr_matrix:
    m = len(blk.idx)
    return sp.csr_matrix((np.ones(m, dtype=np.int64), (np.arange(m), blk.idx)), shape=(m, n), dtype=np.int64)


@dataclasses.dataclass
class Decomposition:
    """Alg. 1 initialisation: potentials, blocks and the per-block parameters of Theorem 1 (x64 integers)."""
    n: int
    lam_q: int
    u: np.ndarray
    W: sp.csr_matrix
    L: sp.csr_matrix
    blocks: List[Block]
    S: List[sp.csr_matrix]
    q: np.ndarray
    u14: List[np.ndarray]          # 2^14 u^_k
    M64: List[sp.csr_matrix]       # 64 (C_k + R_k S_k)
    W64: List[sp.csr_matrix]       # 64 W^_k
    offsets: np.ndarray            # block-major offsets into the concatenated block vectors
    solver: str


def decompose(problem) -> Decomposition:
    n = problem.n
    W = pairwise_matrix(problem.dims, problem.ndim, problem.conn, problem.w)
    d = np.asarray(W.sum(axis=1)).reshape(-1)
    D = sp.diags(d, format="csr", dtype=np.int64)
    L = (D - W).tocsr()
    blocks = make_blocks(problem.dims, problem.block, problem.overlap)
    S = [selector(b, n) for b in blocks]
    Q = sp.csr_matrix((n, n), dtype=np.int64)
    for Sk in S:
        Q = Q + (Sk.T @ Sk)
    q = Q.diagonal().astype(np.int64)
    if np.any(q < 1) or np.any(8 % q != 0):
        raise ValueError("every pixel must lie in 1, 2, 4 or 8 blocks")
    Q8inv = sp.diags(8 // q, format="csr", dtype=np.int64)          # 8 Q^-1
    I8 = sp.diags(np.full(n, 8, dtype=np.int64), format="csr", dtype=np.int64)
    Q8inv_L = (Q8inv @ L).tocsr()
    Q8inv_W_Q8inv = (Q8inv @ W @ Q8inv).tocsr()
    Q8inv_D_Q8inv = (Q8inv @ D @ Q8inv).tocsr()
    u = np.asarray(problem.u, dtype=np.int64)
    u14, M64, W64 = [], [], []
    for Sk in S:
        Pk = (Sk.T @ Sk).tocsr()
        C64 = (Sk @ Q8inv_L @ (I8 - Q8inv @ Pk)).tocsr()                    # 64 C_k
        W64k = (Sk @ Q8inv_W_Q8inv @ Sk.T).tocsr()                           # 64 W^_k
        Dhat64 = sp.diags(np.asarray(W64k.sum(axis=1)).reshape(-1), format="csr", dtype=np.int64)
        R64 = (Sk @ Q8inv_D_Q8inv @ Sk.T - Dhat64).tocsr()                   # 64 R_k
        M64.append((C64 + R64 @ Sk).tocsr())
        W64.append(W64k)
        u14.append(Sk @ ((1 << 14) * u // q))                                # 2^14 S_k Q^-1 u
    for m in M64 + W64 + u14:
        assert m.dtype == np.int64, "Theorem 1 parameters must stay exact integers"
    sizes = np.array([len(b.idx) for b in blocks], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    return Decomposition(n, int(problem.lam_q8), u, W, L, blocks, S, q, u14, M64, W64, offsets, problem.solver)


# ----------------------------------------------------------------------------------------------------------
# ADMM state and one iteration of Algorithm 1
# ----------------------------------------------------------------------------------------------------------

@dataclasses.dataclass
class State:
    Y: np.ndarray          # int64[n], Q16.16
    A: np.ndarray          # int64[sum |Omega_k|], Q16.16, block-major
    yhat: np.ndarray       # uint8[sum |Omega_k|], block-major
    M: int
    t: int

    def copy(self):
        return State(self.Y.copy(), self.A.copy(), self.yhat.copy(), self.M, self.t)


@dataclasses.dataclass
class IterInfo:
    resid2: np.ndarray     # per-block squared residual (Q32.32)
    converged: bool
    overflow: bool


def initial_state(dec: Decomposition, mu0: int) -> State:
    if not (1 <= mu0 <= MU_MAX):
        raise ValueError("mu0 must be in [1, 2^24 - 1]")
    tot = int(dec.offsets[-1])
    return State(np.full(dec.n, Y_HALF, dtype=np.int64), np.zeros(tot, dtype=np.int64),
                 np.zeros(tot, dtype=np.uint8), int(mu0), 0)


def block_subproblem(dec: Decomposition, k: int, Y: np.ndarray, A_k: np.ndarray, M: int):
    """Eq. (8) for block k at the current (y, a_k, mu), scaled by 2^14: (U~, edge list, capacities)."""
    Sk = dec.S[k]
    coupling = dec.M64[k] @ Y                                                # 64 (C_k + R_k S_k) y
    mu_term = (1 << 14) * M * (A_k - Sk @ Y + Y_HALF)                        # 2^14 mu (a_k - S_k y + 1/2)
    Ut = dec.u14[k] + (dec.lam_q * coupling + mu_term) // (1 << 16)
    tri = sp.triu(dec.W64[k], k=1).tocoo()
    return Ut, tri.row.astype(np.int32), tri.col.astype(np.int32), dec.lam_q * tri.data.astype(np.int64)


def solve_block(dec: Decomposition, k: int, state: State) -> np.ndarray:
    a, b = dec.offsets[k], dec.offsets[k + 1]
    Ut, ea, eb, cap = block_subproblem(dec, k, state.Y, state.A[a:b], state.M)
    if dec.solver == "lsatr":
        from . import lsatr
        return lsatr.lsatr(Ut, ea, eb, cap)
    x, _ = solve_subproblem(Ut, ea, eb, cap, "maxflow" if dec.solver == "maxflow" else "exhaustive")
    return x


def consensus(dec: Decomposition, yhat: np.ndarray, A: np.ndarray, M: int) -> np.ndarray:
    """Eq. (10) in Q16.16 with floor (unclamped int64)."""
    Ssum = np.zeros(dec.n, dtype=np.int64)
    H = np.zeros(dec.n, dtype=np.int64)
    for k, Sk in enumerate(dec.S):
        a, b = dec.offsets[k], dec.offsets[k + 1]
        yk = yhat[a:b].astype(np.int64)
        Ssum += Sk.T @ (yk * Y_ONE + A[a:b])
        H += dec.M64[k].T @ yk
    return (M * Ssum - 4 * dec.lam_q * H) // (M * dec.q)


def iterate(dec: Decomposition, state: State, threads: Optional[int] = None,
            yhat_override: Optional[np.ndarray] = None, mu_num: int = 21, mu_den: int = 20,
            eps_q16: Optional[int] = None) -> Tuple[State, IterInfo]:
    """One pass of the main loop of Algorithm 1: block solves (Eq. 8), y update (Eq. 10), multiplier update
    (Eq. 11), mu <- mu * mu_fact.  Returns the new state (the input is not modified).

    yhat_override replaces the block solves (used to check the y / a updates on externally supplied labels)."""
    K = len(dec.blocks)
    if yhat_override is None:
        yhat = np.zeros_like(state.yhat)
        if threads is None:
            threads = os.cpu_count() or 1
        if threads > 1 and K > 1:
            with cf.ThreadPoolExecutor(max_workers=threads) as ex:
                results = list(ex.map(lambda k: solve_block(dec, k, state), range(K)))
        else:
            results = [solve_block(dec, k, state) for k in range(K)]
        for k, x in enumerate(results):
            yhat[dec.offsets[k]:dec.offsets[k + 1]] = x
    else:
        yhat = np.asarray(yhat_override, dtype=np.uint8).copy()
    Ynew = consensus(dec, yhat, state.A, state.M)
    Anew = state.A.copy()
    resid2 = np.zeros(K, dtype=np.int64)
    overflow = bool(np.any(np.abs(Ynew) >= STATE_LIMIT))
    Yc = np.clip(Ynew, -STATE_LIMIT, STATE_LIMIT)
    for k, Sk in enumerate(dec.S):
        a, b = dec.offsets[k], dec.offsets[k + 1]
        yk = yhat[a:b].astype(np.int64)
        Ak = state.A[a:b] + yk * Y_ONE - Sk @ Ynew                            # Eq. (11)
        overflow |= bool(np.any(np.abs(Ak) >= STATE_LIMIT))
        Anew[a:b] = np.clip(Ak, -STATE_LIMIT, STATE_LIMIT)
        r = yk * Y_ONE - Sk @ Yc
        resid2[k] = int(np.sum(r * r))
    new = State(Yc, Anew, yhat, next_mu(state.M, mu_num, mu_den), state.t + 1)
    converged = False
    if eps_q16 is not None:
        converged = bool(np.max(resid2) <= int(eps_q16) ** 2) if K else True
    return new, IterInfo(resid2, converged, overflow)


def next_mu(M: int, num: int = 21, den: int = 20) -> int:
    return min(M * num // den, MU_MAX)


def run(problem, n_iter: Optional[int] = None, threads: Optional[int] = None, record: bool = False,
        dec: Optional[Decomposition] = None):
    """Algorithm 1.  With n_iter given, runs exactly that many iterations (stopping early only on overflow);
    otherwise stops at convergence or problem.max_iter.  Returns (final state, infos, [states per iteration])."""
    if dec is None:
        dec = decompose(problem)
    st = initial_state(dec, problem.mu0)
    infos, states = [], []
    limit = n_iter if n_iter is not None else problem.max_iter
    for _ in range(limit):
        st, info = iterate(dec, st, threads=threads, mu_num=problem.mu_num, mu_den=problem.mu_den,
                           eps_q16=problem.eps_q16)
        infos.append(info)
        if record:
            states.append(st.copy())
        if info.overflow:
            break
        if n_iter is None and info.converged:
            break
    return st, infos, states, dec


# ----------------------------------------------------------------------------------------------------------
# Output and evaluation (Alg. 1 return value, Eq. 1 / Eq. 3, Eq. 12)
# ----------------------------------------------------------------------------------------------------------

def labels(Y: np.ndarray) -> np.ndarray:
    return (np.asarray(Y) > Y_HALF).astype(np.uint8)


def energy_q(dec_or_problem, l: np.ndarray) -> int:
    """E_q = 256 u^T l + lambda_q l^T L l (Eq. 3 scaled by 256; exact int64)."""
    if isinstance(dec_or_problem, Decomposition):
        u, L, lam = dec_or_problem.u, dec_or_problem.L, dec_or_problem.lam_q
    else:
        p = dec_or_problem
        W = pairwise_matrix(p.dims, p.ndim, p.conn, p.w)
        d = np.asarray(W.sum(axis=1)).reshape(-1)
        L = (sp.diags(d, format="csr", dtype=np.int64) - W).tocsr()
        u, lam = np.asarray(p.u, dtype=np.int64), int(p.lam_q8)
    l64 = np.asarray(l, dtype=np.int64)
    return int(256 * (u @ l64) + lam * int(l64 @ (L @ l64)))


def global_mincut(problem) -> Tuple[np.ndarray, int]:
    """Serial graph cut of the whole energy (the sGC comparator of Eq. 12): minimal minimiser and E_q."""
    W = pairwise_matrix(problem.dims, problem.ndim, problem.conn, problem.w)
    tri = sp.triu(W, k=1).tocoo()
    un = 256 * np.asarray(problem.u, dtype=np.int64)
    cap = int(problem.lam_q8) * tri.data.astype(np.int64)
    x, _ = solve_subproblem(un, tri.row, tri.col, cap, "maxflow")
    return x, energy_q(problem, x)
