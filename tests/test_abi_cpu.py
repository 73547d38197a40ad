"""Host-side checks of the C-ABI library (no GPU): it builds, loads, exports every entry point that
include/dope.h declares, and its parameter validation / workspace sizing behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dope.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dope_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def native():
    from paper_1704_03116_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        from paper_1704_03116_amd import build as B
        B.build()
    N.lib()
    return N


def test_header_declares_the_core_entry_points():
    names = header_functions()
    for core in ("dope_create", "dope_set_energy", "dope_iterate", "dope_solve", "dope_labels", "dope_energy",
                 "dope_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol(native):
    L = native.lib()
    for name in header_functions():
        assert hasattr(L, name), name


def test_binding_covers_the_header(native):
    assert sorted(native.SIGNATURES) == header_functions()


def _params(native, dims=(512, 512, 1), conn=8, block=(32, 32, 1), overlap=(2, 2, 0), mu0=1000, solver=0, ndim=2):
    p = native.dope_params()
    p.ndim = ndim
    p.dims[:] = dims
    p.connectivity = conn
    p.block[:] = block
    p.overlap[:] = overlap
    p.mu0 = mu0
    p.mu_fact_num, p.mu_fact_den = 21, 20
    p.eps_q16 = 6554
    p.max_iter = 50
    p.solver = solver
    return p


def _interior_count(dims, block, overlap, r=1):
    """Pixels whose stencil box (radius r) lies in their own block only (the block-solve kernel finishes them)."""
    from oracle import dope as od
    total = 1
    for N, B, o in zip(dims, block, overlap):
        iv = od.partition_axis(N, B, o)
        oo = 0 if len(iv) == 1 else o
        cnt = 0
        for t, (a, b) in enumerate(iv):
            lo = a + oo + r if t > 0 else 0
            hi = b - oo - r if t < len(iv) - 1 else N
            cnt += max(0, hi - lo)
        total *= cnt
    return total


def _workspace_model(dims, h, K, tot, n_int):
    a = lambda x: (x + 255) // 256 * 256  # noqa: E731
    n = dims[0] * dims[1] * dims[2]
    nbl = n - n_int   # boundary pixels (each listed once, through its owner copy)
    chunks = (nbl + 255) // 256
    return (a(128) + a(512) + a(8 * K) + a(8 * chunks) + a(256) + a(K * 32) + a(4 * chunks) + a(8 * nbl)
            + a(4 * n) + 2 * a(4 * h * n) + a(4 * n) + 2 * a(4 * tot) + a(tot) + a(n * (8 if dims[2] > 1 else 4))
            + a(8 * K) + a(16 * K) + a(n) + a(8 * 256) + a(8 * (dims[0] + dims[1] + dims[2])))


@pytest.mark.parametrize("dims,conn,block,overlap,ndim", [
    ((512, 512, 1), 8, (32, 32, 1), (2, 2, 0), 2),
    ((64, 64, 1), 4, (16, 16, 1), (1, 1, 0), 2),
    ((128, 128, 64), 6, (16, 16, 16), (1, 1, 1), 3),
    ((257, 131, 1), 8, (32, 16, 1), (3, 1, 0), 2),
    ((512, 512, 1), 24, (32, 32, 1), (2, 2, 0), 2),
    ((200, 150, 1), 48, (16, 16, 1), (2, 2, 0), 2),
    ((64, 48, 40), 32, (8, 8, 8), (1, 1, 1), 3),
    ((131, 97, 1), 80, (16, 16, 1), (2, 2, 0), 2),
    ((40, 30, 20), 122, (6, 6, 6), (1, 1, 1), 3),
])
def test_workspace_bytes_matches_partition(native, dims, conn, block, overlap, ndim):
    from oracle import dope as od
    p = _params(native, dims, conn, block, overlap, ndim=ndim)
    blocks = od.make_blocks(dims, block, overlap)
    n = dims[0] * dims[1] * dims[2]
    h = {4: 2, 8: 4, 6: 3, 24: 12, 48: 24, 32: 16, 80: 40, 122: 61}[conn]
    r = {24: 2, 48: 3, 32: 2, 80: 4, 122: 3}.get(conn, 1)
    tot = sum(len(b.idx) for b in blocks)
    assert native.dope_workspace_bytes(ctypes.byref(p)) == _workspace_model(dims, h, len(blocks), tot,
                                                                     _interior_count(dims, block, overlap, r))


@pytest.mark.parametrize("kw,msg", [
    (dict(overlap=(17, 2, 0)), "overlap"),
    (dict(conn=6), "connectivity"),
    (dict(mu0=0), "mu0"),
    (dict(block=(160, 160, 1)), "16384 pixels"),          # beyond the LDS and beyond the global-memory solver
    (dict(block=(32, 32, 1), solver=2), "exhaustive"),    # enumeration needs <= 16 pixels
    (dict(dims=(0, 5, 1)), "dims"),
    (dict(conn=48, block=(80, 80, 1)), "4096 pixels"),    # 7x7 neighbourhoods beyond the LDS: 256 threads x 16 px
    (dict(conn=48, block=(4, 4, 1), overlap=(2, 2, 0)), "stencil radius"),   # stride 2 < radius 3
    (dict(conn=24, ndim=3, dims=(16, 16, 16), block=(8, 8, 8), overlap=(1, 1, 1)), "connectivity"),
    (dict(conn=32, ndim=3, dims=(64, 64, 64), block=(20, 20, 20), overlap=(1, 1, 1)), "4096 pixels"),
    (dict(dims=(32768, 32768, 1)), "grid too large"),      # 2^30 pixels: 32-bit byte offsets no longer suffice
    (dict(conn=6, ndim=3, dims=(1024, 1024, 512), block=(16, 16, 16), overlap=(1, 1, 1)), "grid too large"),
])
def test_create_rejects_bad_params(native, kw, msg):
    p = _params(native, **kw)
    ctx = ctypes.c_void_p()
    assert native.dope_create(ctypes.byref(p), ctypes.byref(ctx)) == native.DOPE_EINVAL
    assert msg in native.dope_last_error(None).decode()
    assert native.dope_workspace_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("dims,conn,block,overlap,ndim", [
    ((512, 512, 1), 8, (64, 64, 1), (2, 2, 0), 2),       # 4356-node blocks: 183 KB of max-flow state each
    ((300, 200, 1), 4, (100, 100, 1), (1, 1, 0), 2),
    ((64, 64, 48), 6, (24, 24, 24), (1, 1, 1), 3),
    ((200, 150, 1), 48, (48, 48, 1), (3, 3, 0), 2),      # 7x7: 209 B per node
    ((40, 36, 30), 122, (12, 12, 12), (1, 1, 1), 3),     # radius-3 ball: 513 B per node
])
def test_blocks_beyond_lds_take_workspace_state(native, dims, conn, block, overlap, ndim):
    """Blocks whose max-flow state exceeds the LDS are accepted, with each block's state (64 + np (8h + 9 + m)
    bytes, m the direction-mask bytes, plus alignment, for the largest block, 256-aligned) after the workspace
    layout of the LDS path."""
    from oracle import dope as od
    p = _params(native, dims, conn, block, overlap, ndim=ndim)     # accepted: a nonzero workspace size
    blocks = od.make_blocks(dims, block, overlap)
    h = {4: 2, 8: 4, 6: 3, 48: 24, 122: 61}[conn]
    r = {48: 3, 122: 3}.get(conn, 1)
    mb = 1 if 2 * h <= 8 else (4 if 2 * h <= 32 else (8 if 2 * h <= 64 else 16))   # direction-mask bytes
    slack = 16 if mb > 8 else (8 if mb > 1 else 0)
    np_max = max(len(b.idx) for b in blocks)
    per_block = (64 + np_max * (8 * h + 9 + mb) + slack + 255) // 256 * 256
    assert per_block > 160 * 1024
    tot = sum(len(b.idx) for b in blocks)
    base = _workspace_model(dims, h, len(blocks), tot, _interior_count(dims, block, overlap, r))
    assert native.dope_workspace_bytes(ctypes.byref(p)) == base + len(blocks) * per_block


@pytest.mark.parametrize("dims,conn,block,overlap,ndim", [
    ((128, 128, 64), 6, (16, 16, 16), (1, 1, 1), 3),      # 256 full blocks, 149 clipped at the far faces
    ((512, 512, 1), 8, (32, 32, 1), (2, 2, 0), 2),       # every block full
    ((257, 131, 1), 8, (32, 16, 1), (3, 1, 0), 2),
    ((40, 30, 20), 122, (6, 6, 6), (1, 1, 1), 3),
    ((100, 37, 23), 6, (12, 10, 8), (1, 2, 1), 3),
    ((64, 64, 1), 4, (64, 64, 1), (0, 0, 0), 2),         # one block
    ((33, 17, 9), 6, (8, 8, 8), (1, 1, 1), 3),
])
def test_dispatch_order_full_blocks_first(native, dims, conn, block, overlap, ndim):
    """The one-image block-solve schedule is a permutation of the blocks (numbered x-fastest over the partition);
    the blocks of full extent along every axis take the first workgroups; within each group the workgroups of one
    XCD (one residue of the workgroup index mod 8) take a contiguous, increasing range of the group's raster
    order."""
    from oracle import dope as od
    from paper_1704_03116_amd.solver import dispatch_order
    order = dispatch_order(_params(native, dims, conn, block, overlap, ndim=ndim))
    iv = [od.partition_axis(N, B, o) for N, B, o in zip(dims, block, overlap)]
    nb = [len(a) for a in iv]
    K = nb[0] * nb[1] * nb[2]
    assert sorted(order.tolist()) == list(range(K))
    full = []
    for k in range(K):
        t = (k % nb[0], (k // nb[0]) % nb[1], k // (nb[0] * nb[1]))
        if all(iv[a][t[a]][1] - iv[a][t[a]][0] == block[a] for a in range(3)):
            full.append(k)
    nf = len(full)
    assert sorted(order[:nf].tolist()) == full
    rest = sorted(set(range(K)) - set(full))
    for group, lo in ((full, 0), (rest, nf)):
        rank = {k: i for i, k in enumerate(group)}
        for j in range(8):
            ranks = [rank[int(order[b])] for b in range(lo, lo + len(group)) if b % 8 == j]
            assert ranks == list(range(ranks[0], ranks[0] + len(ranks))) if ranks else True


def test_dispatch_order_rejects_bad_params(native):
    import ctypes as ct
    p = _params(native, overlap=(17, 2, 0))
    K = ct.c_int32()
    assert native.dope_dispatch_order(ct.byref(p), ct.byref(K), None) == native.DOPE_EINVAL
    assert "overlap" in native.dope_last_error(None).decode()


def test_last_error_null_safe(native):
    assert isinstance(native.dope_last_error(None), bytes)


def test_autotune_is_a_pure_function_of_shape(native):
    """dope_autotune returns, for every measured image of the committed MI355X sweep, the fastest candidate of
    that sweep row; every choice fits the LDS and keeps the stride at least the stencil radius; the result
    depends on the shape only."""
    import json
    from paper_1704_03116_amd.solver import autotune
    rec = json.load(open(os.path.join(ROOT, "profiles", "autotune_sweep.json")))
    half = {4: 2, 8: 4, 24: 12, 48: 24, 80: 40, 6: 3, 32: 16, 122: 61}
    radius = {4: 1, 8: 1, 24: 2, 48: 3, 80: 4, 6: 1, 32: 2, 122: 3}
    for sw in rec["sweeps"]:
        nd, conn = sw["ndim"], sw["conn"]
        # of measured images that share a shorter side, the largest decides that side's row
        deciding = {}
        for row in sorted(sw["rows"], key=lambda r: (min(r["dims"]), int(np.prod(r["dims"])))):
            deciding[min(row["dims"])] = row
        for row in deciding.values():
            best = row["best"]
            assert best["mpx_s"] == max(r["mpx_s"] for r in row["runs"])
            blk, ovl = autotune(nd, tuple(row["dims"]), conn)
            assert blk[:nd] == (best["B"],) * nd and ovl[:nd] == (best["o"],) * nd, (conn, row["dims"])
            h = half[conn]
            mb = 1 if 2 * h <= 8 else (4 if 2 * h <= 32 else (8 if 2 * h <= 64 else 16))
            assert 64 + best["B"] ** nd * (8 * h + 9 + mb) + 16 <= 160 * 1024 - 1024
            assert best["B"] - best["o"] >= radius[conn] and 2 * best["o"] <= best["B"]
    assert autotune(2, (512, 300), 8) == autotune(2, (300, 512), 8) == autotune(2, (300, 9000), 8)
    assert autotune(2, (4096, 2048), 8)[0] == (32, 32, 1)
    with pytest.raises(Exception):
        autotune(2, (64, 64), 6)