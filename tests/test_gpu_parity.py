"""Parity of the HIP path (through the C ABI) with the CPU oracle, bit-exact at every ADMM iteration.

Every problem, the full-size workloads included, is compared on the whole state (Y, A, block labels, mu, t,
per-block residuals and the stopping flag) after every iteration."""
import dataclasses
import os

import numpy as np
import pytest

import synth
from oracle import dope as od

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1704_03116_amd import _native as N
    N.lib()   # raises when the library is missing: no fallback


def make_ctx(p, **kw):
    from paper_1704_03116_amd.solver import Dope
    d = Dope.from_problem(p, **kw)
    d.set_energy(np.ascontiguousarray(p.u, np.int32), np.ascontiguousarray(p.w, np.int32), p.lam_q8)
    return d


def first_mismatch(a, b):
    idx = np.flatnonzero(np.asarray(a) != np.asarray(b))
    return None if len(idx) == 0 else (int(idx[0]), a[idx[0]], b[idx[0]], len(idx))


def assert_state_equal(d, S, info_o, t, dec):
    Y, A, yh, mu, tt = d.get_state()
    assert tt == S.t == t, (tt, S.t, t)
    mm = first_mismatch(yh, S.yhat)
    if mm is not None:
        k = int(np.searchsorted(dec.offsets, mm[0], side="right") - 1)
        raise AssertionError(f"iteration {t}: block labels differ at {mm} (block {k})")
    assert first_mismatch(Y, S.Y) is None, f"iteration {t}: Y differs {first_mismatch(Y, S.Y)}"
    assert first_mismatch(A, S.A) is None, f"iteration {t}: A differs {first_mismatch(A, S.A)}"
    assert mu == S.M
    assert np.array_equal(d.block_resid(), info_o.resid2), f"iteration {t}: residuals differ"


# host threads for the oracle's block solves (at most 16, a one-GPU host's share of cores)
ORACLE_THREADS = min(16, os.cpu_count() or 1)


def run_parity(p, n_iter, label, stats=None, dec=None):
    """Runs the oracle and the GPU side by side for n_iter iterations (stopping early only on overflow) and
    compares the whole state (Y, A, block labels, mu, t, per-block residuals, the stopping flag) after every
    iteration.  stats: optional list that receives each iteration's per-block solver statistics."""
    announce(f"{label}: dims={p.dims} conn={p.conn} block={p.block} overlap={p.overlap} mu0={p.mu0} "
             f"solver={p.solver} iters={n_iter}")
    if dec is None:
        dec = od.decompose(p)
    st = od.initial_state(dec, p.mu0)
    d = make_ctx(p)
    try:
        for t in range(1, n_iter + 1):
            st, inf = od.iterate(dec, st, threads=ORACLE_THREADS, mu_num=p.mu_num, mu_den=p.mu_den,
                                 eps_q16=p.eps_q16)
            status, info = d.iterate_status(1)
            if stats is not None:
                stats.append(d.block_stats())
            if inf.overflow:
                assert status == -5, f"oracle overflowed at iteration {t}, GPU status {status}"
                assert_state_equal(d, st, inf, t, dec)
                return d, st, dec
            assert status == 0, f"iteration {t}: status {status}"
            assert info["converged"] == inf.converged == (int(np.max(inf.resid2)) <= p.eps_q16 ** 2)
            assert_state_equal(d, st, inf, t, dec)
        return d, st, dec
    except Exception:
        d.close()
        raise


def test_config1_every_iteration():
    """64x64 disk, 4-connected, 16x16 blocks with 1-px overlap, 50 iterations."""
    p = synth.config1()
    d, st_o, dec = run_parity(p, 50, "config1")
    l = d.labels()
    assert np.array_equal(l, od.labels(st_o.Y))
    assert d.energy() == od.energy_q(dec, od.labels(st_o.Y))
    d.close()


@pytest.mark.parametrize("W,H,seed", [(100, 90, 0), (131, 67, 3)])
def test_config2_small_every_iteration(W, H, seed):
    """config-2 construction (3-channel ellipses, 8-connected contrast weights, lambda 2, 32x32 / o = 2) on
    grids with ragged edge blocks."""
    p = synth.config2(seed=seed, W=W, H=H)
    p.mu0 = 300   # a smaller mu keeps several iterations non-trivial
    d, _, _ = run_parity(p, 8, f"config2 {W}x{H}")
    d.close()


def test_config3_small_every_iteration():
    p = synth.config3(dims=(40, 36, 20))
    d, _, _ = run_parity(p, 6, "config3 40x36x20")
    d.close()


CASES = [
    # dims, conn, block, overlap, lam_q8, mu0
    ((17, 13, 1), 4, (5, 4, 1), (1, 1, 0), 256, 1000),
    ((33, 29, 1), 8, (8, 8, 1), (2, 3, 0), 600, 2000),
    ((19, 23, 1), 8, (16, 16, 1), (8, 8, 0), 300, 500),     # overlap = B/2 (q up to 4 everywhere)
    ((9, 11, 7), 6, (4, 5, 3), (1, 2, 1), 384, 5000),      # 3D, 8 copies at corners
    ((1, 40, 1), 4, (1, 8, 1), (0, 2, 0), 256, 1000),      # one-pixel-wide grid
    ((45, 3, 1), 8, (16, 3, 1), (1, 0, 0), 900, 1500),     # single block along y
    ((21, 21, 1), 4, (0, 0, 0), (0, 0, 0), 256, 1000),     # one block: global cut
    ((50, 40, 1), 8, (32, 32, 1), (2, 2, 0), 1000, 100),   # strong smoothing, small mu
]


@pytest.mark.parametrize("case", CASES)
def test_random_shapes_every_iteration(case):
    dims, conn, block, overlap, lam, mu0 = case
    p = synth.random_problem(11, dims, conn, block, overlap, lam_q8=lam, u_range=(-2500, 2500),
                             w_range=(0, 900), mu0=mu0)
    d, _, _ = run_parity(p, 5, f"random {case}")
    d.close()


@pytest.mark.parametrize("which", ["config1", "config2_small"])
def test_per_iteration_metrics_match_the_oracle(which, tmp_path):
    """iterate_metrics: one record per iteration whose t, max_k r_k, stopping flag, mu and block of the largest
    residual equal the oracle's, iteration by iteration; the loop that converges stops at the oracle's iteration;
    the JSON-lines file holds the same records."""
    import json
    p = synth.config1() if which == "config1" else synth.config2(W=100, H=90)
    n_max = 8
    dec = od.decompose(p)
    st = od.initial_state(dec, p.mu0)
    expect = []
    for _ in range(n_max):
        st, inf = od.iterate(dec, st, threads=ORACLE_THREADS, mu_num=p.mu_num, mu_den=p.mu_den, eps_q16=p.eps_q16)
        expect.append((st.t, int(np.max(inf.resid2)), inf.converged, st.M, int(np.argmax(inf.resid2))))
        if inf.converged:
            break
    d = make_ctx(p)
    try:
        path = tmp_path / "metrics.jsonl"
        recs = d.iterate_metrics(n_max, str(path))
    finally:
        d.close()
    got = [(r["t"], r["max_resid2"], r["converged"], r["mu"], r["worst_block"]) for r in recs]
    assert got == expect
    assert all(r["status"] == 0 for r in recs)
    assert [json.loads(line) for line in path.read_text().splitlines()] == recs
    if which == "config2_small":
        assert recs[-1]["converged"] and len(recs) < n_max


@pytest.mark.timeout(600)
def test_debug_build_cut_checks_hold():
    """The instrumented build (libdope_debug.so: the block max-flow of the 3x3 stencils checks that its marked set
    contains every excess, is closed under residual arcs and holds no sink capacity, else the iteration fails with
    a solver error) runs push-relabel-heavy and tie-prone problems, in LDS and in the two-launch global-memory
    solve, with every iteration succeeding and the whole state equal to the oracle's (in a process of its own,
    which loads that library)."""
    import subprocess
    import sys
    lib = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1704_03116_amd",
                       "libdope_debug.so")
    if not os.path.exists(lib):
        pytest.skip("libdope_debug.so not built (the library build makes it)")
    child = os.path.join(os.path.dirname(os.path.abspath(__file__)), "debug_build_child.py")
    r = subprocess.run([sys.executable, "-u", child], capture_output=True, text=True, timeout=540)
    announce(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("debug build ok")


def test_smoothing_dominated_blocks():
    """Weak unaries, strong edges: almost no node is forced, so push-relabel does all the work."""
    p = synth.random_problem(12, (48, 40, 1), 8, (16, 16, 1), (1, 1, 0), lam_q8=768, u_range=(-400, 400),
                             w_range=(200, 1000), mu0=800)
    d, _, _ = run_parity(p, 6, "smoothing dominated")
    stats = d.block_stats()
    assert stats[:, 0].sum() > 0 and stats[:, 1].sum() > 0
    d.close()


def test_exhaustive_nonsubmodular_every_iteration():
    p = synth.config4(size=40)
    d, _, _ = run_parity(p, 5, "config4 40x40 exhaustive")
    d.close()


def test_exhaustive_equals_maxflow_on_submodular():
    p = synth.random_problem(13, (23, 18, 1), 4, (4, 4, 1), (1, 1, 0), lam_q8=256, mu0=1000)
    d1, _, _ = run_parity(p, 4, "maxflow 4x4")
    p.solver = "exhaustive"
    d2, _, _ = run_parity(p, 4, "exhaustive 4x4")
    assert np.array_equal(d1.get_state()[2], d2.get_state()[2])
    d1.close()
    d2.close()


def test_overflow_matches_oracle():
    p = synth.config1(mu0=1)
    d, _, _ = run_parity(p, 10, "overflow mu0=1")
    status, _ = d.iterate_status(1)
    assert status == -5     # frozen: later calls keep reporting the overflow
    d.close()


def test_solve_to_convergence_and_energy():
    p = synth.config2(W=160, H=160)
    announce("solve config2 160x160")
    st_o, infos, _, dec = od.run(p)
    d = make_ctx(p)
    info = d.solve()
    assert info["iters_done"] == len(infos)
    assert info["converged"] == infos[-1].converged
    Y, A, yh, mu, t = d.get_state()
    assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
    l = d.labels()
    assert np.array_equal(l, od.labels(st_o.Y))
    assert d.energy() == od.energy_q(dec, l)
    d.close()


def test_error_paths():
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Dope
    announce("error paths")
    p = synth.random_problem(14, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0), neg_frac=0.3)
    with Dope.from_problem(p, solver="maxflow") as d:
        with pytest.raises(N.DopeError) as e:
            d.set_energy(p.u, p.w, p.lam_q8)
        assert e.value.status == N.DOPE_ENOTSUBMODULAR
        with pytest.raises(N.DopeError) as e:
            d.iterate(1)
        assert e.value.status == N.DOPE_ESTATE
    q = synth.random_problem(15, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0))
    w = q.w.copy()
    w[0, 19] = 5     # edge leaving the grid on the right
    with Dope.from_problem(q) as d:
        with pytest.raises(N.DopeError) as e:
            d.set_energy(q.u, w, q.lam_q8)
        assert e.value.status == N.DOPE_EINVAL
        with pytest.raises(N.DopeError) as e:
            d.set_energy(q.u, q.w, -1)
        assert e.value.status == N.DOPE_EINVAL


def test_checkpoint_resume_and_determinism():
    p = synth.config1()
    announce("checkpoint / resume")
    a = make_ctx(p)
    a.iterate(7)
    straight = a.get_state()
    b = make_ctx(p)
    b.iterate(3)
    Y, A, yh, mu, t = b.get_state()
    c = make_ctx(p)
    c.set_state(Y, A, yh, mu, t)
    c.iterate(4)
    resumed = c.get_state()
    for x, y in zip(straight, resumed):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    a2 = make_ctx(p)
    a2.iterate(7)
    again = a2.get_state()
    for x, y in zip(straight, again):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    for d in (a, b, c, a2):
        d.close()


def test_block_table_matches_partition():
    p = synth.config3(dims=(40, 36, 20))
    d = make_ctx(p)
    tab = d.block_table()
    blocks = od.make_blocks(p.dims, p.block, p.overlap)
    assert len(tab) == len(blocks)
    off = 0
    for row, b in zip(tab, blocks):
        assert tuple(row[:3]) == b.origin and tuple(row[3:6]) == b.extent and row[6] == off
        off += len(b.idx)
    d.close()


def test_device_inputs_and_labels():
    """Inputs already resident in HBM (torch tensors), labels written to a device tensor."""
    import torch
    p = synth.config1()
    announce("device-resident inputs")
    from paper_1704_03116_amd.solver import Dope
    d = Dope.from_problem(p)
    u = torch.from_numpy(np.ascontiguousarray(p.u, np.int32)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(p.w, np.int32)).cuda()
    d.set_energy(u, w, p.lam_q8)
    d.iterate(5)
    lab = torch.zeros(p.n, dtype=torch.uint8, device="cuda")
    d.labels(lab)
    st_o, _, _, _ = od.run(p, n_iter=5)
    assert np.array_equal(lab.cpu().numpy(), od.labels(st_o.Y))
    d.close()


# ------------------------------------------------------------------------------------------------------------
# full-size workloads: the whole state after every iteration, in the launch configuration the benchmark times
# ------------------------------------------------------------------------------------------------------------

@pytest.mark.timeout(600)
def test_config2_full_size_every_iteration():
    """512x512, 8-connected, 32x32 blocks with o = 2 (289 blocks, the 512-thread block solver): the solve stops
    after 2 iterations; 4 are compared."""
    d, st, dec = run_parity(synth.config2(), 4, "config2 512x512 full size")
    assert np.array_equal(d.labels(), od.labels(st.Y))
    d.close()


@pytest.mark.timeout(900)
def test_config3_full_size_every_iteration():
    """128x128x64, 6-connected, 16^3 blocks with o = 1 (405 blocks, one 1024-thread workgroup per CU): all 50
    iterations of the solve, whole state after each, then labels and energy."""
    p = synth.config3()
    d, st, dec = run_parity(p, p.max_iter, "config3 128x128x64 full size")
    assert np.array_equal(d.labels(), od.labels(st.Y))
    assert d.energy() == od.energy_q(dec, od.labels(st.Y))
    d.close()


@pytest.mark.timeout(600)
def test_config4_full_size_every_iteration():
    """256x256 non-submodular grid, 7225 exhaustive 4x4 blocks: 3 iterations."""
    d, _, _ = run_parity(synth.config4(), 3, "config4 256x256 exhaustive full size")
    d.close()


@pytest.mark.timeout(600)
def test_config2_full_size_solve():
    """dope_solve (speculative iteration chunks, polled readback) on the full 512x512 image: iterations, stopping
    flag, state and labels equal the oracle's solve."""
    p = synth.config2()
    announce("config2 512x512 full-size solve")
    st_o, infos, _, dec = od.run(p, threads=ORACLE_THREADS)
    d = make_ctx(p)
    info = d.solve()
    assert info["iters_done"] == len(infos) and info["converged"] == infos[-1].converged
    Y, A, yh, mu, t = d.get_state()
    assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
    assert np.array_equal(d.labels(), od.labels(st_o.Y))
    d.close()


# ------------------------------------------------------------------------------------------------------------
# larger neighbourhoods: 5x5 (connectivity 24) and 7x7 (48) squares
# ------------------------------------------------------------------------------------------------------------

WIDE_CASES = [
    # dims, conn, block, overlap, lam_q8, mu0
    ((37, 29, 1), 24, (8, 8, 1), (2, 2, 0), 300, 1000),
    ((23, 19, 1), 24, (4, 4, 1), (2, 2, 0), 256, 500),      # stride 2 = radius: q up to 4 everywhere
    ((20, 17, 1), 24, (0, 0, 0), (0, 0, 0), 256, 1000),     # one block: global cut
    ((40, 33, 1), 48, (10, 10, 1), (3, 3, 0), 150, 1000),
    ((31, 26, 1), 48, (6, 6, 1), (3, 3, 0), 120, 800),      # stride 3 = radius
    ((3, 30, 1), 48, (3, 8, 1), (0, 3, 0), 150, 1000),      # grid narrower than the stencil
    ((13, 11, 9), 32, (5, 5, 4), (1, 1, 1), 200, 5000),     # 3D ball of radius 2
    ((9, 9, 8), 32, (4, 4, 4), (2, 2, 2), 150, 3000),       # stride 2 = radius: 8 copies at every corner
    ((41, 35, 1), 80, (12, 12, 1), (2, 2, 0), 100, 1000),   # 9x9 neighbourhood
    ((29, 23, 1), 80, (6, 6, 1), (2, 2, 0), 80, 800),       # 9x9, stride 4 = radius
    ((14, 12, 10), 122, (6, 6, 5), (1, 1, 1), 40, 4000),    # 3D ball of radius 3
    ((13, 11, 10), 256, (5, 5, 5), (1, 1, 1), 20, 4000),    # 3D ball of radius 4, stride 4 = radius
    ((9, 9, 9), 256, (0, 0, 0), (0, 0, 0), 20, 4000),       # radius 4, one block: global cut
]


@pytest.mark.parametrize("case", WIDE_CASES)
def test_wide_stencils_every_iteration(case):
    dims, conn, block, overlap, lam, mu0 = case
    p = synth.random_problem(21, dims, conn, block, overlap, lam_q8=lam, u_range=(-4000, 4000),
                             w_range=(0, 900), mu0=mu0)
    d, _, _ = run_parity(p, 5, f"wide {case}")
    d.close()


@pytest.mark.parametrize("k,W,H", [(5, 100, 90), (7, 90, 70), (9, 80, 75)])
def test_kernel_workloads_small_every_iteration(k, W, H):
    """The larger-kernel workloads (contrast weights on the 5x5 / 7x7 square) on small grids."""
    p = synth.config_kernel(k, W=W, H=H)
    p.mu0 = 300
    d, st_o, dec = run_parity(p, 8, f"kernel{k} {W}x{H}")
    assert np.array_equal(d.labels(), od.labels(st_o.Y))
    assert d.energy() == od.energy_q(dec, od.labels(st_o.Y))
    d.close()


def test_wide_exhaustive_nonsubmodular():
    p = synth.random_problem(14, (16, 15, 1), 24, (4, 4, 1), (1, 1, 0), lam_q8=200, u_range=(-2000, 2000),
                             w_range=(0, 500), neg_frac=0.3, mu0=1000, solver="exhaustive")
    d, _, _ = run_parity(p, 4, "5x5 neighbourhood, 4x4 blocks, exhaustive")
    d.close()


@pytest.mark.parametrize("k,dims", [(5, (40, 36, 20)), (7, (30, 26, 14)), (9, (24, 21, 13))])
def test_ball_kernel_volume_small_every_iteration(k, dims):
    """The spherical kernels of size 5, 7 and 9 on small versions of the config3 volume."""
    p = synth.config3_kernel5(dims=dims, k=k)
    d, st_o, dec = run_parity(p, 5, f"ball kernel {k} {dims}")
    assert np.array_equal(d.labels(), od.labels(st_o.Y))
    assert d.energy() == od.energy_q(dec, od.labels(st_o.Y))
    d.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k,n_iter", [(5, 4), (7, 3), (9, 2)])
def test_kernel_full_size_every_iteration(k, n_iter):
    """The 512x512 image with the 5x5 / 7x7 / 9x9 neighbourhood (its solve stops after 3 / 2 / 1 iterations): the
    whole state after every iteration, one past the stop."""
    d, st, dec = run_parity(synth.config_kernel(k), n_iter, f"kernel{k} 512x512 full size")
    assert np.array_equal(d.labels(), od.labels(st.Y))
    d.close()


def test_batch_wide_stencil_matches_alone():
    from paper_1704_03116_amd.solver import Batch
    probs = [synth.config_kernel(5, seed=s, W=W, H=H) for s, (W, H) in enumerate([(90, 70), (64, 99), (120, 41)])]
    for p in probs:
        p.mu0 = 300
    announce("batch of 5x5-neighbourhood images")
    ctxs = [make_ctx(p) for p in probs]
    with Batch(ctxs, graph=True) as b:
        b.iterate(4)
    for p, c in zip(probs, ctxs):
        st_o, _, _, _ = od.run(p, n_iter=4)
        Y, A, yh, mu, t = c.get_state()
        assert t == 4 and np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
        c.close()


# ------------------------------------------------------------------------------------------------------------
# batched launches: many images, one launch per phase; each image bit-identical to running alone
# ------------------------------------------------------------------------------------------------------------

def _batch_problems():
    out = [synth.config2(seed=s, W=W, H=H) for s, (W, H) in enumerate([(96, 80), (150, 61), (64, 64), (33, 190)])]
    for p in out:
        p.mu0 = 300
    return out


@pytest.mark.parametrize("graph,workers", [(False, 0), (True, 0), (True, 16)])
def test_batch_iterate_matches_alone_and_oracle(graph, workers):
    from paper_1704_03116_amd.solver import Batch
    probs = _batch_problems()
    announce(f"batch of {len(probs)} images, graph={graph} workers={workers}")
    ctxs = [make_ctx(p) for p in probs]
    alone = [make_ctx(p) for p in probs]
    with Batch(ctxs, graph=graph, workers=workers) as b:
        for t in range(1, 6):
            b.iterate(1)
            for p, c, a in zip(probs, ctxs, alone):
                a.iterate(1)
                sc, sa = c.get_state(), a.get_state()
                for x, y in zip(sc, sa):
                    assert np.array_equal(np.asarray(x), np.asarray(y)), f"iteration {t}: batch != alone ({p.name})"
        infos = b.info()
        assert all(i["iters_done"] == 5 for i in infos)
    for p, c in zip(probs, ctxs):
        st_o, _, _, _ = od.run(p, n_iter=5)
        Y, A, yh, mu, t = c.get_state()
        assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
    for c in ctxs + alone:
        c.close()


def test_batch_solve_per_image_stopping():
    """Images converge at different iterations; each stops alone and matches the oracle's own stopping point."""
    from paper_1704_03116_amd.solver import Batch
    probs = _batch_problems()
    probs[1].max_iter = 3
    probs[2].mu0 = 5000
    announce("batch solve with per-image stopping")
    ctxs = [make_ctx(p) for p in probs]
    with Batch(ctxs, graph=True) as b:
        b.solve()
        infos = b.info()
    for p, c, inf in zip(probs, ctxs, infos):
        st_o, infos_o, _, dec = od.run(p)
        assert inf["iters_done"] == len(infos_o), p.name
        assert inf["converged"] == infos_o[-1].converged
        Y, A, yh, mu, t = c.get_state()
        assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
        assert np.array_equal(c.labels(), od.labels(st_o.Y))
        c.close()


def test_batch_solve_again_after_new_energies():
    """A second batch solve after every member got a new energy (asynchronously) starts each image from its own
    reset state, whatever the first solve left in the batch's summaries: the first energies (no pairwise terms)
    stop early, the second ones need more iterations."""
    from paper_1704_03116_amd.solver import Batch
    import torch

    def problems():
        out = []
        for s in range(4):
            q = synth.config5_image(48 + 16 * s, 40 + 8 * s, lam=1.5, seed=s)
            q.block, q.overlap = (16, 16, 1), (1, 1, 0)
            q.max_iter = 12
            out.append(q)
        return out

    second = problems()
    first = problems()
    for q in first:
        q.w = np.zeros_like(q.w)
    announce("batch solve, new energies, batch solve again")
    ctxs = [make_ctx(p) for p in first]
    with Batch(ctxs, graph=True) as b:
        b.solve()
        first_iters = [i["iters_done"] for i in b.info()]
        for c, q in zip(ctxs, second):
            c.set_energy_async(torch.from_numpy(np.ascontiguousarray(q.u)).cuda(),
                               torch.from_numpy(np.ascontiguousarray(q.w)).cuda(), q.lam_q8)
        b.solve()
        infos = b.info()
    more = 0
    for q, c, inf, n1 in zip(second, ctxs, infos, first_iters):
        st_o, infos_o, _, _ = od.run(q)
        assert inf["iters_done"] == len(infos_o), q.name
        more += len(infos_o) > n1
        Y, A, yh, mu, t = c.get_state()
        assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A)
        c.close()
    assert more > 0, "the second energies should need more iterations than the first took"


@pytest.mark.parametrize("device", [True, False])
def test_batch_energy_upload_and_labels(device):
    """One-launch energy upload and labels for a whole batch equal the per-context calls and the oracle; a second
    upload with other energies restarts every image."""
    from paper_1704_03116_amd.solver import Batch
    import torch
    first = _batch_problems()
    second = [synth.config2(seed=30 + i, W=q.dims[0], H=q.dims[1]) for i, q in enumerate(first)]
    for q in second:
        q.mu0 = first[0].mu0
    announce(f"batched energy upload and labels, device inputs={device}")
    ctxs = [make_ctx(p) for p in first]

    def inputs(probs):
        if device:
            return ([torch.from_numpy(np.ascontiguousarray(q.u)).cuda() for q in probs],
                    [torch.from_numpy(np.ascontiguousarray(q.w)).cuda() for q in probs])
        return [np.ascontiguousarray(q.u) for q in probs], [np.ascontiguousarray(q.w) for q in probs]

    with Batch(ctxs, graph=True) as b:
        for probs in (first, second):
            us, ws = inputs(probs)
            b.set_energy_async(us, ws, [q.lam_q8 for q in probs])
            b.solve()
            infos = b.info()
            host = b.labels()
            dev = b.labels([torch.empty(q.n, dtype=torch.uint8, device="cuda") for q in probs])
            torch.cuda.synchronize()
            for q, c, inf, lh, ld in zip(probs, ctxs, infos, host, dev):
                st_o, infos_o, _, _ = od.run(q)
                assert inf["iters_done"] == len(infos_o), q.name
                Y, A, yh, mu, t = c.get_state()
                assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A), q.name
                assert np.array_equal(lh, od.labels(st_o.Y)) and np.array_equal(ld.cpu().numpy(), lh), q.name
    for c in ctxs:
        c.close()


def test_batch_exhaustive_nonsubmodular():
    from paper_1704_03116_amd.solver import Batch
    probs = [synth.config4(seed=s, size=sz) for s, sz in enumerate([24, 37, 16])]
    announce("exhaustive batch")
    ctxs = [make_ctx(p) for p in probs]
    with Batch(ctxs, graph=True) as b:
        b.iterate(3)
    for p, c in zip(probs, ctxs):
        st_o, _, _, _ = od.run(p, n_iter=3)
        Y, A, yh, mu, t = c.get_state()
        assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
        c.close()


def test_batch_rejects_mixed_connectivity():
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Batch
    a = make_ctx(synth.config1(size=32))
    b = make_ctx(synth.config2(W=40, H=40))
    with pytest.raises(N.DopeError) as e:
        Batch([a, b])
    assert e.value.status == N.DOPE_EINVAL
    a.close()
    b.close()


def test_async_energy_upload_and_deferred_validation():
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Dope
    import torch
    announce("asynchronous energy upload")
    p = synth.config1()
    d = Dope.from_problem(p)
    d.set_energy_async(torch.from_numpy(np.ascontiguousarray(p.u)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(p.w)).cuda(), p.lam_q8)
    d.iterate(4)
    st_o, _, _, _ = od.run(p, n_iter=4)
    Y, A, yh, mu, t = d.get_state()
    assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
    d.close()
    q = synth.random_problem(16, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0), neg_frac=0.3)
    with Dope.from_problem(q, solver="maxflow") as e:
        e.set_energy_async(q.u, q.w, q.lam_q8)          # returns at once; the verdict comes with the next readback
        with pytest.raises(N.DopeError) as err:
            e.iterate(1)
        assert err.value.status == N.DOPE_ENOTSUBMODULAR
        assert e.get_state()[4] == 0                     # no iteration ran


BEYOND_LDS_CASES = [
    ("8-connected 2x2 blocks of 98x82", lambda: dataclasses.replace(synth.config2(W=192, H=160), block=(98, 82, 1))),
    ("4-connected 3x2 blocks of 112x100", lambda: synth.random_problem(21, (230, 150, 1), 4, (112, 100, 1),
                                                                         (1, 1, 0))),
    ("6-connected 2x2x2 blocks of 22x20x16", lambda: synth.random_problem(22, (40, 36, 30), 6, (22, 20, 16),
                                                                            (1, 1, 1))),
    ("5x5 2x2 blocks of 60x60", lambda: synth.random_problem(26, (118, 100, 1), 24, (60, 60, 1), (2, 2, 0))),
    ("7x7 2x2 blocks of 48x48", lambda: synth.random_problem(23, (90, 88, 1), 48, (48, 48, 1), (3, 3, 0))),
    ("9x9 2x2 blocks of 40x40", lambda: synth.random_problem(24, (70, 66, 1), 80, (40, 40, 1), (4, 4, 0),
                                                             w_range=(0, 400))),   # 80 edges: sum |c| < 2^29
    ("radius-2 ball 2x2x2 blocks of 14^3", lambda: synth.random_problem(25, (26, 24, 22), 32, (14, 14, 14),
                                                                          (2, 2, 2))),
    ("radius-3 ball 2x2x2 blocks of 12^3", lambda: dataclasses.replace(
        synth.config3_kernel5(dims=(22, 22, 20), k=7), block=(12, 12, 12), overlap=(1, 1, 1))),
]


@pytest.mark.parametrize("label,make", BEYOND_LDS_CASES, ids=[c[0] for c in BEYOND_LDS_CASES])
def test_blocks_beyond_lds_every_iteration(label, make):
    """Blocks whose max-flow state exceeds the LDS (7040 to 11200 nodes with the 3x3 stencils, 1600 to 3600 with
    the wide ones) run the same solver with that state in the workspace: Y, A, yhat, mu, t and the block
    residuals equal the oracle's after every iteration."""
    p = make()
    stats = []
    d, st_o, dec = run_parity(p, 6, f"beyond LDS, {label}", stats=stats)
    d.close()
    # the global-memory solver runs its elimination on these random weights (free nodes after the forcing test)
    assert sum(int(s[:, 0].sum()) for s in stats) > 0


def test_blocks_beyond_lds_smoothing_dominated_flow():
    """Large blocks in global memory with smoothing far above the unaries: the push-relabel phase (its global-memory
    atomics, barrier slots and list compaction) runs in every block of the first iterations, and the state still
    equals the oracle's after every iteration."""
    # 8000 and 5760 nodes: one launch per block; 9000 (above 8192): the prologue and a first elimination spread
    # over several workgroups per block, then the flow phases
    for conn, dims, block in [(8, (180, 150, 1), (100, 80, 1)), (6, (34, 30, 26), (20, 18, 16)),
                              (8, (190, 170, 1), (100, 90, 1))]:
        p = synth.random_problem(27, dims, conn, block, (2, 2, 2 if conn == 6 else 0), lam_q8=512,
                                 u_range=(-400, 400), w_range=(200, 1000), mu0=4000)
        stats = []
        d, _, _ = run_parity(p, 4, f"beyond LDS, smoothing-dominated conn={conn}", stats=stats)
        d.close()
        assert int(stats[0][:, 0].sum()) > 0 and int(stats[0][:, 1].sum()) > 0 and int(stats[0][:, 2].sum()) > 0


@pytest.mark.parametrize("conn,dims,block,overlap", [(8, (40, 30, 1), (2, 2, 1), (1, 1, 0)),
                                                     (6, (14, 12, 10), (2, 2, 2), (1, 1, 1))],
                         ids=["8-connected 2x2 blocks", "6-connected 2x2x2 blocks"])
def test_tiny_blocks_every_iteration(conn, dims, block, overlap):
    """Blocks of 2 pixels per axis overlapping by 1: every pixel is a boundary pixel owned by its own block, so a
    256-pixel consensus chunk spans far more owner blocks than it keeps residual slots for in LDS and most residuals
    go to the global sums directly.  Whole state equal to the oracle's after every iteration."""
    p = synth.random_problem(29, dims, conn, block, overlap)
    d, _, _ = run_parity(p, 4, f"tiny blocks conn={conn}")
    d.close()


# blocks whose per-node arrays alone exceed the LDS too (9 + m bytes per node: 16384-pixel blocks with the 3x3
# stencils, 16^3 blocks of the radius-4 ball), so the whole max-flow state stays in the workspace
GLOBAL_STATE_CASES = [
    ("8-connected 2x2 blocks of 128x128", 8, (250, 250, 1), (128, 128, 1), (2, 2, 0), 1),
    ("radius-4 ball 2x2x1 blocks of 16^3", 256, (24, 24, 16), (16, 16, 16), (4, 4, 4), 32),
]


@pytest.mark.parametrize("label,conn,dims,block,overlap,mb", GLOBAL_STATE_CASES, ids=[c[0] for c in GLOBAL_STATE_CASES])
def test_blocks_with_all_state_in_global_memory(label, conn, dims, block, overlap, mb):
    """The global-memory block solver keeps its per-node arrays in LDS when they fit; these blocks are too large
    even for that, so the whole state (and the barrier slots) lives in the workspace.  Smoothing well above the
    unaries makes the push-relabel phase run; the state equals the oracle's after every iteration."""
    np_max = block[0] * block[1] * block[2]
    assert 64 + np_max * (9 + mb) > 160 * 1024 - 1024   # beyond the LDS for the per-node arrays alone
    p = synth.random_problem(28, dims, conn, block, overlap, lam_q8=512 if conn == 8 else 64,
                             u_range=(-400, 400), w_range=(200, 1000) if conn == 8 else (20, 100), mu0=4000)
    stats = []
    d, _, _ = run_parity(p, 3, f"all state in global memory, {label}", stats=stats)
    d.close()
    assert int(stats[0][:, 0].sum()) > 0 and int(stats[0][:, 1].sum()) > 0


PAPER_PARTITIONS = [(32, 25), (64, 10), (64, 0), (128, 0), (128, 25)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("K,pct", PAPER_PARTITIONS, ids=[f"K{k}_size{p:02d}" for k, p in PAPER_PARTITIONS])
def test_paper_partitions_2d_every_iteration(K, pct):
    """The 512x512 image in the 2D experiments' partitions (K even blocks, Size_00 / Size_10 / Size_25): blocks of
    2048 to 12800 pixels, in LDS or beyond it; whole state after every iteration, then the labels of the solve."""
    p = synth.config2_sized(K, pct)
    d, st, dec = run_parity(p, 3, f"paper partition K={K} Size_{pct:02d}: block={p.block} overlap={p.overlap}")
    d.close()
    st_o, infos, _, _ = od.run(p, dec=dec)
    with make_ctx(p) as e:
        info = e.solve()
        assert info["iters_done"] == len(infos) and np.array_equal(e.labels(), od.labels(st_o.Y))


@pytest.mark.timeout(900)
def test_paper_partition_3d_every_iteration():
    """The 128x128x64 volume in 128 blocks grown by 10 % (the paper's 3D setting): 18x35x18 blocks of 11340 voxels
    in global memory; whole state after each of 3 iterations."""
    p = synth.config3_sized(128, 10)
    d, st, dec = run_parity(p, 3, f"paper partition 3D K=128 Size_10: block={p.block} overlap={p.overlap}")
    d.close()


@pytest.mark.parametrize("K", [32, 64])
def test_even_partition_full_solve(K):
    """The 512x512 image split into 32 or 64 even blocks (66x130 / 66x66 pixels, beyond the LDS): the solve
    equals the oracle's (iterations, state, labels, energy); a batch refuses such blocks."""
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Batch
    p = synth.config2_even(K)
    announce(f"even partition K={K}: block={p.block}")
    st_o, infos, _, dec = od.run(p)
    d = make_ctx(p)
    try:
        info = d.solve()
        assert info["iters_done"] == len(infos)
        assert info["converged"] == infos[-1].converged
        Y, A, yh, mu, t = d.get_state()
        assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
        l = d.labels()
        assert np.array_equal(l, od.labels(st_o.Y))
        assert d.energy() == od.energy_q(dec, l)
        with pytest.raises(N.DopeError) as err:
            Batch([d])
        assert err.value.status == N.DOPE_EINVAL
    finally:
        d.close()


def test_solve_straight_after_upload():
    """A solve straight after an energy upload runs under the loop control that the setup kernel leaves
    (validated, limit max_iter, halting when the stopping rule holds), with no control-setup launch; a solve after
    iterate() goes through the control-setup kernel.  Every order equals the oracle, also when max_iter cuts the
    solve short."""
    import torch
    from paper_1704_03116_amd.solver import Dope
    announce("solve straight after the energy upload")
    full = synth.config2(W=96, H=80)
    short = synth.config2(W=96, H=80)
    short.max_iter = 1
    for p in (full, short):
        st_o, infos_o, _, _ = od.run(p)
        for mode in ("sync", "async", "async-device", "iterate0", "iterate1"):
            with Dope.from_problem(p) as d:
                u = np.ascontiguousarray(p.u, np.int32)
                w = np.ascontiguousarray(p.w, np.int32)
                if mode == "sync":
                    d.set_energy(u, w, p.lam_q8)
                elif mode == "async-device":
                    d.set_energy_async(torch.from_numpy(u).cuda(), torch.from_numpy(w).cuda(), p.lam_q8)
                else:
                    d.set_energy_async(u, w, p.lam_q8)
                if mode.startswith("iterate"):
                    d.iterate(int(mode[-1]))
                info = d.solve()
                assert info["iters_done"] == len(infos_o), (p.max_iter, mode)
                assert info["converged"] == infos_o[-1].converged, (p.max_iter, mode)
                Y, A, yh, mu, t = d.get_state()
                assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)
                assert d.solve()["iters_done"] == len(infos_o)   # nothing more to do


def test_setup_verdict_sees_every_workgroup():
    """The set-up's validation verdict is taken by its last workgroup over the bits of all of them (1024
    workgroups at 512x512): a single bad weight anywhere is reported, by the blocking and the deferred upload."""
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Dope
    announce("setup verdict over every workgroup (512x512)")
    base = synth.config2()
    W, H = base.dims[0], base.dims[1]
    rng = np.random.default_rng(5)
    cases = []
    for pos in (0, (H - 2) * W + W - 1, int(rng.integers(W * (H - 1)))):
        neg = np.array(base.w, np.int32, copy=True)
        neg[1, pos] = -3           # the (0, 1) edge of a pixel above the last row
        cases.append((neg, N.DOPE_ENOTSUBMODULAR))
    off = np.array(base.w, np.int32, copy=True)
    off[0, W * H - 1] = 7          # +x neighbour of the last pixel lies off the grid
    cases.append((off, N.DOPE_EINVAL))
    for w, status in cases:
        with Dope.from_problem(base, solver="maxflow") as d:
            with pytest.raises(N.DopeError) as err:
                d.set_energy(np.ascontiguousarray(base.u, np.int32), w, base.lam_q8)
            assert err.value.status == status
            d.set_energy_async(np.ascontiguousarray(base.u, np.int32), w, base.lam_q8)
            with pytest.raises(N.DopeError) as err:
                d.solve()
            assert err.value.status == status
            assert d.get_state()[4] == 0
            d.set_energy(np.ascontiguousarray(base.u, np.int32), np.ascontiguousarray(base.w, np.int32),
                         base.lam_q8)
            assert d.solve()["converged"]


def test_upload_after_an_unvalidated_rejected_one():
    """Two uploads in a row with no readback between them: the first (negative weights, max-flow solver) is
    rejected by its verdict, taken before the second set-up runs, so its bits do not reach the second's; the
    second solves like the oracle."""
    from paper_1704_03116_amd.solver import Dope
    announce("upload after an unvalidated rejected upload")
    q = synth.random_problem(16, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0), neg_frac=0.3)
    good = synth.random_problem(17, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0))
    st_o, infos, _, _ = od.run(good)
    with Dope.from_problem(good, solver="maxflow") as e:
        e.set_energy_async(q.u, q.w, q.lam_q8)
        e.set_energy_async(good.u, good.w, good.lam_q8)
        info = e.solve()
        assert info["iters_done"] == len(infos)
        Y, A, yh, mu, t = e.get_state()
        assert np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)


def test_deferred_validation_through_solve_and_batch():
    """The verdict of an asynchronous energy is taken by whichever call comes next: a solve, or a batch; a valid
    energy loaded after an invalid one runs normally."""
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Batch, Dope
    announce("deferred validation: solve, batch, reload")
    q = synth.random_problem(16, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0), neg_frac=0.3)
    good = synth.random_problem(17, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0))
    with Dope.from_problem(q, solver="maxflow") as e:
        e.set_energy_async(q.u, q.w, q.lam_q8)
        with pytest.raises(N.DopeError) as err:
            e.solve()
        assert err.value.status == N.DOPE_ENOTSUBMODULAR
        e.set_energy_async(good.u, good.w, good.lam_q8)
        e.iterate(3)
        st_o, _, _, _ = od.run(good, n_iter=3)
        Y, A, yh, mu, t = e.get_state()
        assert t == 3 and np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A)
    a = Dope.from_problem(good, solver="maxflow")
    b = Dope.from_problem(q, solver="maxflow")
    try:
        a.set_energy_async(good.u, good.w, good.lam_q8)
        b.set_energy_async(q.u, q.w, q.lam_q8)
        with Batch([a, b]) as bt:
            with pytest.raises(N.DopeError) as err:
                bt.iterate(2)
            assert err.value.status == N.DOPE_ENOTSUBMODULAR
            info = bt.info()
        assert info[0]["iters_done"] == 2 and info[1]["iters_done"] == 0
        st_o, _, _, _ = od.run(good, n_iter=2)
        assert np.array_equal(a.get_state()[0], st_o.Y)
    finally:
        a.close()
        b.close()


# ------------------------------------------------------------------------------------------------------------
# serving: continuous batching; every request equals its solve alone; admission within the HBM budget
# ------------------------------------------------------------------------------------------------------------

def _serve_requests():
    reqs = []
    for r, (W, H, B) in enumerate([(70, 50, 16), (40, 90, 16), (128, 96, 32), (33, 33, 16), (150, 40, 32),
                                   (64, 64, 16), (96, 120, 32), (48, 48, 16)]):
        p = synth.config2(seed=40 + r, W=W, H=H)
        p.block, p.overlap = (B, B, 1), ((2, 2, 0) if B == 32 else (1, 1, 0))
        p.mu0 = 250
        p.max_iter = 12
        reqs.append(p)
    return reqs


@pytest.mark.parametrize("iters_per_step", [1, 3])
def test_serving_mix_equals_alone(iters_per_step):
    import torch
    from paper_1704_03116_amd.solver import Server, params_from_problem
    reqs = _serve_requests()
    announce(f"serving {len(reqs)} requests, staggered submission, {iters_per_step} iterations per step")
    outs = [torch.zeros(p.n, dtype=torch.uint8, device="cuda") for p in reqs]
    ins = [(torch.from_numpy(np.ascontiguousarray(p.u)).cuda(), torch.from_numpy(np.ascontiguousarray(p.w)).cuda())
           for p in reqs]
    torch.cuda.synchronize()
    done, tickets = {}, {}
    with Server(hbm_budget=64 << 20, max_active=5, iters_per_step=iters_per_step) as srv:
        nxt = 0
        for tick in range(200):
            if nxt < len(reqs) and tick % 2 == 0:            # a request arrives every other tick
                p = reqs[nxt]
                tickets[srv.submit(params_from_problem(p), ins[nxt][0], ins[nxt][1], p.lam_q8, outs[nxt])] = nxt
                nxt += 1
            for t in srv.step():
                done[tickets[t]] = srv.result(t)
            waiting, active, used = srv.load()
            assert active <= 5 and used <= 64 << 20
            if len(done) == len(reqs):
                break
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    for i, p in enumerate(reqs):
        status, info = done[i]
        assert status == 0
        d = make_ctx(p)
        alone = d.solve()
        assert info["iters_done"] == alone["iters_done"] and info["converged"] == alone["converged"], p.name
        assert np.array_equal(outs[i].cpu().numpy(), d.labels()), f"request {i}: served labels differ from alone"
        d.close()
    # and against the oracle for two of them
    for i in (0, 2):
        st_o, infos, _, _ = od.run(reqs[i])
        assert np.array_equal(outs[i].cpu().numpy(), od.labels(st_o.Y))


def test_serving_admission_budget_and_busy():
    import torch
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Server, params_from_problem
    from paper_1704_03116_amd._native import dope_workspace_bytes
    import ctypes
    reqs = _serve_requests()[:6]
    need = [dope_workspace_bytes(ctypes.byref(params_from_problem(p))) for p in reqs]
    budget = (sorted(need)[-1] + sorted(need)[-2] + 1024) // 256 * 256 + 512
    announce(f"serving with a budget of {budget} bytes")
    outs = [torch.zeros(p.n, dtype=torch.uint8, device="cuda") for p in reqs]
    with Server(hbm_budget=budget, max_active=16) as srv:
        tk = {}
        for i, p in enumerate(reqs):
            tk[srv.submit(params_from_problem(p), np.ascontiguousarray(p.u), np.ascontiguousarray(p.w), p.lam_q8,
                          outs[i])] = i
        big = synth.config2(W=900, H=900)
        with pytest.raises(N.DopeError) as e:
            srv.submit(params_from_problem(big), np.ascontiguousarray(big.u), np.ascontiguousarray(big.w),
                       big.lam_q8, torch.zeros(big.n, dtype=torch.uint8, device="cuda"))
        assert e.value.status == N.DOPE_EBUSY
        finished = 0
        for _ in range(400):
            finished += len(srv.step())
            waiting, active, used = srv.load()
            assert used <= budget
            if finished == len(reqs):
                break
        assert finished == len(reqs)


# ------------------------------------------------------------------------------------------------------------
# ties: energies with many minimisers, where only the canonical choice of the block labelling decides the result
# ------------------------------------------------------------------------------------------------------------

TIE_CASES = [
    # label, dims, conn, block, overlap, solver, unary range, weight range
    ("4-connected LDS", (40, 36, 1), 4, (8, 8, 1), (1, 1, 0), "maxflow", (-2, 2), (0, 2)),
    ("8-connected LDS", (48, 40, 1), 8, (16, 16, 1), (2, 2, 0), "maxflow", (-2, 2), (0, 2)),
    ("6-connected LDS", (20, 18, 16), 6, (8, 8, 8), (1, 1, 1), "maxflow", (-2, 2), (0, 2)),
    ("5x5 LDS", (30, 28, 1), 24, (10, 10, 1), (2, 2, 0), "maxflow", (-6, 6), (0, 1)),
    ("8-connected beyond the LDS", (150, 120, 1), 8, (100, 90, 1), (2, 2, 0), "maxflow", (-2, 2), (0, 2)),
    ("4-connected exhaustive", (23, 19, 1), 4, (4, 4, 1), (1, 1, 0), "exhaustive", (-2, 2), (0, 2)),
]


def tie_counts(p, dec):
    """Iteration-1 block problems with more than one minimiser.  Max-flow blocks: the minimal minimiser differs
    from the maximal one, which is 1 - (minimal minimiser of the problem with negated unaries).  Enumerated
    blocks: brute force over all 2^|block| labellings counts the minimisers."""
    st = od.initial_state(dec, p.mu0)
    n_multi = 0
    for k in range(len(dec.blocks)):
        a, b = dec.offsets[k], dec.offsets[k + 1]
        Ut, ea, eb, cap = od.block_subproblem(dec, k, st.Y, st.A[a:b], st.M)
        if p.solver == "maxflow":
            lo, _ = od.solve_subproblem(Ut, ea, eb, cap, "maxflow")
            neg, _ = od.solve_subproblem(-Ut, ea, eb, cap, "maxflow")
            n_multi += int(not np.array_equal(lo, 1 - neg))
        else:
            m = len(Ut)
            codes = np.arange(1 << m, dtype=np.int64)
            bits = (codes[:, None] >> np.arange(m)) & 1
            e = bits @ np.asarray(Ut, np.int64)
            for i, j, c in zip(ea, eb, cap):
                e += int(c) * (bits[:, i] != bits[:, j])
            n_multi += int(np.sum(e == e.min()) > 1)
    return n_multi, len(dec.blocks)


@pytest.mark.parametrize("case", TIE_CASES, ids=[c[0] for c in TIE_CASES])
def test_tie_prone_energies_every_iteration(case):
    """Unaries in {-2..2} (zeros included) and weights in {0, 1, 2} at lambda = 1 (the 5x5 stencil: {-6..6} and
    {0, 1}): at iteration 1 the block unary
    is u 2^14 / q and an edge's capacity w 2^14 / (q_i q_j), so zero unaries, |U~| equal to the sum of the node's
    capacities and blocks with several minimisers are common (asserted first, through the oracle: at least 20 % of
    the iteration-1 block solves).  The whole state is then compared bit for bit after every iteration."""
    label, dims, conn, block, overlap, solver, u_range, w_range = case
    p = synth.random_problem(51, dims, conn, block, overlap, lam_q8=256, u_range=u_range, w_range=w_range,
                             neg_frac=0.3 if solver == "exhaustive" else 0.0, mu0=3, solver=solver)
    dec = od.decompose(p)
    n_multi, K = tie_counts(p, dec)
    announce(f"ties, {label}: {n_multi} of {K} iteration-1 block solves have several minimisers")
    assert n_multi >= 0.2 * K
    stats = []
    d, _, _ = run_parity(p, 6, f"ties, {label}", stats=stats, dec=dec)
    if solver == "maxflow":
        # the flow phase ran (free nodes after forcing, push-relabel rounds)
        assert sum(int(s[:, 0].sum()) for s in stats) > 0
    d.close()


def test_solve_with_no_iteration_reports_a_rejected_upload():
    """max_iter = 0: a solve straight after an asynchronous upload runs no iteration, yet takes the pending
    verdict: a rejected energy (negative weights, max-flow solver) is reported by the solve, and a valid energy
    uploaded next is accepted (the rejected one's validation bits do not reach it) and solves like the oracle."""
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import Dope
    announce("max_iter = 0 after a rejected asynchronous upload")
    bad = synth.random_problem(16, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0), neg_frac=0.3)
    good = synth.random_problem(17, (20, 20, 1), 4, (8, 8, 1), (1, 1, 0))
    with Dope.from_problem(good, solver="maxflow", max_iter=0) as e:
        e.set_energy_async(bad.u, bad.w, bad.lam_q8)
        with pytest.raises(N.DopeError) as err:
            e.solve()
        assert err.value.status == N.DOPE_ENOTSUBMODULAR
        e.set_energy_async(good.u, good.w, good.lam_q8)
        info = e.solve()
        assert info["iters_done"] == 0
        e.iterate(3)
        st_o, _, _, _ = od.run(good, n_iter=3)
        Y, A, yh, mu, t = e.get_state()
        assert t == 3 and np.array_equal(Y, st_o.Y) and np.array_equal(A, st_o.A) and np.array_equal(yh, st_o.yhat)


# ------------------------------------------------------------------------------------------------------------
# non-submodular blocks beyond enumeration: the LSA-TR block solver
# ------------------------------------------------------------------------------------------------------------

LSATR_CASES = [
    # label, dims, conn, block, overlap
    ("4-connected 8x8 blocks", (40, 34, 1), 4, (8, 8, 1), (1, 1, 0)),
    ("4-connected 16x16 blocks o=2", (70, 50, 1), 4, (16, 16, 1), (2, 2, 0)),
    ("8-connected 12x12 blocks", (45, 40, 1), 8, (12, 12, 1), (1, 1, 0)),
    ("6-connected 6^3 blocks", (20, 17, 14), 6, (6, 6, 6), (1, 1, 1)),
    ("4-connected 40x40 blocks", (100, 90, 1), 4, (40, 40, 1), (2, 2, 0)),
]


@pytest.mark.parametrize("case", LSATR_CASES, ids=[c[0] for c in LSATR_CASES])
def test_lsatr_nonsubmodular_every_iteration(case):
    """Repulsive edges (30 %) in blocks larger than enumeration allows: the LSA-TR steps of every block, the
    consensus and the multipliers equal the oracle's bit for bit after every iteration; the block search takes
    several steps somewhere."""
    label, dims, conn, block, overlap = case
    p = synth.random_problem(61, dims, conn, block, overlap, lam_q8=256, u_range=(-1000, 1000),
                             w_range=(50, 500), neg_frac=0.3, mu0=2000, solver="lsatr")
    stats = []
    d, _, _ = run_parity(p, 6, f"LSA-TR, {label}", stats=stats)
    assert max(int(s[:, 2].max()) for s in stats) >= 2
    d.close()


def test_lsatr_on_submodular_blocks_equals_maxflow():
    """Without repulsive edges the first LSA-TR step of every block is the minimal minimum cut and the second finds
    nothing better and stops: the whole ADMM state equals the max-flow solver's."""
    p = synth.random_problem(62, (60, 44, 1), 8, (16, 16, 1), (2, 2, 0), lam_q8=256, mu0=1000)
    q = dataclasses.replace(p, solver="lsatr")
    a, b = make_ctx(p, solver="maxflow"), make_ctx(q, solver="lsatr")
    for _ in range(5):
        a.iterate(1)
        b.iterate(1)
        sa, sb = a.get_state(), b.get_state()
        assert all(np.array_equal(x, y) for x, y in zip(sa[:3], sb[:3])) and sa[3:] == sb[3:]
    assert int(b.block_stats()[:, 2].max()) <= 2
    a.close()
    b.close()


@pytest.mark.timeout(600)
def test_config4_lsatr_full_size_every_iteration():
    """The 256x256 non-submodular grid in 16x16 blocks (289 LSA-TR blocks): 3 iterations, whole state."""
    d, st, dec = run_parity(synth.config4_lsatr(), 3, "config4 256x256 LSA-TR 16x16 blocks full size")
    d.close()
