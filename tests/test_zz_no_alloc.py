"""The entry point that allocates nothing (dope_solve_noalloc, device state in the library's static array) against
the context path (dope_set_energy_async + dope_solve + dope_labels on a dope_ctx) and the oracle: two calls in a row,
the second on a smaller image, so that the second reuses the array the first left behind."""
import numpy as np
import pytest

import synth
from oracle import dope as od

pytestmark = pytest.mark.gpu


def _context_solve(p, u, w):
    import torch
    from paper_1704_03116_amd.solver import Dope
    lab = torch.empty(p.n, dtype=torch.uint8, device="cuda")
    with Dope.from_problem(p) as d:
        d.set_energy_async(u, w, p.lam_q8)
        info = d.solve()
        d.labels(lab)
        torch.cuda.synchronize()
    return lab.cpu().numpy(), info


def _noalloc_solve(p, u, w):
    import torch
    from paper_1704_03116_amd.solver import params_from_problem, solve_noalloc
    lab = torch.full((p.n,), 7, dtype=torch.uint8, device="cuda")
    info = solve_noalloc(params_from_problem(p), u, w, p.lam_q8, lab)
    return lab.cpu().numpy(), info


def test_noalloc_matches_context_solve_twice_shrinking():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    cases = [synth.config2(W=300, H=260, seed=4),                # 8-connected, 32x32 blocks, o = 2
             synth.config3(dims=(40, 36, 20), seed=2),           # smaller, 6-connected volume
             synth.config1(size=48)]                             # smaller still, 4-connected
    for p in cases:
        print(f"\n[gpu] no-alloc solve: {p.name} dims={p.dims} conn={p.conn} block={p.block}", flush=True)
        u = torch.from_numpy(np.ascontiguousarray(p.u, np.int32)).cuda()
        w = torch.from_numpy(np.ascontiguousarray(p.w, np.int32)).cuda()
        lab_n, info_n = _noalloc_solve(p, u, w)
        lab_c, info_c = _context_solve(p, u, w)
        assert info_n == info_c, (info_n, info_c)
        assert np.array_equal(lab_n, lab_c)
        st_o, infos, _, _ = od.run(p)
        assert info_n["iters_done"] == len(infos) and info_n["converged"] == infos[-1].converged
        assert np.array_equal(lab_n, od.labels(st_o.Y))


def test_noalloc_rejects_problems_beyond_the_array():
    import torch
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import make_params, solve_noalloc
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    prm = make_params((4096, 4096), 8, (32, 32), (2, 2), 1000)
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
    lab = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.DopeError) as e:
        solve_noalloc(prm, dummy, dummy, 256, lab)
    assert e.value.status == N.DOPE_EINVAL
    assert "static scratch" in str(e.value)
