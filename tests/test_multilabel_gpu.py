"""Alpha-expansion around DOPE on the GPU (dope_ml_*, through the C ABI) against the oracle's loop: labels and
energy after every expansion move, bit for bit, and the whole solve."""
import numpy as np
import pytest

from oracle import multilabel as ml
from synth.multilabel import multilabel_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1704_03116_amd import _native as N
    N.lib()


CASES = [
    ("8-connected, 4 labels", dict(seed=1, W=96, H=80, n_labels=4, conn=8, block=(32, 32), overlap=(2, 2))),
    ("4-connected, 3 labels, 16x16 blocks", dict(seed=2, W=70, H=50, n_labels=3, conn=4, block=(16, 16),
                                                  overlap=(1, 1))),
    ("5x5, 5 labels", dict(seed=3, W=64, H=48, n_labels=5, conn=24, block=(24, 24), overlap=(2, 2), lam=0.3)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_every_move_matches_the_oracle(case):
    from paper_1704_03116_amd.solver import MultiLabel
    label, kw = case
    p = multilabel_image(**kw)
    print(f"\n[gpu] multi-label {label}: {p.template.dims} nl={p.n_labels}", flush=True)
    L_o, E_o, recs = ml.alpha_expansion(p.template, p.D, p.V, max_cycles=3)
    with MultiLabel.from_problem(p) as m:
        m.set_energy(p.D, p.V)
        assert m.info()["energy"] == ml.energy(p.D, p.V, ml.initial_labels(p.D), p.template.dims, 2, p.template.conn)
        assert np.array_equal(m.labels(), ml.initial_labels(p.D))
        for r in recs:
            acc, e = m.step(r.label)
            assert (bool(acc), e) == (r.accepted, r.energy), (r.label, acc, e, r.accepted, r.energy)
            assert np.array_equal(m.labels(), r.labels)
    assert any(r.accepted for r in recs)


def test_solve_matches_the_oracle_and_counts():
    from paper_1704_03116_amd.solver import MultiLabel
    p = multilabel_image(seed=7, W=120, H=100, n_labels=4, conn=8, block=(32, 32), overlap=(2, 2))
    L_o, E_o, recs = ml.alpha_expansion(p.template, p.D, p.V, max_cycles=5)
    with MultiLabel.from_problem(p) as m:
        m.set_energy(p.D, p.V)
        info = m.solve(5)
        assert info["energy"] == E_o
        assert np.array_equal(m.labels(), L_o)
        assert info["moves"] == len(recs)
        assert info["accepted"] == sum(r.accepted for r in recs)
        assert info["binary_iterations"] == sum(r.binary_iterations for r in recs)


def test_device_inputs_and_errors():
    import torch
    from paper_1704_03116_amd import _native as N
    from paper_1704_03116_amd.solver import MultiLabel
    p = multilabel_image(seed=8, W=40, H=30, n_labels=3, conn=8, block=(16, 16), overlap=(1, 1))
    L_o, E_o, _ = ml.alpha_expansion(p.template, p.D, p.V, max_cycles=2)
    with MultiLabel.from_problem(p) as m:
        m.set_energy(torch.from_numpy(p.D).cuda(), torch.from_numpy(p.V).cuda())
        info = m.solve(2)
        out = torch.zeros(p.template.n, dtype=torch.uint8, device="cuda")
        m.labels(out)
        torch.cuda.synchronize()
        assert info["energy"] == E_o and np.array_equal(out.cpu().numpy(), L_o)
        bad = p.V.copy()
        bad[0, 5] = -1
        with pytest.raises(N.DopeError) as e:
            m.set_energy(p.D, bad)
        assert e.value.status == N.DOPE_ENOTSUBMODULAR
        bad = p.V.copy()
        bad[0, 39] = 7     # edge (+1, 0) of the last pixel of the first row leaves the grid
        with pytest.raises(N.DopeError) as e:
            m.set_energy(p.D, bad)
        assert e.value.status == N.DOPE_EINVAL
        with pytest.raises(N.DopeError):
            m.step(3)
