"""Run by test_debug_build_cut_checks_hold in a process of its own: problems whose blocks run push-relabel go
through the instrumented library (libdope_debug.so, whose 3x3-stencil block max-flow checks its canonical cut
and reports a violation as a solver error).  Every iteration must succeed and leave the whole state equal to the
oracle's.  Prints one line per case and exits non-zero on the first failure."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1704_03116_amd import _native as N  # noqa: E402

N.LIB_PATH = os.path.join(ROOT, "paper_1704_03116_amd", "libdope_debug.so")

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import dope as od  # noqa: E402
from paper_1704_03116_amd.solver import Dope  # noqa: E402

CASES = [
    # label, problem, iterations
    ("8-connected smoothing-dominated, LDS", synth.random_problem(12, (48, 40, 1), 8, (16, 16, 1), (1, 1, 0),
                                                                  lam_q8=768, u_range=(-400, 400),
                                                                  w_range=(200, 1000), mu0=800), 4),
    ("4-connected tie-prone, LDS", synth.random_problem(51, (40, 36, 1), 4, (8, 8, 1), (1, 1, 0), lam_q8=256,
                                                        u_range=(-2, 2), w_range=(0, 2), mu0=3), 4),
    ("6-connected tie-prone, LDS", synth.random_problem(51, (20, 18, 16), 6, (8, 8, 8), (1, 1, 1), lam_q8=256,
                                                        u_range=(-2, 2), w_range=(0, 2), mu0=3), 4),
    ("8-connected smoothing-dominated, two-launch global memory",
     synth.random_problem(27, (190, 170, 1), 8, (100, 90, 1), (2, 2, 0), lam_q8=512, u_range=(-400, 400),
                          w_range=(200, 1000), mu0=4000), 3),
]


def main():
    threads = min(16, os.cpu_count() or 1)
    for label, p, n_iter in CASES:
        print(f"[debug build] {label}: dims={p.dims} conn={p.conn} block={p.block} iters={n_iter}", flush=True)
        dec = od.decompose(p)
        st = od.initial_state(dec, p.mu0)
        rounds = 0
        with Dope.from_problem(p) as d:
            d.set_energy(np.ascontiguousarray(p.u, np.int32), np.ascontiguousarray(p.w, np.int32), p.lam_q8)
            for t in range(1, n_iter + 1):
                st, inf = od.iterate(dec, st, threads=threads, mu_num=p.mu_num, mu_den=p.mu_den,
                                     eps_q16=p.eps_q16)
                status, info = d.iterate_status(1)
                if status != N.DOPE_OK:
                    print(f"FAIL {label}: iteration {t} status {status} ({N.STATUS_NAMES.get(status)})", flush=True)
                    return 1
                rounds += int(d.block_stats()[:, 1].sum())
                Y, A, yh, mu, tt = d.get_state()
                if not (np.array_equal(Y, st.Y) and np.array_equal(A, st.A) and np.array_equal(yh, st.yhat)
                        and mu == st.M and tt == st.t):
                    print(f"FAIL {label}: state differs from the oracle at iteration {t}", flush=True)
                    return 1
        if rounds == 0:
            print(f"FAIL {label}: no push-relabel round ran", flush=True)
            return 1
        print(f"ok {label}: {rounds} push-relabel rounds", flush=True)
    print("debug build ok", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
