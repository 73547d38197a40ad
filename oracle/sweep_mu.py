"""Sweep of the ADMM penalty mu0 on the 64x64 disk, the 512x512 ellipse image and the 128x128x64 sphere volume,
with the oracle only (test infrastructure: run by hand, not by the library).

The paper gives mu0 = 100 (2D) and 500 (3D) with mu_fact = 1.05 in units it does not state, and says only that
the method is not very sensitive to mu as long as mu is large enough (Sec. 2, after Eq. 11; Sec. 3 setup).
With the x1000 integer inputs used here the scale differs, so this sweep picks the defaults: for each mu0 it
records the iterations until the stopping rule holds (eps = 0.1, cap 50), the final sqrt(max_k r_k) in units of y,
the relative energy gap of Eq. (12) against the global minimum cut, and the Dice overlap with that cut.

    python -m oracle.sweep_mu [--out oracle/mu_sweep.json] [--configs 1,2,3]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dope  # noqa: E402

SWEEP = {
    1: [100, 300, 1000, 3000, 10000],
    2: [100, 300, 1000, 3000, 10000],
    3: [500, 1500, 5000, 15000, 50000],
}


def problem(cfg):
    return {1: synth.config1, 2: synth.config2, 3: synth.config3}[cfg]()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "mu_sweep.json"))
    ap.add_argument("--configs", default="1,2,3")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    rows = []
    for cfg in [int(c) for c in args.configs.split(",")]:
        p = problem(cfg)
        t0 = time.perf_counter()
        dec = dope.decompose(p)
        x_gc, e_gc = dope.global_mincut(p)
        print(f"config {cfg} {p.name}: decomposition and global cut {time.perf_counter() - t0:.1f} s, "
              f"E_GC = {e_gc}", flush=True)
        for mu0 in SWEEP[cfg]:
            p.mu0 = mu0
            t0 = time.perf_counter()
            st, infos, _, _ = dope.run(p, threads=args.threads, dec=dec)
            el = time.perf_counter() - t0
            l = dope.labels(st.Y)
            e = dope.energy_q(dec, l)
            dice = 2.0 * float(np.sum(l & x_gc)) / max(1.0, float(np.sum(l) + np.sum(x_gc)))
            row = {"config": cfg, "workload": p.name, "mu0": mu0, "iterations": len(infos),
                   "converged": bool(infos[-1].converged), "overflow": bool(infos[-1].overflow),
                   "final_resid_y": round(float(np.sqrt(np.max(infos[-1].resid2))) / 65536.0, 4),
                   "E_dope": e, "E_GC": e_gc, "dE_eq12": (e - e_gc) / e_gc if e_gc else None,
                   "dE_rel_abs": (e - e_gc) / abs(e_gc) if e_gc else None, "dice_vs_GC": round(dice, 5),
                   "seconds": round(el, 2)}
            rows.append(row)
            print(json.dumps(row), flush=True)
    with open(args.out, "w") as f:
        json.dump({"eps_q16": synth.DEFAULT_EPS_Q16, "max_iter": 50, "mu_fact": "21/20", "rows": rows}, f,
                  indent=1)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
