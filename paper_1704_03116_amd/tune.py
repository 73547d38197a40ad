#!/usr/bin/env python3
"""Offline sweep behind dope_autotune: times whole solves (energy upload, dope_solve to the stopping rule or the
iteration cap, labels) of serving-style images for every candidate block size and overlap, per stencil and image
size, on the GPU, and writes the winners as the table the library compiles in (csrc/autotune_table.h) together
with the raw measurements (JSON).  The table maps (connectivity, shorter side) to (B, o), so the library's choice
stays a pure function of the image shape and stencil.

Candidates are the blocks whose max-flow state fits the LDS (batches and the server take only those) with stride
B - o at least the stencil radius.  Images: the serving workload's grey disk at each size (2D; contrast weights of
the stencil) and the sphere volume (3D).  Run from the repository root on an MI355X:

    python paper_1704_03116_amd/tune.py --json autotune_sweep.json --header autotune_table.h
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

LDS_LIMIT = 163840 - 1024   # the max-flow kernels keep 1 KiB of the 160 KiB for static arrays
HALF = {4: 2, 8: 4, 24: 12, 48: 24, 80: 40, 6: 3, 32: 16, 122: 61, 256: 128}
RADIUS = {4: 1, 8: 1, 24: 2, 48: 3, 80: 4, 6: 1, 32: 2, 122: 3, 256: 4}

# stencil -> (image sizes: shorter side of a square image or cube edge, candidate (B, o))
SWEEP_2D = {
    4: ([128, 256, 512, 1024, 2048], [(16, 1), (16, 2), (32, 1), (32, 2), (64, 1), (64, 2)]),
    8: ([128, 256, 512, 1024, 2048], [(16, 1), (16, 2), (32, 1), (32, 2), (48, 1), (48, 2)]),
    24: ([128, 256, 512, 1024], [(16, 2), (16, 4), (24, 2), (32, 2), (32, 4)]),
    48: ([128, 256, 512], [(16, 1), (16, 2), (24, 1), (24, 2)]),
    80: ([128, 256, 512], [(16, 1), (16, 2), (20, 1), (20, 2)]),
}
SWEEP_3D = {
    6: ([32, 64, 96], [(8, 1), (12, 1), (12, 2), (16, 1), (16, 2)]),
    32: ([32, 64], [(6, 1), (8, 1), (8, 2), (10, 1), (10, 2)]),
    122: ([24, 32], [(5, 1), (6, 1), (6, 2)]),
}


def dir_mask_bytes(h):
    return 1 if 2 * h <= 8 else (4 if 2 * h <= 32 else (8 if 2 * h <= 64 else 16))


def fits_lds(B, ndim, conn):
    h = HALF[conn]
    mb = dir_mask_bytes(h)
    n = B ** ndim
    return 64 + n * (8 * h + 9 + mb) + (16 if mb > 8 else (8 if mb > 1 else 0)) <= LDS_LIMIT


def image(ndim, conn, side, seed):
    import synth
    if ndim == 2:
        return synth.config5_image(side, side, lam=1.5, seed=seed, conn=conn)
    dims = (side, side, max(16, side // 2))
    if conn == 6:
        return synth.config3(seed=seed, dims=dims)
    return synth.config3_kernel5(seed=seed, dims=dims, k=5 if conn == 32 else 7)


def time_solve(p, B, o, reps):
    import numpy as np
    import torch
    from paper_1704_03116_amd.solver import Dope
    blk = (B, B, B if p.ndim == 3 else 1)
    ovl = (o, o, o if p.ndim == 3 else 0)
    d = Dope(p.dims, p.conn, blk, ovl, p.mu0, ndim=p.ndim, mu_fact=(p.mu_num, p.mu_den), eps_q16=p.eps_q16,
             max_iter=p.max_iter, solver="maxflow")
    u = torch.from_numpy(np.ascontiguousarray(p.u, np.int32)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(p.w, np.int32)).cuda()
    lab = torch.empty(p.n, dtype=torch.uint8, device="cuda")
    info = None
    times = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.set_energy_async(u, w, p.lam_q8)
        info = d.solve()
        d.labels(lab)
        torch.cuda.synchronize()
        if r > 0:
            times.append(time.perf_counter() - t0)
    d.close()
    best = min(times)
    return {"B": B, "o": o, "ms": round(best * 1e3, 4), "mpx_s": round(p.n / best / 1e6, 2),
            "iterations": info["iters_done"], "converged": bool(info["converged"])}


def table_rows(results):
    """(ndim, conn, largest shorter side, B, o) per measured shorter side: an image takes the row of the measured
    image whose shorter side is nearest (class bounds at the geometric means of neighbouring shorter sides); the
    last row of a stencil has no upper bound."""
    table = []
    for sw in results:
        # one row per shorter side: of measured images with the same shorter side the largest decides
        by_short = {}
        for r in sorted(sw["rows"], key=lambda r: (min(r["dims"]), math.prod(r["dims"]))):
            by_short[min(r["dims"])] = r
        rows = [by_short[k] for k in sorted(by_short)]
        for i, r in enumerate(rows):
            if i + 1 < len(rows):
                bound = int(math.sqrt(min(r["dims"]) * min(rows[i + 1]["dims"])))
            else:
                bound = 2 ** 31 - 1
            table.append((sw["ndim"], sw["conn"], bound, r["best"]["B"], r["best"]["o"]))
    return table


def write_header(path, table):
    lines = ["// Block partition table of dope_autotune, written by paper_1704_03116_amd/tune.py from an MI355X sweep",
             "// (whole-solve throughput of serving-style images per stencil and size; the measurements are kept in",
             "// profiles/autotune_sweep.json).  Row: ndim, connectivity, largest shorter side, block edge B, overlap o.",
             "#pragma once", "", "namespace dope {", "",
             "struct TuneRow {", "    int ndim, conn, max_short_side, block, overlap;", "};", "",
             "constexpr TuneRow TUNE_TABLE[] = {"]
    for ndim, conn, bound, B, o in table:
        lines.append(f"    {{{ndim}, {conn}, {bound}, {B}, {o}}},")
    lines += ["};", "", "}  // namespace dope", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--json", required=True)
    ap.add_argument("--header", required=True)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--from-json", action="store_true",
                    help="write the header from an existing sweep file (--json) instead of measuring")
    args = ap.parse_args()
    if args.from_json:
        write_header(args.header, table_rows(json.load(open(args.json))["sweeps"]))
        print(f"[tune] wrote {args.header} from {args.json}", flush=True)
        return
    import torch
    torch.cuda.set_device(0)
    results = []
    for ndim, sweep in ((2, SWEEP_2D), (3, SWEEP_3D)):
        for conn, (sides, cands) in sweep.items():
            rows = []
            for side in sides:
                p = image(ndim, conn, side, seed=side)
                runs = []
                for B, o in cands:
                    if not fits_lds(B, ndim, conn) or B - o < RADIUS[conn] or 2 * o > B or B >= side:
                        continue
                    runs.append(time_solve(p, B, o, args.reps))
                best = max(runs, key=lambda r: r["mpx_s"])
                print(f"[tune] ndim={ndim} conn={conn} side={side}: best B={best['B']} o={best['o']} "
                      f"{best['mpx_s']} Mpx/s of {len(runs)} candidates", flush=True)
                rows.append({"side": side, "dims": list(p.dims[:ndim]), "runs": runs, "best": best})
            results.append({"ndim": ndim, "conn": conn, "rows": rows})
    with open(args.json, "w") as f:
        json.dump({"gpu": torch.cuda.get_device_name(0), "reps": args.reps,
                   "metric": "Mpixel/s of a whole solve (upload, solve to the stopping rule or 50 iterations, labels); "
                             "best of reps after one warm-up",
                   "sweeps": results}, f, indent=1)
    write_header(args.header, table_rows(results))
    print(f"[tune] wrote {args.json} and {args.header}", flush=True)


if __name__ == "__main__":
    main()
