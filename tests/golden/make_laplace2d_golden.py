"""Write tests/golden/laplace2d_256_s8_m30.json: the oracle's complete FP64
solves of the 2-D Laplacian workload (256 x 256 grid, n = 65536, s = 8
N(0,1) right-hand sides from seed 2, m = 30, tol 1e-8), BFOM and BGMRES with
the BCGSI+LS, BMGS-CWY and BMGS-ICWY skeletons and CholQR.

Calls only the oracle and the seeded input builder.  Stored per solve:
status, iteration count, cycle lengths, m after each cycle (restart points),
the paper's counters, the residual estimate at the end of every cycle and at
every column of the first and last cycles, ||X||_F, and the rows of X at a
fixed stride (for a sampled X comparison).  Takes tens of minutes (the six
solves run in parallel processes):

    python tests/golden/make_laplace2d_golden.py
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SOLVES = [(m, k) for k in ("bcgsi_ls", "bmgs_cwy", "bmgs_icwy") for m in ("fom", "gmres")]
ROW_STRIDE = 1024


def one(arg):
    method, skel = arg
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    import numpy as np

    import oracle
    from paper_2208_09899_amd import workloads as w
    wl = w.workload("laplace2d")
    r = oracle.solve(wl.A.to_scipy(), wl.B, method, skel, "cholqr", m=wl.m, tol=wl.tol,
                     max_cycles=wl.max_cycles)
    h = r.res_hist
    ends, pos = [], 0
    for c in r.cycle_len:
        pos += c
        ends.append(h[pos - 1])
    first, last = r.cycle_len[0], r.cycle_len[-1]
    rows = list(range(0, wl.A.n, ROW_STRIDE))
    return {
        "method": method, "skeleton": skel, "status": r.status, "iters": r.iters,
        "cycle_len": list(r.cycle_len), "m_after": list(r.m_after), "counts": list(r.counts),
        "res_cycle_end": [float(x) for x in ends],
        "res_first_cycle": [float(x) for x in h[:first]],
        "res_last_cycle": [float(x) for x in h[len(h) - last:]],
        "x_norm": float(np.linalg.norm(r.X)),
        "x_rows": rows,
        "x_sampled": [[float(v) for v in r.X[i]] for i in rows],
    }


def main():
    with ProcessPoolExecutor(max_workers=len(SOLVES)) as ex:
        out = list(ex.map(one, SOLVES))
    rec = {"workload": "2-D 5-point Laplacian 256x256, s=8 (seed 2), m=30, tol 1e-8, CholQR",
           "generator": "tests/golden/make_laplace2d_golden.py (oracle only)",
           "solves": out}
    with open(os.path.join(HERE, "laplace2d_256_s8_m30.json"), "w") as f:
        json.dump(rec, f, indent=0)
    for o in out:
        print(o["method"], o["skeleton"], o["status"], o["iters"], len(o["cycle_len"]))


if __name__ == "__main__":
    main()
