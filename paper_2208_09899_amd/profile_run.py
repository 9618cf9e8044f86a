"""Short runs for hardware-counter profiling (rocprofv3 --pmc).

Counter collection serialises every dispatch, so the full benchmark (hundreds
of thousands of launches) is too long to profile this way.  This driver runs
the same workload and launch configuration for a capped number of block
iterations, and a plain device copy of known size whose FETCH_SIZE /
WRITE_SIZE readings calibrate the byte counters:

    rocprofv3 --pmc FETCH_SIZE -- python3 paper_2208_09899_amd/profile_run.py \
        --workload laplace2d --max-iters 120
    rocprofv3 --pmc FETCH_SIZE -- python3 paper_2208_09899_amd/profile_run.py --copy

It prints the algorithmic bytes per launch of each kernel class (from HIP
events on an identical second run) so that the counter totals can be set
beside them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

if __package__ in (None, ""):
    # run by path (e.g. under rocprofv3 from another directory)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


# kernel class: (kernel-name substrings, source file)
KERNEL_CLASSES = {"update": (("update_kernel", "update_mfma"), "kernels_update.hip"),
                  "gram": (("gram_stage1", "gram_mfma"), "kernels_gram.hip"),
                  "spmm": (("spmm_kernel", "spmm_coop_kernel"), "kernels_sparse.hip"),
                  "precond": (("ilu_sweep_kernel",), "kernels_ilu.hip")}


def _counter_means(path, counter):
    """Mean counter value (KiB) per dispatch, by kernel-name substring."""
    import csv
    sums = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        sums.setdefault(name, []).append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in sums.items()}


def summarize(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, alg_json, workload, out):
    """Scale the per-dispatch FETCH_SIZE / WRITE_SIZE of each kernel class by
    the readings of a plain copy of known size and write the HBM bytes per
    launch, beside the algorithmic bytes per launch of an identical run."""
    import hashlib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    copy_bytes = (1 << 26) * 8
    cf = _counter_means(copy_fetch_csv, "FETCH_SIZE")
    cw = _counter_means(copy_write_csv, "WRITE_SIZE")
    pick = lambda d: max((v for k, v in d.items() if "copy" in k.lower() or "elementwise" in k),
                         key=lambda t: t[0])[0]
    fscale = copy_bytes / (pick(cf) * 1024.0)
    wscale = copy_bytes / (pick(cw) * 1024.0)
    fe = _counter_means(fetch_csv, "FETCH_SIZE")
    wr = _counter_means(write_csv, "WRITE_SIZE")
    alg = json.load(open(alg_json))["kernel_stats"]
    rec = {"workload": workload, "fetch_scale": fscale, "write_scale": wscale,
           "copy_bytes": copy_bytes, "kernels": {}}
    for cls, (sub, src) in KERNEL_CLASSES.items():
        fk = [v for k, v in fe.items() if any(x in k for x in sub)]
        wk = [v for k, v in wr.items() if any(x in k for x in sub)]
        if not fk or not wk or not alg.get(cls, {}).get("launches"):
            continue
        n = sum(c for _, c in fk)
        f = sum(m * c for m, c in fk) / n
        wn = sum(c for _, c in wk)
        wv = sum(m * c for m, c in wk) / wn
        hbm = f * 1024.0 * fscale + wv * 1024.0 * wscale
        a = alg[cls]["alg_bytes"] / alg[cls]["launches"]
        sha = hashlib.sha256(open(os.path.join(root, "paper_2208_09899_amd", "csrc", src),
                                  "rb").read()).hexdigest()
        rec["kernels"][cls] = {"launches": n, "fetch_kib_per_launch": f,
                               "write_kib_per_launch": wv, "hbm_bytes_per_launch": hbm,
                               "alg_bytes_per_launch": a, "traffic_over_alg": hbm / a,
                               "source_sha256": sha}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="laplace2d")
    ap.add_argument("--method", default="gmres")
    ap.add_argument("--skeleton", default="bcgsi_ls")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--max-iters", type=int, default=120)
    ap.add_argument("--precond", choices=["none", "ilu0"], default="none",
                    help="right ILU(0) preconditioning (factorization before the solve)")
    ap.add_argument("--copy", action="store_true",
                    help="run only a device-to-device copy of 512 MiB, 5 times")
    ap.add_argument("--stats", action="store_true",
                    help="record HIP-event statistics per kernel class and print them")
    ap.add_argument("--summarize", nargs=5, metavar=("FETCH", "WRITE", "COPY_FETCH",
                                                     "COPY_WRITE", "ALG_JSON"),
                    help="write the calibrated traffic record (--out) from the counter "
                         "CSVs of the four runs and the --stats output of a fifth")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.summarize:
        rec = summarize(*args.summarize, workload=args.workload, out=args.out)
        print(json.dumps(rec, indent=1))
        return

    import torch

    if args.copy:
        x = torch.ones(1 << 26, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8,
                          "launches": 5}))
        return

    from paper_2208_09899_amd import lsba, workloads as w

    wl = w.workload(args.workload)
    dev = torch.device("cuda:0")
    B = torch.from_numpy(wl.B).to(dev)
    X = torch.empty_like(B)
    ctx = lsba.Context(0, stream="torch")
    op = lsba.Operator(ctx, wl.A)
    pc = lsba.Precond(ctx, op) if args.precond == "ilu0" else None
    if args.stats:
        ctx.set_timing(True)
    r = lsba.solve(ctx, op, B, X=X, method=args.method, skeleton=args.skeleton,
                   precision=args.precision, m=wl.m, tol=wl.tol, max_cycles=wl.max_cycles,
                   max_iters=args.max_iters, precond=pc)
    torch.cuda.synchronize()
    out = {"workload": args.workload, "iters": r.iters, "status": r.status}
    if args.stats:
        out["kernel_stats"] = {k: {"launches": v[0], "ms": v[1], "alg_bytes": v[2]}
                               for k, v in ctx.kernel_stats().items()}
    print(json.dumps(out))
    if pc is not None:
        pc.close()
    op.close()
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
