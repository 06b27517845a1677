"""HBM traffic per launch from rocprofv3 counter runs.

Reads two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of

    python bench.py --steps 1 --warmup 0 --iters 10 --no-cpu-baseline \\
        --latency-reps 1 --copy-calibration-mb 1024

(``--output-format csv``), scales each counter by what it reads for the plain
device-to-device copy of known size that ``--copy-calibration-mb`` runs
first, and prints one line per kernel kind of the benchmark:

    traffic <kind> <fetch KiB per launch> <write KiB per launch> \\
        <fetch scale> <write scale> <kernel-source digest>

A "launch" is what bench.py times for that kind: one iteration kernel over
the whole batch, or the whole batched adjoint / forward contraction (all
its dispatches).  The digest is bench.csrc_digest() of the sources the run
was built from; bench.py reports the traffic only while it still matches.

Usage: python -m paper_0908_3252_amd.pmc_summary FETCH.csv WRITE.csv \\
           --batch 128 --copy-mib 1024 [--digest HEX]
"""
from __future__ import annotations

import argparse
import csv
import collections
import sys


def _per_dispatch(path: str, counter: str):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        out.append((r["Kernel_Name"], int(r["Grid_Size"]), int(r["Workgroup_Size"]),
                    float(r["Counter_Value"])))
    return out


def _calibration(disp, copy_bytes: float) -> float:
    """counter KiB of the largest plain copy dispatch -> scale to true bytes."""
    copies = [v for (k, g, w, v) in disp if "copyBuffer" in k]
    if not copies:
        raise SystemExit("no copy kernel in the counter run (use --copy-calibration-mb)")
    return copy_bytes / 1024.0 / max(copies)


def _kind_of(name: str):
    if "k_adjoint_" in name or "k_split_reduce" in name:
        return "adjoint"
    if "k_forward_" in name:
        return "forward"
    if "k_colpass_f64<" in name:  # the FP64 column pass (L = 512, 1024)
        return "colpass"
    for k in ("k_dir_rowfft", "k_colpass", "k_update"):
        if k + "<" in name or k + "(" in name:
            return k[2:]
    return None


def summarize(fetch_csv: str, write_csv: str, batch: int, copy_mib: int, group: int = 1):
    res = {}
    for which, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"),
                                 ("write", write_csv, "WRITE_SIZE")):
        disp = _per_dispatch(path, counter)
        scale = _calibration(disp, copy_mib * 1048576.0)
        groups = collections.defaultdict(list)
        for (name, grid, wg, v) in disp:
            kind = _kind_of(name)
            if kind:
                groups[(kind, name, grid // wg)].append(v)
        per_kind = collections.defaultdict(float)
        for kind in ("dir_rowfft", "colpass", "update", "forward"):
            # the batched launch is the one with the most workgroups
            cand = [(blocks, vals) for (k, n, blocks), vals in groups.items() if k == kind]
            if cand:
                blocks, vals = max(cand)
                per_kind[kind] = sum(vals) / len(vals)
        # adjoint: the batched contraction runs batch / group dispatches of the
        # split-K contraction, each followed by its split reduction
        contr = [vals for (k, n, blocks), vals in groups.items()
                 if k == "adjoint" and "k_adjoint_" in n]
        red = [vals for (k, n, blocks), vals in groups.items()
               if k == "adjoint" and "k_split_reduce" in n]
        if contr:
            c = [v for vals in contr for v in vals]
            r = [v for vals in red for v in vals]
            per = sum(c) / len(c) + (sum(r) / len(r) if r else 0.0)
            per_kind["adjoint"] = per * batch / group
        res[which] = (dict(per_kind), scale)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--group", type=int, default=1,
                    help="frames per adjoint dispatch (1 at the benchmark workloads)")
    ap.add_argument("--digest", default=None)
    args = ap.parse_args(argv)
    digest = args.digest
    if digest is None:
        import os
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        digest = bench.csrc_digest()
    res = summarize(args.fetch_csv, args.write_csv, args.batch, args.copy_mib, args.group)
    fk, fs = res["fetch"]
    wk, ws = res["write"]
    for kind in ("adjoint", "forward", "dir_rowfft", "colpass", "update"):
        if kind in fk and kind in wk:
            print(f"traffic {kind} {fk[kind]:.1f} {wk[kind]:.1f} {fs:.4f} {ws:.4f} {digest}")


if __name__ == "__main__":
    main()
