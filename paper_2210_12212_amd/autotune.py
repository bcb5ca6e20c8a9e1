"""Offline tuner of the A^T A product tilings (run on the GPU it tunes for).

For one matrix shape (n x d, FP32 or FP64) and one product arithmetic (FP64
or FP32 matrix cores) it times W = A^T A U through ``ihsbin_ata_apply_tiled``
for every width class nb = ceil(w / 16) asked for, over every column-tile
width q in 1..7 (c = ceil(nb / q) tiles of 16 q columns) and split-K counts
around the cost model's choice, and records the fastest (median of a few
calls after a warm-up).  The results are merged into
``csrc/tuned_tiles.inc`` (entries of other shapes are kept), which the library
consults before its cost model; rebuild the library afterwards.

    python -m paper_2210_12212_amd.autotune --n 131072 --d 2048 --dtype f32 \\
        --prec f64 --nb 1-16 --write
"""
from __future__ import annotations

import argparse
import os
import re
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "tuned_tiles.inc")

HEADER = """// Column tilings and split-K counts of the A^T A products measured best by
// paper_2210_12212_amd/autotune.py on MI355X, per matrix shape, arithmetic
// and width class (nb = ceil(w / 16)).  Regenerate with that script; the
// products fall back to pick_col_tiles / pick_splits_cols for any shape or
// width not listed.
// {n, d, A dtype (0 FP32, 1 FP64), product (0 FP64, 1 FP32), nb, q, splits}
"""


def read_table(path=TABLE):
    """Entries (n, d, dtype, prec, nb, q, splits) of the current table."""
    rows = []
    if not os.path.exists(path):
        return rows
    for m in re.finditer(r"\{\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+)\s*\}",
                         open(path).read()):
        row = tuple(int(x) for x in m.groups())
        if row[4] > 0:
            rows.append(row)
    return rows


def write_table(rows, path=TABLE):
    rows = sorted(set(rows))
    body = "".join("    {%d, %d, %d, %d, %d, %d, %d},\n" % r for r in rows) or \
        "    {0, 0, 0, 0, 0, 0, 0},\n"
    with open(path, "w") as f:
        f.write(HEADER)
        f.write("static const TunedTile kTunedTiles[] = {\n" + body + "};\n")
        f.write("static const int kNumTunedTiles = %d;\n" % len(rows))


def merge(old, new):
    """new entries replace old ones with the same (n, d, dtype, prec, nb)."""
    keyed = {r[:5]: r for r in old}
    for r in new:
        keyed[r[:5]] = r
    return list(keyed.values())


def parse_range(spec):
    out = []
    for part in spec.split(","):
        if "-" in part:
            a, b = part.split("-")
            out += list(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def tune(n, d, dtype, prec, nbs, reps=3, split_choices=(1, 2, 4, 8, 16, 32, 64)):
    import torch
    from paper_2210_12212_amd import Context

    dev = torch.device("cuda", 0)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    g = torch.Generator(device=dev).manual_seed(1234)
    A = torch.randn((n, d), generator=g, device=dev, dtype=tdt)
    ctx = Context(0)
    rows = []
    for nb in nbs:
        w = 16 * nb
        U = torch.randn((d, w), generator=g, device=dev, dtype=torch.float64)
        best = None
        for q in range(1, 8):
            c = -(-nb // q)
            if q > nb and q > 1:
                break
            for sp in (0,) + tuple(split_choices):
                ctx.ata_apply_tiled(A, U, prec, q, sp)
                torch.cuda.synchronize()
                ts = []
                for _ in range(reps):
                    t = time.perf_counter()
                    ctx.ata_apply_tiled(A, U, prec, q, sp)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t)
                ms = sorted(ts)[len(ts) // 2] * 1e3
                if best is None or ms < best[0]:
                    best = (ms, q, sp, c)
        base_t = []
        for _ in range(reps):
            t = time.perf_counter()
            ctx.ata_apply_tiled(A, U, prec, 0, 0)
            torch.cuda.synchronize()
            base_t.append(time.perf_counter() - t)
        base = sorted(base_t)[len(base_t) // 2] * 1e3
        ms, q, sp, c = best
        print(f"nb {nb:3d} (w {w}): best q={q} c={c} splits={sp or 'model'} {ms:.3f} ms "
              f"({4.0 * n * d * w / ms / 1e9:.1f} TFLOP/s); library choice {base:.3f} ms",
              flush=True)
        rows.append((n, d, 0 if dtype == "f32" else 1, 0 if prec == "f64" else 1, nb, q, sp))
    ctx.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--d", type=int, required=True)
    ap.add_argument("--dtype", choices=("f32", "f64"), default="f32")
    ap.add_argument("--prec", choices=("f64", "f32"), default="f64")
    ap.add_argument("--nb", default="1-16", help="width classes, e.g. 1-16 or 2,4,8")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--write", action="store_true", help="merge the results into the table")
    ap.add_argument("--table", default=TABLE)
    args = ap.parse_args(argv)
    rows = tune(args.n, args.d, args.dtype, args.prec, parse_range(args.nb), args.reps)
    if args.write:
        write_table(merge(read_table(args.table), rows), args.table)
        print(f"wrote {len(rows)} entries into {args.table}")
    return 0


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    sys.exit(main())
