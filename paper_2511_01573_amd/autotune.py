"""Autotuner for the batched rule kernel's tile shape.

For every (d, family) group of a batch workload it times the batched
integration of a representative sub-batch of that group under each candidate
tile (lanes per region x workgroups launched) and keeps the fastest.  The
table is written as JSON and applied with `apply()` (gm_set_tile).

Usage (on a GPU):  python -m paper_2511_01573_amd.autotune [--out tile_table.json]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import gm, workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tile_table.json")


def candidates(d: int):
    lanes = [1]
    lanes += [L for L, dmin in ((4, 6), (16, 8), (64, 10)) if d >= dmin]
    grids = [512, 1024, 2048, 4096]
    return [(L, g) for L in lanes for g in grids]


def group_batches(batch):
    groups = {}
    for i, (fam, d) in enumerate(zip(batch["families"], batch["ds"])):
        groups.setdefault((d, fam), []).append(i)
    return groups


def sub_batch(batch, idx):
    return ([batch["families"][i] for i in idx], [batch["params"][i] for i in idx],
            [batch["ds"][i] for i in idx], [batch["los"][i] for i in idx],
            [batch["his"][i] for i in idx], [batch["rel_tols"][i] for i in idx],
            [batch["abs_tols"][i] for i in idx])


def time_batch(args, cap, reps=2):
    best = np.inf
    for _ in range(reps):
        t0 = time.perf_counter()
        gm.integrate_batch(*args, cap)
        best = min(best, time.perf_counter() - t0)
    return best


def tune(batch=None, per_group=128, cap=1 << 27, verbose=True):
    batch = batch or W.config4()
    table = {}
    for (d, fam), idx in sorted(group_batches(batch).items()):
        args = sub_batch(batch, idx[:per_group])
        results = []
        for lanes, grid in candidates(d):
            gm.set_tile(d, fam, lanes, grid)
            results.append((time_batch(args, cap), lanes, grid))
        gm.set_tile(d, fam, 0, 0)
        t, lanes, grid = min(results)
        table[f"{d},{fam}"] = {"d": d, "family": fam, "lanes_per_region": lanes,
                               "grid_blocks": grid, "seconds": t,
                               "tried": [{"lanes": L, "grid": g, "seconds": s}
                                         for s, L, g in results]}
        if verbose:
            print(f"d={d} fam={fam}: lanes={lanes} grid={grid} {t * 1e3:.2f} ms", flush=True)
    return table


def apply(table) -> None:
    for v in table.values():
        gm.set_tile(v["d"], v["family"], v["lanes_per_region"], v["grid_blocks"])


def load(path: str = DEFAULT_TABLE):
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    apply(table)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--per-group", type=int, default=128)
    args = ap.parse_args()
    table = tune(per_group=args.per_group)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
