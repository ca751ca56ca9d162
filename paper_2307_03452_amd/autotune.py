"""Autotuner for plan tiles: for each class (la lb|lc ld) and contraction-size
bucket, time every tile choice (16 or 32 bra rows x R layout box / two boxes /
slab) that fits, on a seeded synthetic batch of that class, and keep the
fastest.  Writes the tile table the library reads (tune_<arch>.txt, for
eri4_plan_create_tunefile / eri4.Plan(tune_file=...)) and a JSON record of
every timing (tune_<arch>.json, whose "entries" eri4.Plan(tiles=...) also
accepts).  Both are keyed by the device's architecture name (gcnArchName up to
its first ':').

  python -m paper_2307_03452_amd.autotune [--lvals 4,5,6,7] [--only-with 7] [--buckets 0,1,2]
                                          [--merge] [--reps 2]

The buckets are ranges of K_a K_b K_c K_d (primitive quartets per quartet);
each is timed at one contraction length per shell inside it.  --only-with l
tunes only the classes with a shell of angular momentum l; --merge keeps the
entries of the existing table for the classes and buckets not tuned now.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))

# (kq_min, kq_max, K per shell used to time it)
BUCKETS = [(1, 1, 1), (2, 40, 2), (41, 400, 3), (401, 4096, 5)]
# timed batches hold at least this many of the largest (64-row) tiles, two per
# compute unit, so that the timing reflects the cost of a tile, not an idle GPU
MIN_TILES = 512
TILE_ROWS = 64
CANDIDATES = [(4, "box2"), (2, "box2"), (1, "box2"), (4, "box"), (2, "box"), (1, "box"), (2, "slab"), (1, "slab")]


def _time(plan, args, reps):
    import torch
    out = plan.execute(*args)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        plan.execute(*args, out=out)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def tune(classes, reps=2, log=print, buckets=BUCKETS):
    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2307_03452_amd import eri4, inputs
    eri4.init()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    entries, timings = [], []
    for ci, ls in enumerate(classes):
        nab = ((ls[0] + 1) * (ls[0] + 2) // 2) * ((ls[1] + 1) * (ls[1] + 2) // 2)
        nq = -(-MIN_TILES // -(-nab // TILE_ROWS))
        for kq_min, kq_max, k in buckets:
            b = inputs.class_batch(ls, nq, k, seed=7000 + 17 * ci + k, exp_range=(0.05, 200.0))
            lq = np.tile(np.array(ls, np.int32), (nq, 1))
            args = (d(b.centers), d(b.exps), d(b.coefs))
            default = _time(eri4.Plan(lq, b.nprim, b.kmax), args, reps)
            best = None
            res = {}
            for rows16, lay in CANDIDATES:
                tile = {"l": list(ls), "kq": [kq_min, kq_max], "rows16": rows16, "layout": lay}
                try:
                    plan = eri4.Plan(lq, b.nprim, b.kmax, tiles=[tile])
                except eri4.Eri4Error:
                    continue  # does not fit
                ms = _time(plan, args, reps)
                res[f"{rows16}x16/{lay}"] = ms
                if best is None or ms < best[0]:
                    best = (ms, tile)
            entries.append(best[1])
            timings.append({"class": list(ls), "kq": [kq_min, kq_max], "K_per_shell": k, "quartets": nq,
                            "default_ms": default, "best_ms": best[0], "candidates_ms": res})
            log(f"({ls[0]}{ls[1]}|{ls[2]}{ls[3]}) K={k}: default {default:.3f} ms, best {best[0]:.3f} ms "
                f"({best[1]['rows16']}x16/{best[1]['layout']})")
    return entries, timings


def arch_name() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def write_table(path, arch, entries):
    lines = ["# eri4 tile table (autotune.py): la lb lc ld kq_min kq_max rows16 layout", f"arch {arch}"]
    for e in entries:
        lines.append(" ".join(str(x) for x in (*e["l"], *e["kq"], e["rows16"], e["layout"])))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lvals", default="4,5,6")
    ap.add_argument("--only-with", type=int, default=None)
    ap.add_argument("--buckets", default=",".join(str(i) for i in range(len(BUCKETS))))
    ap.add_argument("--merge", action="store_true")
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args()
    lvals = [int(x) for x in a.lvals.split(",")]
    buckets = [BUCKETS[int(i)] for i in a.buckets.split(",")]
    classes = sorted(itertools.product(lvals, repeat=4), key=lambda t: (sum(t), t))
    if a.only_with is not None:
        classes = [c for c in classes if a.only_with in c]
    arch = arch_name()
    jpath, tpath = os.path.join(HERE, f"tune_{arch}.json"), os.path.join(HERE, f"tune_{arch}.txt")
    t0 = time.time()
    entries, timings = tune(classes, a.reps, log=lambda m: print(m, flush=True), buckets=buckets)
    if a.merge and os.path.exists(jpath):
        with open(jpath) as f:
            old = json.load(f)
        done = {(tuple(e["l"]), tuple(e["kq"])) for e in entries}
        entries = [e for e in old["entries"] if (tuple(e["l"]), tuple(e["kq"])) not in done] + entries
        timings = [t for t in old["timings"] if (tuple(t["class"]), tuple(t["kq"])) not in done] + timings
        lvals = sorted(set(old.get("lvals", [])) | set(lvals))
    entries.sort(key=lambda e: (sum(e["l"]), e["l"], e["kq"]))
    doc = {"arch": arch, "lvals": lvals, "buckets": BUCKETS, "seconds": time.time() - t0, "entries": entries,
           "timings": timings}
    with open(jpath, "w") as f:
        json.dump(doc, f, indent=1)
    write_table(tpath, arch, entries)
    print(jpath, tpath)


if __name__ == "__main__":
    main()
