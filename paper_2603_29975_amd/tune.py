"""Tuning driver: runs ozaki_autotune over a list of shapes on the current GPU
and writes the tuning table as JSON (the format ozaki_tune_load reads).

    python -m paper_2603_29975_amd.tune --out tune_cache.json \
        --shape z:2048:2048:2048:7 --shape z:4096:4096:4096:7

Without --shape it tunes the default set below: square complex and real
products from 256 to 8192 at the slice counts 4..10 that reach FP64-level
accuracy on well-scaled data, plus the tall-skinny shapes of a blocked LU
update. Each entry covers a whole size bucket (ceil log2 of m, n' and the
32-deep contraction blocks), so a table of a few dozen shapes covers most
calls. Load it with OZAKI_TUNE_CACHE=<file> or ozaki_tune_load(<file>).
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_SLICES = (4, 5, 6, 7, 8, 9, 10)


def default_shapes():
    shapes = []
    for kind in ("z", "d"):
        for n in (256, 512, 1024, 2048, 4096, 8192):
            for s in DEFAULT_SLICES:
                if kind == "z" and n == 8192 and s > 7:
                    continue
                shapes.append((kind, n, n, n, s))
        for s in (6, 7, 8):
            shapes.append((kind, 8192, 256, 8192, s))
            shapes.append((kind, 256, 8192, 8192, s))
    return shapes


def parse_shape(text: str):
    kind, m, n, k, s = text.split(":")
    return kind, int(m), int(n), int(k), int(s)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--shape", action="append", type=parse_shape,
                    help="kind:m:n:k:slices (repeatable); default: the built-in set")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--merge", action="store_true", help="start from the entries already in --out")
    args = ap.parse_args(argv)

    import torch
    import paper_2603_29975_amd as oz
    if not torch.cuda.is_available():
        raise SystemExit("tune.py needs a GPU")
    torch.cuda.init()
    oz.library()
    oz.ozaki_tune_clear()
    if args.merge and os.path.exists(args.out):
        rc = oz.ozaki_tune_load(args.out)
        if rc != 0:
            raise SystemExit(f"ozaki_tune_load({args.out}): {oz.ozaki_status_string(rc)}")
    for kind, m, n, k, s in (args.shape or default_shapes()):
        rc, best, ms = oz.ozaki_autotune(kind, m, n, k, s, reps=args.reps)
        if rc != 0:
            raise SystemExit(f"ozaki_autotune {kind} {m}x{n}x{k} s={s}: {oz.ozaki_status_string(rc)}")
        print(f"{kind} {m}x{n}x{k} s={s}: id {best}  {ms:.4f} ms", flush=True)
    rc = oz.ozaki_tune_save(args.out)
    if rc != 0:
        raise SystemExit(f"ozaki_tune_save({args.out}): {oz.ozaki_status_string(rc)}")
    print("wrote", args.out)


if __name__ == "__main__":
    main()
