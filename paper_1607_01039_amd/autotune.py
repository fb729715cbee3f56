"""Autotuner for the pass schedule of fwht_int / fwht_float on the local GPU.

For each (dtype, n) it times every schedule with the minimum number of HBM
passes: a contiguous pass of c bits followed by strided passes whose bit
counts and row-segment widths (2^cb entries) vary, each strided pass using the
variant whose tile height equals its bit count.  The fastest schedule per
(dtype, n) is written to tune/gfx950.txt, which libfwht.so reads at start-up.
With --batched it times the tile groupings of the batched FP32 transform
instead and writes the fastest as the table's "batched fp32" line.

    python -m paper_1607_01039_amd.autotune --dtype int32 --n 16-30
    python -m paper_1607_01039_amd.autotune --batched
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, "tune", "gfx950.txt")

# Compiled variants (must match csrc/fwht_variants_*.hip).
CONTIG = {"int32": (12, 13, 14, 15, 16), "float32": (12, 13, 14, 15, 16), "int64": (11, 12, 13, 14)}
SEGMENT_BITS = {"int32": (5, 6, 7, 8, 9), "float32": (5, 6, 7, 8, 9), "int64": (4, 5, 6, 7)}
# 256 KiB strided variants held in registers (2^16 4-byte or 2^15 8-byte
# entries): column bits -> their (only) bit count
PINNED = {"int32": {7: 9, 8: 8, 9: 7}, "float32": {7: 9, 8: 8, 9: 7}, "int64": {6: 9, 7: 8}}
MAX_TILE_BYTES = 128 * 1024
RMAX = 9
# strided variants from this tile size up (and C16) also exist as twins with
# non-temporal loads and stores, named with a trailing "n"
NT_MIN_TB = {"int32": 13, "float32": 13, "int64": 12}


# first passes held in registers, which must be followed by strided passes:
# 256 KiB tiles in 1024 threads, 128 KiB tiles in 512 threads (two
# workgroups per CU), each with a non-temporal twin
WHOLE_FIRST = {"int32": {16: ("C16", "C16n"), 15: ("C15p", "C15pn")},
               "float32": {16: ("C16", "C16n"), 15: ("C15p", "C15pn")},
               "int64": {14: ("C14p", "C14pn")}}
# strided variants held in registers by 512 threads, two workgroups per CU:
# (column bits, row bits) -> name
HELD = {"int64": {(6, 8): "S14c6p"},
        "int32": {(7, 8): "S15c7p", (8, 7): "S15c8p"},
        "float32": {(7, 8): "S15c7p", (8, 7): "S15c8p"}}
# 8-byte strided tiles of 2^14 entries also held by 1024 threads (16 entries
# each instead of 32): (column bits, row bits) -> name
WIDE = {"int64": {(5, 9): "S14c5w", (6, 8): "S14c6w", (7, 7): "S14c7w"}}


# row-segment widths compiled for the tile variants of up to 2^15 entries
TILE_SEGMENT_BITS = {"int32": (5, 6, 7, 8), "float32": (5, 6, 7, 8), "int64": (4, 5, 6, 7)}


def strided_variants(dtype: str, r: int, cb: int):
    """Names of the strided variants that transform r bits over 2^cb columns."""
    esz = 8 if dtype == "int64" else 4
    tb = cb + r
    if (1 << tb) * esz == 256 * 1024:
        return [f"S{tb}c{cb}"] if PINNED[dtype].get(cb) == r else []
    if cb not in TILE_SEGMENT_BITS[dtype]:
        return []
    if (1 << tb) * esz > MAX_TILE_BYTES:
        return []
    vec = 16 // esz
    nt = (1 << tb) // 32 if tb >= 14 else max(64, (1 << tb) // 16)
    if (1 << tb) // nt < vec:
        return []
    out = [f"S{tb}c{cb}"]
    for extra in (HELD, WIDE):
        if (cb, r) in extra.get(dtype, {}):
            out.append(extra[dtype][(cb, r)])
    return out


def _tile_bits(name: str) -> int:
    """Tile bits of a strided variant name such as "S15c8" or "S15c7p"."""
    return int(name[1:].split("c")[0])


def compositions(s: int, k: int, lo: int = 1, hi: int = RMAX):
    if k == 1:
        if lo <= s <= hi:
            yield (s,)
        return
    for first in range(lo, hi + 1):
        for rest in compositions(s - first, k - 1, lo, hi):
            yield (first,) + rest


def first_passes(dtype: str, n: int):
    """Contiguous first passes for n bits: C16 only with strided passes after it."""
    return [c for c in CONTIG[dtype] if c <= n and (c < 16 or n > c)]


def candidates(dtype: str, n: int, max_cands: int = 1000):
    single = max(c for c in CONTIG[dtype] if c < 16)
    if n <= single:
        return [f"C{max(min(CONTIG[dtype]), n)}"]
    best_p = min(1 + -(-(n - c) // RMAX) for c in first_passes(dtype, n))
    out = []
    for c in first_passes(dtype, n):
        s = n - c
        ns = best_p - 1
        if ns < 1 or s > ns * RMAX or s < ns:
            continue
        # a 2^15-entry first pass also comes held in registers
        firsts = (f"C{c}",)
        if c in WHOLE_FIRST[dtype]:
            firsts = WHOLE_FIRST[dtype][c] if c == 16 else firsts + WHOLE_FIRST[dtype][c]
        for comp in compositions(s, ns, 2 if s >= 2 * ns else 1):
            if max(comp) - min(comp) > 2:
                continue
            strided = itertools.chain.from_iterable(
                itertools.product(*[strided_variants(dtype, r, cb) for r, cb in zip(comp, cbs)])
                for cbs in itertools.product(SEGMENT_BITS[dtype], repeat=ns))
            # cache policy of the first pass and of the strided passes, chosen
            # independently
            for parts, first, nt in itertools.product(list(strided), firsts, (False, True)):
                names = [v + "n" if nt and _tile_bits(v) >= NT_MIN_TB[dtype] else v for v in parts]
                spec = ",".join([first] + [f"{v}:{r}" for v, r in zip(names, comp)])
                if spec not in out:
                    out.append(spec)
    return out[:max_cands]


def time_schedule(F, torch, buf, dtype, n, spec, reps=5, src=None):
    """Median device time of one transform under `spec`.  With `src`, the
    input is restored from it (untimed) before every run, so each run starts
    from freshly written data as a real call does (cache state matters: a pass
    with non-temporal loads is slower on data that was just written)."""
    F.set_schedule(dtype, n, spec)
    run = (lambda: F.fwht_float_(buf)) if dtype == "float32" else (lambda: F.fwht_int_(buf))
    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        if src is not None:
            buf.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(dtype: str, ns, min_total_bits: int = 0, log=print):
    import torch

    import paper_1607_01039_amd as F
    tdt = {"int32": torch.int32, "int64": torch.int64, "float32": torch.float32}[dtype]
    results = {}
    for n in ns:
        total_bits = max(n, min_total_bits) if dtype == "float32" else n
        if dtype == "float32":
            buf = torch.randn((1 << (total_bits - n), 1 << n), device="cuda", dtype=tdt)
        else:
            buf = torch.randint(-1, 2, (1 << n,), device="cuda", dtype=tdt)
        src = buf.clone()
        F.set_schedule(dtype, n, None)
        default = F.get_schedule(dtype, n)
        cands = candidates(dtype, n)
        if default not in cands:
            cands.append(default)
        best = None
        t0 = time.time()
        for spec in cands:
            try:
                ms = time_schedule(F, torch, buf, dtype, n, spec, src=src)
            except F.FWHTError:
                continue  # refused by the library (e.g. a pass whose lane offsets would not fit 32 bits)
            if best is None or ms < best[1]:
                best = (spec, ms)
        F.set_schedule(dtype, n, None)
        ms_def = time_schedule(F, torch, buf, dtype, n, default, src=src) if len(cands) > 1 else best[1]
        F.set_schedule(dtype, n, None)
        results[n] = best
        log(f"[tune] {dtype} n={n} total=2^{total_bits}: {len(cands)} schedules in {time.time() - t0:.1f}s; "
            f"best {best[0]} {best[1]:.4f} ms (default {default} {ms_def:.4f} ms)")
        del buf, src
        torch.cuda.empty_cache()
    return results


# Tile groupings of the batched FP32 transform (see fwht_set_batched_tiles).
BATCHED_TILES = ["16:2-16", "16:16,15:2-15", "16:16,15:15,14:2-14", "16:15-16,14:2-14", "16:16,15:14-15,14:2-13"]


def tune_batched(log=print, reps=30):
    """Time every tile grouping of the batched FP32 transform on 4096
    transforms of sizes 2^8..2^16 (N(0,1), seed 4), as the mean of the warm
    median (input just transformed) and the cold median (1 GiB written in
    between), and return the fastest as (spec, ms)."""
    import torch

    import paper_1607_01039_amd as F
    import synth
    lg, off, tot = synth.ragged(4096, 8, 16, 4)
    x = torch.from_numpy(synth.normal(tot, 4)).cuda()
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    best = None
    for spec in BATCHED_TILES:
        F.set_batched_tiles("fp32", spec)
        F.fwht_batched_(x, off, lg)
        torch.cuda.synchronize()
        med = []
        for cold in (False, True):
            ts = []
            for _ in range(reps):
                if cold:
                    flush.add_(1.0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                F.fwht_batched_(x, off, lg)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            med.append(float(np.median(ts)))
        ms = (med[0] + med[1]) / 2
        log(f"[tune] batched fp32 {spec}: warm {med[0]:.4f} ms, cold {med[1]:.4f} ms")
        if best is None or ms < best[1]:
            best = (spec, ms)
    F.set_batched_tiles("fp32", None)
    log(f"[tune] batched fp32 best {best[0]} {best[1]:.4f} ms")
    return best


def write_table(path: str, updates: dict):
    """Merge {(dtype, n): (spec, ms)} into the table file."""
    rows = {}
    if os.path.exists(path):
        for line in open(path):
            line = line.split("#")[0].split()
            if len(line) >= 3:
                key = (line[0], line[1] if line[0] == "batched" else int(line[1]))
                rows[key] = (line[2], float(line[3]) if len(line) > 3 else float("nan"))
    rows.update(updates)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("# dtype n schedule ms  -- written by paper_1607_01039_amd/autotune.py on MI355X (gfx950)\n")
        for (dt, n) in sorted(rows, key=lambda k: (k[0], str(k[1]).zfill(8))):
            spec, ms = rows[(dt, n)]
            f.write(f"{dt} {n} {spec} {ms:.4f}\n")


def parse_range(s: str):
    out = []
    for part in s.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", default="int32", choices=["int32", "int64", "float32"])
    ap.add_argument("--n", default="16-30")
    ap.add_argument("--float-total-bits", type=int, default=28,
                    help="float32: batch so that batch * 2^n = 2^this (the transform size stays 2^n)")
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--batched", action="store_true", help="tune the tile groups of the batched FP32 transform")
    args = ap.parse_args()
    if args.batched:
        write_table(args.out, {("batched", "fp32"): tune_batched(log=lambda m: print(m, flush=True))})
        print(f"wrote {args.out}", flush=True)
        return
    res = tune(args.dtype, parse_range(args.n), args.float_total_bits,
               log=lambda m: print(m, flush=True))
    write_table(args.out, {(args.dtype, n): v for n, v in res.items()})
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(PKG))
    main()
