"""Sweep the launch-tuning knobs of libcurvealign on this GPU and write the
cache that default_context() loads.

    python -m paper_2501_17779_amd.tune_all [--out FILE] [--quick]

Tunes the team-kernel grid and the all-pairs tile width for n = 64..1024,
the thread count of the two largest block-engine size classes (FP32), the
persistent grid of the five classes, and the radix
schedule of every block-engine transform size from 16 to 8192 with no prime
factor above 7 that some n in [2, 4096] uses (--quick: powers of two and the
class maxima only).  Each (knob, key) is measured by ca_autotune on a
synthetic batch generated on the device; progress is printed per knob.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import paper_2501_17779_amd as ca


def _smooth7(m: int) -> bool:
    for p in (2, 3, 5, 7):
        while m % p == 0:
            m //= p
    return m == 1


def _transform_size(n: int) -> int:
    if _smooth7(n):
        return n
    m = 2 * n
    while not _smooth7(m):
        m += 1
    return m


def plan_sizes(quick: bool) -> list[int]:
    used = {_transform_size(n) for n in range(2, ca.MAX_N + 1)}
    sizes = sorted(m for m in used if m >= 16)
    if quick:
        sizes = [m for m in sizes if m & (m - 1) == 0 or m in (512, 1024, 2048, 4096, 8192)]
    return sizes


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=ca.TUNE_CACHE)
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 2
    os.environ["CURVEALIGN_TUNE_FILE"] = ""        # start from the defaults
    ctx = ca.Context(0)
    t0 = time.time()
    for knob, keys in (("team_grid", [64, 128, 256, 512, 1024]),
                       ("allpairs_cols", [64, 128, 256, 512, 1024]),
                       ("block_threads", [3, 4]),
                       ("block_grid", [0, 1, 2, 3, 4])):
        for key in keys:
            ms = ca.autotune(knob, key, ctx=ctx)
            print(f"{knob}[{key}] = {ca.tune_get(knob, key, ctx=ctx)}  {ms:.4f} ms", flush=True)
    sizes = plan_sizes(args.quick)
    changed = 0
    for i, m in enumerate(sizes):
        ca.autotune("block_plan", m, ctx=ctx)
        r = ca.tune_get("block_plan", m, ctx=ctx)
        changed += r != _default_radices(m)
        if i % 25 == 0 or i == len(sizes) - 1:
            print(f"block_plan: {i + 1}/{len(sizes)} sizes, {changed} non-default "
                  f"({time.time() - t0:.1f} s)", flush=True)
    ca.tune_save(args.out, ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    print(f"wrote {args.out} ({time.time() - t0:.1f} s)", flush=True)
    return 0


def _default_radices(m: int) -> list[int]:
    r = []
    while m % 8 == 0:
        r.append(8)
        m //= 8
    if m % 4 == 0:
        r.append(4)
        m //= 4
    if m % 2 == 0:
        r.append(2)
        m //= 2
    for p in (3, 5, 7):
        while m % p == 0:
            r.append(p)
            m //= p
    return r


if __name__ == "__main__":
    sys.exit(main())
