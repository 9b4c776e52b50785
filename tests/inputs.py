"""Test inputs: seeded raw polygons from synth/ resampled by the FP64 oracle.

The alignment parity tests feed the same FP32-rounded uniform nodes to the GPU
library and to the oracle; those nodes come from the oracle's resampler, never
from the GPU path.
"""
from __future__ import annotations

import functools

import numpy as np

from oracle import resample_ref as rr
from synth import curves


def _xy_to_c64(z: np.ndarray) -> np.ndarray:
    return z.astype(np.complex64)


def resample_many(raw: np.ndarray, n: int, mode: int = rr.SPLINE) -> np.ndarray:
    """raw float32 (B, M, 2) -> complex64 (B, n) via the oracle resampler."""
    out = np.empty((raw.shape[0], n), dtype=np.complex64)
    for b in range(raw.shape[0]):
        z, _ = rr.resample(raw[b].astype(np.float64), n, mode)
        out[b] = z
    return out


@functools.lru_cache(maxsize=None)
def batch(seed: int, B: int, n: int, n_raw: int | None = None):
    """Pairs like the N=1024 batch workload: curve 2 is a rotated, restarted,
    noisy copy sampled at jittered parameters; both resampled to n nodes."""
    r1, r2 = curves.batch_pairs(seed, B, n_raw or n)
    return resample_many(r1, n), resample_many(r2, n)


@functools.lru_cache(maxsize=None)
def single(seed: int, n: int = 256):
    """The one-pair workload (n_raw = n vertices, FP64 nodes)."""
    r1, r2, truth = curves.single_pair(seed, n_raw=n)
    z1, _ = rr.resample(r1.astype(np.float64), n)
    z2, _ = rr.resample(r2.astype(np.float64), n)
    return z1, z2, truth


@functools.lru_cache(maxsize=None)
def gallery(seed: int, M: int, n: int, n_raw: int = 2048):
    g = curves.gallery(seed, M, n_raw)
    return resample_many(g, n)


@functools.lru_cache(maxsize=None)
def ragged(seed: int, B: int, nmin: int = 64, nmax: int = 4096):
    """Ragged pairs: raw CSR polygons plus oracle-resampled nodes (flat, CSR)."""
    d = curves.ragged_pairs(seed, B, nmin, nmax)
    n = d["n"].astype(np.int64)
    off = np.zeros(B + 1, dtype=np.int64)
    off[1:] = np.cumsum(n)
    z1 = np.empty(off[-1], dtype=np.complex64)
    z2 = np.empty(off[-1], dtype=np.complex64)
    for b in range(B):
        p1 = d["raw1"][d["off1"][b]:d["off1"][b + 1]].astype(np.float64)
        p2 = d["raw2"][d["off2"][b]:d["off2"][b + 1]].astype(np.float64)
        z1[off[b]:off[b + 1]] = rr.resample(p1, int(n[b]))[0]
        z2[off[b]:off[b + 1]] = rr.resample(p2, int(n[b]))[0]
    d = dict(d)
    d.update({"z1": z1, "z2": z2, "off": off})
    return d
