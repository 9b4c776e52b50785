"""Seeded synthetic closed curves: raw polygons only.

This module draws random star-shaped curves and samples them into raw vertex
lists.  It contains none of the alignment method's arithmetic (no arc length,
no interpolation, no FFT, no correlation): turning a raw polygon into uniform
arc-length nodes is the resampler's job, done by the library on the GPU or by
the oracle on the CPU.  Both sides take their inputs from here.

Curve family (a stand-in for the paper's cell boundaries and synthetic
shapes, which are not available): r(t) = 1 + sum_{k=1..K} a_k cos(k t + phi_k),
z(t) = r(t) e^{it}, with a_k ~ N(0, (A/k)^2), phi_k ~ U[0, 2 pi).  A draw
with min r <= 0.05 on a 4096-point grid is rejected and redrawn, so every
curve is a simple, counter-clockwise, star-shaped loop.

Templates follow the paper's validation protocol (same curve with a moved
starting point and a rotation): curve 2 is curve 1 rotated by theta0, started
at another parameter, optionally sampled at jittered positions, plus Gaussian
noise per coordinate.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
KMAX = 16


def seed_for(config: int) -> int:
    return 17779 + int(config)


def _draw_coeffs(rng: np.random.Generator, B: int, K, A: float):
    """Complex Fourier coefficients c_k = a_k e^{i phi_k}, shape (B, KMAX)."""
    K = np.broadcast_to(np.asarray(K), (B,))
    c = np.zeros((B, KMAX), dtype=np.complex128)
    todo = np.arange(B)
    grid = np.exp(1j * np.outer(np.arange(1, KMAX + 1), np.linspace(0, TWO_PI, 4096,
                                                                   endpoint=False)))
    while todo.size:
        k = np.arange(1, KMAX + 1)
        a = rng.normal(size=(todo.size, KMAX)) * (A / k)
        phi = rng.uniform(0.0, TWO_PI, size=(todo.size, KMAX))
        a[k[None, :] > K[todo][:, None]] = 0.0
        cc = a * np.exp(1j * phi)
        r = 1.0 + (cc @ grid).real
        ok = r.min(axis=1) > 0.05
        c[todo[ok]] = cc[ok]
        todo = todo[~ok]
    return c


def _star(c: np.ndarray, t: np.ndarray) -> np.ndarray:
    """z(t) for coefficient rows c (B, KMAX) at parameters t (B, M)."""
    w = np.exp(1j * t)
    acc = np.zeros_like(w)
    for k in range(KMAX, 0, -1):          # Horner in w = e^{it}
        acc = (acc + c[:, k - 1:k]) * w
    r = 1.0 + acc.real
    return r * w


def _to_xy32(z: np.ndarray) -> np.ndarray:
    out = np.empty(z.shape + (2,), dtype=np.float32)
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return out


def single_pair(seed: int, n_raw: int = 256, K: int = 8, A: float = 0.1,
                sigma: float = 1e-3):
    """One star curve sampled at n_raw uniform parameters and its template:
    rotated by theta0 ~ U[0, 2pi), cyclically shifted by s0 ~ U{0..n_raw-1}
    vertices, plus N(0, sigma^2) noise per coordinate.

    Returns (raw1, raw2, truth) with raw* float32 (n_raw, 2).
    """
    rng = np.random.default_rng(seed)
    c = _draw_coeffs(rng, 1, K, A)
    t = np.arange(n_raw) * (TWO_PI / n_raw)
    z1 = _star(c, t[None, :])[0]
    theta0 = rng.uniform(0.0, TWO_PI)
    s0 = int(rng.integers(0, n_raw))
    z2 = np.exp(1j * theta0) * np.roll(z1, -s0)
    z2 = z2 + sigma * (rng.normal(size=n_raw) + 1j * rng.normal(size=n_raw))
    return _to_xy32(z1), _to_xy32(z2), {"theta0": theta0, "s0": s0}


def batch_pairs(seed: int, B: int, n_raw: int, kmin: int = 8, kmax: int = 16,
                A: float = 0.1, sigma_max: float = 1e-2, jitter: float = 0.4,
                chunk: int = 4096):
    """B independent pairs.  Curve 1: n_raw vertices at uniform parameters.
    Curve 2: the same curve rotated by theta0 ~ U[0, 2pi), started at a
    continuous parameter offset tau ~ U[0, 2pi), sampled at jittered
    parameters 2pi (j + u_j) / n_raw + tau with u_j ~ U(-jitter, jitter),
    plus noise sigma ~ U[0, sigma_max] per coordinate.

    Returns (raw1, raw2) float32 (B, n_raw, 2).
    """
    raw1 = np.empty((B, n_raw, 2), dtype=np.float32)
    raw2 = np.empty((B, n_raw, 2), dtype=np.float32)
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn((B + chunk - 1) // chunk)
    j = np.arange(n_raw)
    for ci, kid in enumerate(kids):
        rng = np.random.default_rng(kid)
        lo, hi = ci * chunk, min(B, (ci + 1) * chunk)
        b = hi - lo
        K = rng.integers(kmin, kmax + 1, size=b)
        c = _draw_coeffs(rng, b, K, A)
        t1 = np.broadcast_to(j * (TWO_PI / n_raw), (b, n_raw))
        raw1[lo:hi] = _to_xy32(_star(c, t1))
        theta0 = rng.uniform(0.0, TWO_PI, size=(b, 1))
        tau = rng.uniform(0.0, TWO_PI, size=(b, 1))
        sigma = rng.uniform(0.0, sigma_max, size=(b, 1))
        u = rng.uniform(-jitter, jitter, size=(b, n_raw))
        t2 = (j[None, :] + u) * (TWO_PI / n_raw) + tau
        z2 = np.exp(1j * theta0) * _star(c, t2)
        z2 = z2 + sigma * (rng.normal(size=(b, n_raw)) + 1j * rng.normal(size=(b, n_raw)))
        raw2[lo:hi] = _to_xy32(z2)
    return raw1, raw2


def gallery(seed: int, M: int, n_raw: int, K: int = 16, A: float = 0.2, chunk: int = 1024):
    """M independent shapes, each sampled at n_raw uniform parameters.
    Returns float32 (M, n_raw, 2)."""
    out = np.empty((M, n_raw, 2), dtype=np.float32)
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn((M + chunk - 1) // chunk)
    j = np.arange(n_raw)
    for ci, kid in enumerate(kids):
        rng = np.random.default_rng(kid)
        lo, hi = ci * chunk, min(M, (ci + 1) * chunk)
        c = _draw_coeffs(rng, hi - lo, K, A)
        t = np.broadcast_to(j * (TWO_PI / n_raw), (hi - lo, n_raw))
        out[lo:hi] = _to_xy32(_star(c, t))
    return out


def smooth7(lo: int = 64, hi: int = 4096) -> np.ndarray:
    """All integers in [lo, hi] whose prime factors are 2, 3, 5 or 7."""
    vals = []
    for n in range(lo, hi + 1):
        m = n
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        if m == 1:
            vals.append(n)
    return np.array(vals, dtype=np.int64)


def ragged_pairs(seed: int, B: int, nmin: int = 64, nmax: int = 4096,
                 ratio=(1.2, 5.0), A: float = 0.1, sigma_max: float = 1e-2,
                 jitter: float = 0.4, chunk: int = 2048):
    """B pairs of raw polygons with uneven sizes.

    Node count N per pair: log-uniform in [nmin, nmax], snapped to the
    nearest (in log distance) 7-smooth integer.  Each raw curve has
    round(U[ratio] * N) vertices (at least 8) placed at density-modulated,
    jittered parameters g(2 pi (j + u_j) / M) with g(t) = t + alpha sin(t - psi),
    alpha ~ U[0, 0.5].  Curve 2 is curve 1 rotated, started at a random
    parameter and noisy, with its own vertex count and placement.

    Returns dict with float32 vertex buffers raw1/raw2, int64 CSR offsets
    off1/off2 (B+1), and int32 node counts n (B).
    """
    cand = smooth7(nmin, nmax)
    logc = np.log(cand)
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn((B + chunk - 1) // chunk)
    Ns, r1, r2, m1s, m2s = [], [], [], [], []
    for ci, kid in enumerate(kids):
        rng = np.random.default_rng(kid)
        b = min(B, (ci + 1) * chunk) - ci * chunk
        draw = rng.uniform(math.log(nmin), math.log(nmax), size=b)
        N = cand[np.abs(logc[None, :] - draw[:, None]).argmin(axis=1)]
        K = rng.integers(8, 17, size=b)
        c = _draw_coeffs(rng, b, K, A)
        theta0 = rng.uniform(0.0, TWO_PI, size=b)
        tau = rng.uniform(0.0, TWO_PI, size=b)
        sigma = rng.uniform(0.0, sigma_max, size=b)
        for i in range(b):
            for which in (1, 2):
                M = max(8, int(round(rng.uniform(*ratio) * N[i])))
                alpha = rng.uniform(0.0, 0.5)
                psi = rng.uniform(0.0, TWO_PI)
                u = rng.uniform(-jitter, jitter, size=M)
                t = (np.arange(M) + u) * (TWO_PI / M)
                t = t + alpha * np.sin(t - psi)
                if which == 1:
                    z = _star(c[i:i + 1], t[None, :])[0]
                    r1.append(_to_xy32(z))
                    m1s.append(M)
                else:
                    z = np.exp(1j * theta0[i]) * _star(c[i:i + 1], (t + tau[i])[None, :])[0]
                    z = z + sigma[i] * (rng.normal(size=M) + 1j * rng.normal(size=M))
                    r2.append(_to_xy32(z))
                    m2s.append(M)
        Ns.append(N)
    n = np.concatenate(Ns).astype(np.int32)
    off1 = np.zeros(B + 1, dtype=np.int64)
    off2 = np.zeros(B + 1, dtype=np.int64)
    off1[1:] = np.cumsum(m1s)
    off2[1:] = np.cumsum(m2s)
    return {"raw1": np.concatenate(r1), "raw2": np.concatenate(r2),
            "off1": off1, "off2": off2, "n": n}


# ----------------------------------------------------------------------------
# The same curve families drawn with torch on a device (fast at full size).
# Streams differ from the numpy versions above but are seeded the same way
# (one torch.Generator per call).

def _t_coeffs(gen, B, K, A, device, grid_pts=4096):
    import torch
    K = torch.as_tensor(K, device=device).expand(B)
    k = torch.arange(1, KMAX + 1, device=device, dtype=torch.float64)
    out = torch.zeros(B, KMAX, dtype=torch.complex128, device=device)
    todo = torch.arange(B, device=device)
    tg = torch.linspace(0, TWO_PI, grid_pts + 1, device=device, dtype=torch.float64)[:-1]
    grid = torch.exp(1j * torch.outer(k, tg))                # (KMAX, G)
    while todo.numel():
        a = torch.randn(todo.numel(), KMAX, generator=gen, device=device, dtype=torch.float64) * (A / k)
        phi = torch.rand(todo.numel(), KMAX, generator=gen, device=device, dtype=torch.float64) * TWO_PI
        a = torch.where(k[None, :] > K[todo][:, None], torch.zeros_like(a), a)
        cc = a * torch.exp(1j * phi)
        r = 1.0 + (cc @ grid).real
        ok = r.min(dim=1).values > 0.05
        out[todo[ok]] = cc[ok]
        todo = todo[~ok]
    return out


def _t_star(c, t, seg=None):
    """z(t) with per-row coefficients c (R, KMAX); t is (R, M), or flat with
    segment ids `seg` mapping each parameter to its coefficient row."""
    import torch
    w = torch.exp(1j * t)
    acc = torch.zeros_like(w)
    for k in range(KMAX, 0, -1):
        ck = c[:, k - 1]
        acc = (acc + (ck[seg] if seg is not None else ck[:, None])) * w
    return (1.0 + acc.real) * w


def _t_xy32(z):
    import torch
    return torch.stack([z.real, z.imag], dim=-1).to(torch.float32)


def batch_pairs_torch(seed: int, B: int, n_raw: int, device, kmin: int = 8, kmax: int = 16,
                      A: float = 0.1, sigma_max: float = 1e-2, jitter: float = 0.4,
                      chunk: int = 8192):
    """Device version of batch_pairs: float32 tensors (B, n_raw, 2)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    raw1 = torch.empty(B, n_raw, 2, dtype=torch.float32, device=device)
    raw2 = torch.empty_like(raw1)
    j = torch.arange(n_raw, device=device, dtype=torch.float64)
    for lo in range(0, B, chunk):
        b = min(B, lo + chunk) - lo
        K = torch.randint(kmin, kmax + 1, (b,), generator=gen, device=device)
        c = _t_coeffs(gen, b, K, A, device)
        raw1[lo:lo + b] = _t_xy32(_t_star(c, (j * (TWO_PI / n_raw)).expand(b, n_raw)))
        theta0 = torch.rand(b, 1, generator=gen, device=device, dtype=torch.float64) * TWO_PI
        tau = torch.rand(b, 1, generator=gen, device=device, dtype=torch.float64) * TWO_PI
        sigma = torch.rand(b, 1, generator=gen, device=device, dtype=torch.float64) * sigma_max
        u = (torch.rand(b, n_raw, generator=gen, device=device, dtype=torch.float64) * 2 - 1) * jitter
        t2 = (j[None, :] + u) * (TWO_PI / n_raw) + tau
        z2 = torch.exp(1j * theta0) * _t_star(c, t2)
        nz = torch.randn(b, n_raw, 2, generator=gen, device=device, dtype=torch.float64)
        z2 = z2 + sigma * (nz[..., 0] + 1j * nz[..., 1])
        raw2[lo:lo + b] = _t_xy32(z2)
    return raw1, raw2


def gallery_torch(seed: int, M: int, n_raw: int, device, K: int = 16, A: float = 0.2):
    """Device version of gallery: float32 tensor (M, n_raw, 2)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    c = _t_coeffs(gen, M, K, A, device)
    j = torch.arange(n_raw, device=device, dtype=torch.float64)
    return _t_xy32(_t_star(c, (j * (TWO_PI / n_raw)).expand(M, n_raw)))


def ragged_pairs_torch(seed: int, B: int, device, nmin: int = 64, nmax: int = 4096,
                       ratio=(1.2, 5.0), A: float = 0.1, sigma_max: float = 1e-2,
                       jitter: float = 0.4, chunk: int = 8192, snap: bool = True):
    """Device version of ragged_pairs.  Returns dict of device tensors:
    raw1, raw2 complex64 flat; off1, off2 int64 (B+1); n int32 (B).
    snap=False keeps the rounded log-uniform draw (any integer size)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    cand = torch.as_tensor(smooth7(nmin, nmax), device=device)
    logc = torch.log(cand.double())
    draw = torch.rand(B, generator=gen, device=device, dtype=torch.float64)
    draw = math.log(nmin) + draw * (math.log(nmax) - math.log(nmin))
    if snap:
        N = cand[(logc[None, :] - draw[:, None]).abs().argmin(dim=1)]
    else:
        N = torch.clamp(torch.round(torch.exp(draw)), nmin, nmax).long()
    out = {"n": N.to(torch.int32)}
    for which in (1, 2):
        rr = torch.rand(B, generator=gen, device=device, dtype=torch.float64)
        Mc = torch.clamp(torch.round((ratio[0] + rr * (ratio[1] - ratio[0])) * N.double()), min=8).long()
        off = torch.zeros(B + 1, dtype=torch.int64, device=device)
        off[1:] = torch.cumsum(Mc, 0)
        out[f"off{which}"] = off
        out[f"_m{which}"] = Mc
    raws = {1: torch.empty(int(out["off1"][-1]), dtype=torch.complex64, device=device),
            2: torch.empty(int(out["off2"][-1]), dtype=torch.complex64, device=device)}
    for lo in range(0, B, chunk):
        b = min(B, lo + chunk) - lo
        K = torch.randint(8, 17, (b,), generator=gen, device=device)
        c = _t_coeffs(gen, b, K, A, device)
        theta0 = torch.rand(b, generator=gen, device=device, dtype=torch.float64) * TWO_PI
        tau = torch.rand(b, generator=gen, device=device, dtype=torch.float64) * TWO_PI
        sigma = torch.rand(b, generator=gen, device=device, dtype=torch.float64) * sigma_max
        for which in (1, 2):
            off = out[f"off{which}"]
            Mc = out[f"_m{which}"][lo:lo + b]
            p0, p1 = int(off[lo]), int(off[lo + b])
            seg = torch.repeat_interleave(torch.arange(b, device=device), Mc)
            jj = torch.arange(p1 - p0, device=device) - (off[lo:lo + b] - p0)[seg]
            alpha = torch.rand(b, generator=gen, device=device, dtype=torch.float64) * 0.5
            psi = torch.rand(b, generator=gen, device=device, dtype=torch.float64) * TWO_PI
            u = (torch.rand(p1 - p0, generator=gen, device=device, dtype=torch.float64) * 2 - 1) * jitter
            t = (jj.double() + u) * (TWO_PI / Mc.double()[seg])
            t = t + alpha[seg] * torch.sin(t - psi[seg])
            if which == 1:
                z = _t_star(c, t, seg)
            else:
                z = torch.exp(1j * theta0[seg]) * _t_star(c, t + tau[seg], seg)
                nz = torch.randn(p1 - p0, 2, generator=gen, device=device, dtype=torch.float64)
                z = z + sigma[seg] * (nz[:, 0] + 1j * nz[:, 1])
            raws[which][p0:p1] = z.to(torch.complex64)
    out["raw1"], out["raw2"] = raws[1], raws[2]
    del out["_m1"], out["_m2"]
    return out
