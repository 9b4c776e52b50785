"""Pins for the FP64 arc-length resampling oracle (CPU only)."""
import os

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import resample_ref as rr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "square_resample.txt")


def load_square_golden():
    out = {"linear": np.zeros((8, 2)), "spline": np.zeros((8, 2))}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        mode, n, x, y = line.split()
        out[mode][int(n)] = (float(x), float(y))
    return out


SQUARE = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float64)


@pytest.mark.parametrize("mode,name", [(rr.LINEAR, "linear"), (rr.SPLINE, "spline")])
def test_square_worked_example(mode, name):
    z, info = rr.resample(SQUARE, 8, mode)
    g = load_square_golden()[name]
    assert info["L"] == 4.0
    assert np.max(np.abs(z.real - g[:, 0])) < 1e-15
    assert np.max(np.abs(z.imag - g[:, 1])) < 1e-15


def test_spline_matches_library_periodic_spline():
    rng = np.random.default_rng(0)
    K = 57
    ang = np.sort(rng.uniform(0, 2 * np.pi, K))
    P = np.stack([(1 + 0.2 * np.cos(3 * ang)) * np.cos(ang),
                  (1 + 0.2 * np.cos(3 * ang)) * np.sin(ang)], 1)
    s, h, L = rr.arclength_parameters(P)
    M = rr.periodic_spline_moments(h, P)
    t = np.linspace(0, 1, 1000, endpoint=False)
    ours = rr.evaluate(s, h, P, M, t)
    ref = CubicSpline(np.append(s, 1.0), np.vstack([P, P[:1]]), bc_type="periodic")(t)
    assert np.max(np.abs(ours - ref)) < 1e-12


def test_arclength_parameters_closed_form():
    """Eq. (arc-length-param) on a 3-4-5 triangle: s = (0, 3/12, 7/12), L = 12."""
    P = np.array([[0, 0], [3, 0], [3, 4]], dtype=float)
    s, h, L = rr.arclength_parameters(P)
    assert L == 12.0
    assert np.allclose(s, [0, 3 / 12, 7 / 12], atol=0, rtol=1e-15)
    assert np.allclose(h, [3 / 12, 4 / 12, 5 / 12], atol=0, rtol=1e-15)


def test_regular_polygon_nodes_are_the_vertices():
    """Equal chords put the knots at s = j/K, so N = K nodes hit the knots."""
    K = 24
    a = 2 * np.pi * np.arange(K) / K + 0.3
    P = np.stack([np.cos(a), np.sin(a)], 1)
    z, info = rr.resample(P, K, rr.SPLINE)
    expect = (P[:, 0] + 1j * P[:, 1]) / info["L"]
    assert np.max(np.abs(z - (expect - expect.mean()))) < 1e-15


def test_linear_nodes_on_polygon_equally_spaced():
    rng = np.random.default_rng(2)
    K, N = 11, 64
    ang = np.sort(rng.uniform(0, 2 * np.pi, K))
    P = np.stack([np.cos(ang), 0.6 * np.sin(ang)], 1)
    z, info = rr.resample(P, N, rr.LINEAR)
    # undo centering by locating node 0 on the first vertex's chord: the
    # uncentred nodes are z*L + c with c the common offset; node 0 is vertex 0.
    c = P[0, 0] + 1j * P[0, 1] - z[0] * info["L"]
    w = z * info["L"] + c
    # equal spacing in arc length: consecutive nodes on the same chord are L/N apart
    d = np.abs(np.diff(np.append(w, w[0])))
    assert np.all(d <= info["L"] / N + 1e-12)
    assert np.sum(d > info["L"] / N - 1e-12) >= N - K
    # every node lies on a chord of the polygon
    Q = P[:, 0] + 1j * P[:, 1]
    for x in w:
        best = np.inf
        for j in range(K):
            p, q = Q[j], Q[(j + 1) % K]
            u = np.clip(np.real((x - p) * np.conj(q - p)) / abs(q - p) ** 2, 0, 1)
            best = min(best, abs(x - (p + u * (q - p))))
        assert best < 1e-12


def test_spline_fourth_order_on_circle():
    """The periodic cubic spline through a regular K-gon deviates from the circle
    by O(h^4): halving h divides the radial error by about 16."""
    errs = []
    for K in (16, 32, 64):
        a = 2 * np.pi * np.arange(K) / K
        P = np.stack([np.cos(a), np.sin(a)], 1)
        z, info = rr.resample(P, 4 * K, rr.SPLINE)
        errs.append(np.max(np.abs(np.abs(z * info["L"]) - 1.0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13 < r1 < 19 and 13 < r2 < 19


def test_spline_fourth_order_nonuniform_ellipse():
    """Non-uniform but centrally symmetric knots on an ellipse: the nodes stay on
    the ellipse to O(h^4) (normal error), ratio ~16 per halving."""
    errs = []
    for K in (32, 64, 128):
        p = 2 * np.pi * np.arange(K) / K
        p = p + 0.25 * np.sin(2 * p)
        P = np.stack([2.0 * np.cos(p), np.sin(p)], 1)
        z, info = rr.resample(P, 2 * K, rr.SPLINE)
        w = z * info["L"]
        errs.append(np.max(np.abs((w.real / 2.0) ** 2 + w.imag ** 2 - 1.0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 11 < r1 < 22 and 11 < r2 < 22


@pytest.mark.parametrize("mode", [rr.SPLINE, rr.LINEAR])
def test_rigid_and_scale_equivariance(mode):
    rng = np.random.default_rng(4)
    K = 40
    ang = np.sort(rng.uniform(0, 2 * np.pi, K))
    P = np.stack([(1 + 0.3 * np.cos(2 * ang)) * np.cos(ang), (1 + 0.3 * np.cos(2 * ang)) * np.sin(ang)], 1)
    z, _ = rr.resample(P, 50, mode)
    phi, c = 0.8, np.array([3.0, -2.0])
    Rm = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
    z2, _ = rr.resample(2.5 * P @ Rm.T + c, 50, mode)
    assert np.max(np.abs(z2 - np.exp(1j * phi) * z)) < 1e-13


def test_cleaning_drops_closing_and_repeated_vertices():
    rng = np.random.default_rng(6)
    K = 30
    ang = np.sort(rng.uniform(0, 2 * np.pi, K))
    P = np.stack([np.cos(ang), np.sin(ang)], 1)
    Q = np.vstack([P[:5], P[4:5], P[4:5], P[5:], P[:1], P[:1]])   # dup run + closing copies
    a, ia = rr.resample(P, 32)
    b, ib = rr.resample(Q, 32)
    assert ib["K"] == K
    assert np.max(np.abs(a - b)) == 0.0


def test_degenerate_inputs():
    z, info = rr.resample(np.array([[1.0, 1.0], [1.0, 1.0], [2.0, 2.0]]), 16)
    assert info["degenerate"] and np.all(z == 0)
    z, info = rr.resample(np.array([[1.0, 1.0]] * 5), 16)
    assert info["degenerate"]


def test_signed_area_pins():
    """Shoelace area: the unit square, a triangle's half cross product, a
    regular n-gon's closed form (n/2) sin(2 pi / n) r^2; sign flips with the
    vertex order, value invariant under translation, rotation and a change
    of starting vertex, scaled by s^2."""
    sq = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    assert rr.signed_area(sq) == 1.0
    assert rr.signed_area(sq[::-1]) == -1.0
    a, b, c = np.array([0.3, -0.2]), np.array([2.0, 0.5]), np.array([0.7, 1.9])
    cross = (b - a)[0] * (c - a)[1] - (b - a)[1] * (c - a)[0]
    assert abs(rr.signed_area(np.stack([a, b, c])) - 0.5 * cross) < 1e-15
    for n in (3, 7, 64):
        t = 2 * np.pi * np.arange(n) / n
        P = 1.7 * np.stack([np.cos(t), np.sin(t)], 1)
        assert abs(rr.signed_area(P) - 0.5 * n * np.sin(2 * np.pi / n) * 1.7 ** 2) < 1e-12
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0, 2 * np.pi, 50))
    P = np.stack([(1 + 0.2 * np.cos(3 * t)) * np.cos(t), (1 + 0.2 * np.cos(3 * t)) * np.sin(t)], 1)
    A = rr.signed_area(P)
    assert A > 0
    th = 0.8
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    assert abs(rr.signed_area(P @ R.T + [5.0, -3.0]) - A) < 1e-12
    assert abs(rr.signed_area(np.roll(P, 17, axis=0)) - A) < 1e-12
    assert abs(rr.signed_area(2.5 * P) - 6.25 * A) < 1e-12
    # the resampler reports the cleaned polygon's area
    z, info = rr.resample(np.vstack([P, P[:1]]), 64)
    assert abs(info["area"] - A) < 1e-12
    z, info = rr.resample(P[::-1], 64)
    assert abs(info["area"] + A) < 1e-12
