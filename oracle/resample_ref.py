"""FP64 reference for uniform arc-length resampling of a closed polygon.

TEST INFRASTRUCTURE ONLY: the GPU resampler is checked against this module.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it; the library never imports it and it imports nothing from the library.

Steps, in the order of section 2 of the paper (the two-step arc-length
parametrization that precedes the numerical experiments):

1. Clean the node list (reading of the input format: the paper lists closed
   curves with first == last point; a repeated closing vertex and runs of
   consecutive duplicate vertices carry no geometry and are dropped).
2. Eq. (arc-length-param): s^l = L^l / L^N with L^l the cumulative sum of the
   chord lengths ||beta^m - beta^{m-1}||; the closing chord back to the first
   vertex is included, so s runs over [0, 1) and s = 1 is the first vertex
   again.
3. Cubic-spline interpolation through the pairs (s^l, beta^l).  The paper
   says "cubic splines"; for a closed curve the reading taken here is the
   periodic C2 interpolating cubic spline.  A piecewise-linear mode is kept
   as the simplest interpolant.
4. Evaluation at the uniform parameters t_n = n / N, n = 0..N-1 (N distinct
   nodes; the paper's duplicated end point is omitted).
5. Scaling by 1 / L (unit length, section 1 and the first paragraph of
   section 2) and subtraction of the mean of the N nodes (centering: reading,
   the node mean is the translation that minimises the discrete energy).

The spline's second derivatives come from the standard cyclic tridiagonal
system, solved with a sparse direct solver (a library step).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

SPLINE = 0
LINEAR = 1


def clean_polygon(P: np.ndarray) -> np.ndarray:
    """Drop trailing copies of the first vertex, then consecutive duplicates."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 2)
    k = len(P)
    while k > 1 and P[k - 1, 0] == P[0, 0] and P[k - 1, 1] == P[0, 1]:
        k -= 1
    P = P[:k]
    if k <= 1:
        return P
    keep = np.ones(k, dtype=bool)
    keep[1:] = np.any(P[1:] != P[:-1], axis=1)
    return P[keep]


def signed_area(P: np.ndarray) -> float:
    """Shoelace area of the closed polygon P (K, 2), positive when the vertices
    run counter-clockwise (the orientation the paper assumes, section 1)."""
    P = np.asarray(P, dtype=np.float64).reshape(-1, 2)
    x, y = P[:, 0], P[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def arclength_parameters(P: np.ndarray):
    """Eq. (arc-length-param) for a closed polygon.

    Returns (s, h, L): s[j] = L_j / L for j = 0..K-1 (s[0] = 0), the chord
    lengths normalised by L as h[j] = ||P[j+1] - P[j]|| / L (indices mod K),
    and the perimeter L.
    """
    nxt = np.roll(P, -1, axis=0)
    seg = np.hypot(nxt[:, 0] - P[:, 0], nxt[:, 1] - P[:, 1])
    L = float(seg.sum())
    cum = np.concatenate([[0.0], np.cumsum(seg)[:-1]])
    return cum / L, seg / L, L


def periodic_spline_moments(h: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Second derivatives M_j of the periodic cubic spline through (s_j, P_j).

    Row j of the cyclic system (indices mod K):
      h[j-1] M[j-1] + 2 (h[j-1] + h[j]) M[j] + h[j] M[j+1]
          = 6 ((P[j+1] - P[j]) / h[j] - (P[j] - P[j-1]) / h[j-1])
    """
    K = len(h)
    j = np.arange(K)
    jm = (j - 1) % K
    jp = (j + 1) % K
    rows = np.concatenate([j, j, j])
    cols = np.concatenate([jm, j, jp])
    vals = np.concatenate([h[jm], 2.0 * (h[jm] + h), h])
    A = sp.csc_matrix((vals, (rows, cols)), shape=(K, K))
    dP = (P[jp] - P) / h[:, None]
    rhs = 6.0 * (dP - dP[jm])
    M = np.empty_like(P)
    lu = spla.splu(A)
    M[:, 0] = lu.solve(rhs[:, 0])
    M[:, 1] = lu.solve(rhs[:, 1])
    return M


def evaluate(s: np.ndarray, h: np.ndarray, P: np.ndarray, M: np.ndarray | None,
             t: np.ndarray) -> np.ndarray:
    """Evaluate the interpolant at parameters t in [0, 1).

    M is None for the piecewise-linear interpolant.  On [s_j, s_j + h_j]
    with a = s_j + h_j - t and b = t - s_j the cubic is
      M_j a^3/(6h) + M_{j+1} b^3/(6h) + (P_j - M_j h^2/6) a/h
                                     + (P_{j+1} - M_{j+1} h^2/6) b/h.
    """
    K = len(s)
    j = np.searchsorted(s, t, side="right") - 1
    j = np.clip(j, 0, K - 1)
    jp = (j + 1) % K
    hj = h[j][:, None]
    b = (t - s[j])[:, None]
    a = hj - b
    if M is None:
        return P[j] + (P[jp] - P[j]) * (b / hj)
    return (M[j] * a ** 3 / (6.0 * hj) + M[jp] * b ** 3 / (6.0 * hj)
            + (P[j] - M[j] * hj ** 2 / 6.0) * (a / hj)
            + (P[jp] - M[jp] * hj ** 2 / 6.0) * (b / hj))


def resample(P, n: int, mode: int = SPLINE):
    """Raw closed polygon (K, 2) -> n centred unit-length nodes (complex128).

    Returns (z, info) where info holds the cleaned polygon size, the
    perimeter L, the squared norm (1/n) sum |z|^2 and the signed area of the
    cleaned polygon (negative: clockwise vertices, kept in the given order).
    A polygon with fewer than 3 distinct vertices or zero perimeter is
    degenerate: z is all zero and info['degenerate'] is True.
    """
    Q = clean_polygon(P)
    K = len(Q)
    if K < 3:
        return np.zeros(n, dtype=np.complex128), {"K": K, "L": 0.0, "degenerate": True,
                                                  "sqnorm": 0.0}
    s, h, L = arclength_parameters(Q)
    if not (L > 0.0):
        return np.zeros(n, dtype=np.complex128), {"K": K, "L": L, "degenerate": True,
                                                  "sqnorm": 0.0}
    M = periodic_spline_moments(h, Q) if mode == SPLINE else None
    t = np.arange(n, dtype=np.float64) / n
    X = evaluate(s, h, Q, M, t) / L
    z = X[:, 0] + 1j * X[:, 1]
    z = z - z.mean()
    return z, {"K": K, "L": L, "degenerate": False, "sqnorm": float(np.mean(np.abs(z) ** 2)),
               "area": signed_area(Q)}
