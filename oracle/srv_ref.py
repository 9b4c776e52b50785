"""FP64 reference for the square-root-velocity (SRV) step of section 3.

TEST INFRASTRUCTURE ONLY (see the package docstring): the GPU SRV transform
is checked against this module; the library never imports it.

Section 3 represents a closed curve beta of unit length by its SRV function
q = beta' / |beta'|^(1/2) and proposes to run the rigid alignment of section
2 on SRV functions inside the elastic solver: with gamma fixed, (t0, R)
minimise Eq. (dist2-energy), the integral of |R q1(t + t0) - q2*(t)|^2 with
q2* = sqrt(gamma') q2(gamma).

Discretisation (reading: the paper gives none).  The curve is the closed
polygon through its n nodes z[k] at the uniform parameters t_k = k / n, so
beta' is constant on each segment [t_k, t_{k+1}):  beta'_k = n (z[k+1] - z[k])
(indices mod n), and q is piecewise constant with the value
q_k = beta'_k / |beta'_k|^(1/2) on segment k (0 on a segment of zero length).
For piecewise-constant functions on the same grid and t0 = m / n the integral
of Eq. (dist2-energy) is exactly (1/n) sum_k |R q1[k + m] - q2*[k]|^2, the
discrete energy of section 2 with curve 1 <- q2* and curve 2 <- q1; its
minimiser is therefore the slow method of the alignment oracle on (q2*, q1).
No centring is applied to q: the energy of Eq. (dist2-energy) has no
translation, and the rigid alignment never translates.
"""
from __future__ import annotations

import numpy as np


def srv(z) -> np.ndarray:
    """SRV values q_k (complex128, one per segment) of the closed polygon through z."""
    z = np.asarray(z, dtype=np.complex128)
    n = z.shape[0]
    d = n * (np.roll(z, -1) - z)           # beta' on segment k
    a = np.abs(d)
    q = np.zeros(n, dtype=np.complex128)
    nz = a > 0
    q[nz] = d[nz] / np.sqrt(a[nz])
    return q


def srv_step(q1, q2s):
    """Minimiser of Eq. (dist2-energy) over (t0, R) for piecewise-constant q1
    and q2* on the same grid: returns (t0, R, E) with t0 = m / n, R = R(theta)
    of section 2 and E the minimal discrete energy."""
    from . import initializer
    t0, R, res = initializer(np.asarray(q2s), np.asarray(q1))
    return t0, R, res["E"]
