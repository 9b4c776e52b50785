"""Pins for the SRV oracle (section 3): closed forms, invariances and the
exact recovery of a known (t0, R) in Eq. (dist2-energy)."""
import math

import numpy as np
import pytest

import oracle
from oracle import srv_ref


def curve(seed, n, K=8, A=0.2):
    rng = np.random.default_rng(seed)
    t = np.arange(n) * (2 * np.pi / n)
    k = np.arange(1, K + 1)
    a = rng.normal(size=K) * (A / k)
    phi = rng.uniform(0, 2 * np.pi, size=K)
    r = 1.0 + (a[:, None] * np.cos(np.outer(k, t) + phi[:, None])).sum(0)
    return r * np.exp(1j * t)


@pytest.mark.parametrize("n", [3, 17, 256])
def test_squared_norm_is_the_perimeter(n):
    """int |q|^2 dt = int |beta'| dt = length: (1/n) sum |q_k|^2 = polygon perimeter."""
    z = curve(n, n)
    q = srv_ref.srv(z)
    per = np.sum(np.abs(np.roll(z, -1) - z))
    assert abs(np.mean(np.abs(q) ** 2) - per) < 1e-13 * per


@pytest.mark.parametrize("n,r", [(8, 1.0), (100, 0.3), (1024, 2.5)])
def test_regular_polygon_closed_form(n, r):
    """Regular n-gon of radius r, counter-clockwise: every |beta'_k| equals
    n * 2 r sin(pi/n) and q_k points along the chord, at angle
    2 pi k/n + pi/2 + pi/n."""
    k = np.arange(n)
    z = r * np.exp(2j * np.pi * k / n)
    q = srv_ref.srv(z)
    speed = n * 2 * r * math.sin(math.pi / n)
    want = math.sqrt(speed) * np.exp(1j * (2 * np.pi * k / n + np.pi / 2 + np.pi / n))
    assert np.max(np.abs(q - want)) < 1e-12 * math.sqrt(speed)


def test_equivariances():
    """Translation invariance, rotation and start-index equivariance, and
    q(c beta) = sqrt(c) q(beta) for a scale c > 0."""
    z = curve(5, 200)
    q = srv_ref.srv(z)
    assert np.max(np.abs(srv_ref.srv(z + (3 - 2j)) - q)) < 1e-12
    phi = 0.7
    assert np.max(np.abs(srv_ref.srv(np.exp(1j * phi) * z) - np.exp(1j * phi) * q)) < 1e-12
    assert np.max(np.abs(srv_ref.srv(np.roll(z, -37)) - np.roll(q, -37))) < 1e-12
    assert np.max(np.abs(srv_ref.srv(4.0 * z) - 2.0 * q)) < 1e-12


def test_zero_length_segment():
    z = np.array([0, 1, 1, 1j], dtype=np.complex128)
    q = srv_ref.srv(z)
    assert q[1] == 0 and np.all(q[[0, 2, 3]] != 0)


@pytest.mark.parametrize("n,m0,theta0", [(64, 5, 0.9), (300, 123, -2.0)])
def test_step_recovers_known_start_and_rotation(n, m0, theta0):
    """q2* = R(theta0) q1(t + t0) with t0 = m0 / n (matrix form of section 2):
    the step returns that t0 and R with zero energy."""
    q1 = srv_ref.srv(curve(n + 1, n))
    R0 = oracle.R_paper(theta0)
    b1 = np.stack([q1.real, q1.imag], 1)
    b2s = np.stack([R0 @ b1[(k + m0) % n] for k in range(n)])
    q2s = b2s[:, 0] + 1j * b2s[:, 1]
    t0, R, E = srv_ref.srv_step(q1, q2s)
    assert t0 == m0 / n
    assert np.max(np.abs(R - R0)) < 1e-12
    assert E < 1e-24


def test_step_energy_is_the_minimum_over_shifts_and_angles():
    """Brute force over every start index and a fine angle grid of the
    discrete Eq. (dist2-energy)."""
    n = 48
    q1, q2s = srv_ref.srv(curve(7, n)), srv_ref.srv(curve(8, n))
    t0, R, E = srv_ref.srv_step(q1, q2s)
    best = np.inf
    for m in range(n):
        sh = np.roll(q1, -m)
        for th in np.linspace(-np.pi, np.pi, 721):
            Rm = oracle.R_paper(th)
            v = Rm @ np.stack([sh.real, sh.imag])
            e = np.mean((v[0] - q2s.real) ** 2 + (v[1] - q2s.imag) ** 2)
            best = min(best, e)
    assert E <= best + 1e-12
    assert best - E < 1e-4 * (np.mean(np.abs(q1) ** 2) + np.mean(np.abs(q2s) ** 2))
    # the returned (t0, R) attain E
    m = round(t0 * n)
    v = R @ np.stack([np.roll(q1, -m).real, np.roll(q1, -m).imag])
    assert abs(np.mean((v[0] - q2s.real) ** 2 + (v[1] - q2s.imag) ** 2) - E) < 1e-13
