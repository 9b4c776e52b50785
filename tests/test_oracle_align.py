"""Pins for the FP64 alignment oracle (CPU only).

Each test ties the oracle to something other than itself: a library SVD
with the determinant test of Algorithm 1, brute force over every start index
and a fine angle grid, the paper's FFT formulation of Eq. A-mtx (the fast
method gives exactly the slow method's alignment errors, section 2
experiments), closed forms and invariants.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import resample_ref as rr
from synth import curves


def random_curve(rng, n, K=8, A=0.15):
    """A smooth random closed curve sampled at n uniform parameters (test-only)."""
    t = np.arange(n) * (2 * np.pi / n)
    k = np.arange(1, K + 1)
    a = rng.normal(size=K) * (A / k)
    phi = rng.uniform(0, 2 * np.pi, size=K)
    r = 1.0 + (a[:, None] * np.cos(np.outer(k, t) + phi[:, None])).sum(0)
    z = r * np.exp(1j * t)
    return z - z.mean()


def R_paper(theta):
    """Rotation of section 2: R(theta) = [[cos, sin], [-sin, cos]]."""
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, s], [-s, c]])


def kabsch_svd(A):
    """Algorithm 1 with a library SVD: R = U S~ V^T, S~ = diag(1, +-1)."""
    U, S, Vt = np.linalg.svd(A)
    d = np.linalg.det(U) * np.linalg.det(Vt.T)
    St = np.diag([1.0, 1.0 if d > 0 else -1.0])
    return U @ St @ Vt


@pytest.mark.parametrize("seed", range(6))
def test_closed_form_equals_algorithm1_svd(seed):
    rng = np.random.default_rng(seed)
    n = 48
    z1 = random_curve(rng, n)
    z2 = random_curve(rng, n) if seed % 2 else np.exp(0.7j) * np.roll(z1, 5) + 0.05 * rng.normal(size=n)
    T, H = oracle.shift_scores(z1, z2)
    for m in rng.integers(0, n, size=8):
        A = oracle.a_matrix(z1, z2, m)
        R = kabsch_svd(A)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12
        # same optimal value of tr(R A^T)
        assert abs(np.trace(R @ A.T) - T[m]) <= 1e-12 * max(1.0, abs(T[m]))
        # same rotation: the oracle's angle reproduces the SVD rotation
        assert np.allclose(R_paper(H[m]), R, atol=1e-10)
        # singular values: tr max = s1 + sgn(det A) s2
        s = np.linalg.svd(A, compute_uv=False)
        assert abs(s[0] + np.sign(np.linalg.det(A)) * s[1] - T[m]) < 1e-12 * max(1.0, T[m])


def test_reflection_case_keeps_a_rotation():
    """det(U) det(V) < 0 branch of Algorithm 1: still a proper rotation."""
    A = np.array([[0.3, 0.1], [0.2, -0.5]])     # det A < 0
    R = kabsch_svd(A)
    c, s = A[0, 0] + A[1, 1], A[0, 1] - A[1, 0]
    th = math.atan2(s, c)
    assert np.allclose(R, R_paper(th), atol=1e-12)
    assert abs(np.trace(R @ A.T) - math.hypot(c, s)) < 1e-12


def energy_numpy(z1, z2, m, theta):
    """Eq. disc-energy written with complex numbers (test-side brute force)."""
    n = len(z1)
    w = np.exp(-1j * theta) * np.roll(z2, -m)      # R(theta) beta2^{l (+) m}
    return float(np.sum(np.abs(z1 - w) ** 2) / n)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_over_shifts_and_angle_grid(seed):
    rng = np.random.default_rng(100 + seed)
    n = 16 + 4 * seed
    z1 = random_curve(rng, n)
    z2 = np.exp(1j * rng.uniform(0, 6.28)) * np.roll(random_curve(rng, n) * 0.3 + z1, 3)
    grid = np.linspace(-np.pi, np.pi, 1 << 16, endpoint=False)
    best = (np.inf, None, None)
    for m in range(n):
        w = np.roll(z2, -m)
        # E(theta) = n1 + n2 - (2/n) Re(e^{-i theta} sum conj(z1) w), evaluated on the grid
        d = np.sum(np.conj(z1) * w)
        E = np.mean(np.abs(z1) ** 2) + np.mean(np.abs(w) ** 2) - 2.0 / n * np.real(np.exp(-1j * grid) * d)
        k = int(np.argmin(E))
        # golden-section refinement around the grid minimum on the direct energy
        a, b = grid[k] - 2e-4, grid[k] + 2e-4
        g = (math.sqrt(5) - 1) / 2
        for _ in range(80):
            c1, c2 = b - g * (b - a), a + g * (b - a)
            if energy_numpy(z1, z2, m, c1) < energy_numpy(z1, z2, m, c2):
                b = c2
            else:
                a = c1
        th = 0.5 * (a + b)
        e = energy_numpy(z1, z2, m, th)
        if e < best[0]:
            best = (e, m, th)
    res = oracle.align_pair(z1, z2)
    assert res["m"] == best[1]
    assert abs(oracle.wrap_angle(res["theta_paper"] - best[2])) < 1e-7
    assert abs(res["E"] - best[0]) <= 1e-12 + 1e-10 * best[0]


@pytest.mark.parametrize("n", [17, 64, 100])
def test_fft_formulation_of_a_matrix(n):
    """Convolution-theorem form of Eq. A-mtx: with the reversed curve
    beta~1^l = beta1^{(-l) mod n}, IDFT(DFT(beta~1k) . DFT(beta2j))[m] = A_kj(t_m)."""
    rng = np.random.default_rng(n)
    z1, z2 = random_curve(rng, n), random_curve(rng, n)
    b1 = np.stack([z1.real, z1.imag])
    b2 = np.stack([z2.real, z2.imag])
    rev = (-np.arange(n)) % n
    for k in range(2):
        for j in range(2):
            conv = np.fft.ifft(np.fft.fft(b1[k][rev]) * np.fft.fft(b2[j])).real
            for m in range(n):
                A = oracle.a_matrix(z1, z2, m)
                assert abs(conv[m] - A[k, j]) < 1e-12


def test_fast_method_reaches_the_same_alignment_error():
    """Algorithm 2 in FP64 numpy (12 FFTs, then Kabsch by SVD per start index)
    returns the same (t0, R) and the same error as the slow method."""
    rng = np.random.default_rng(7)
    for n in (64, 128, 256):
        z1 = random_curve(rng, n)
        z2 = np.exp(2.1j) * np.roll(z1, n // 4) + 0.01 * (rng.normal(size=n) + 1j * rng.normal(size=n))
        b1 = np.stack([z1.real, z1.imag])
        b2 = np.stack([z2.real, z2.imag])
        rev = (-np.arange(n)) % n
        A = np.empty((n, 2, 2))
        for k in range(2):
            for j in range(2):
                A[:, k, j] = np.fft.ifft(np.fft.fft(b1[k][rev]) * np.fft.fft(b2[j])).real
        tr = np.empty(n)
        Rs = []
        for m in range(n):
            R = kabsch_svd(A[m])
            Rs.append(R)
            tr[m] = np.trace(R @ A[m].T)
        m_fast = int(np.argmax(tr))
        th_fast = math.atan2(Rs[m_fast][0, 1], Rs[m_fast][0, 0])
        res = oracle.align_pair(z1, z2)
        assert res["m"] == m_fast
        assert abs(oracle.wrap_angle(res["theta_paper"] - th_fast)) < 1e-12
        assert abs(oracle.energy(z1, z2, m_fast, th_fast) - res["E"]) < 1e-14


@pytest.mark.parametrize("n,s0,theta0", [(64, 17, 1.1), (100, 3, -2.5), (256, 200, 0.3), (33, 1, 3.0)])
def test_rotated_shifted_exact_copy(n, s0, theta0):
    """z2[j] = e^{i theta0} z1[(j + s0) mod n]: start index m = n - s0, the
    clockwise angle undoes theta0, zero energy; library convention (s0, -theta0)."""
    rng = np.random.default_rng(n + s0)
    z1 = random_curve(rng, n)
    z2 = np.exp(1j * theta0) * np.roll(z1, -s0)
    res = oracle.align_pair(z1, z2)
    assert res["m"] == (n - s0) % n
    assert abs(oracle.wrap_angle(res["theta_paper"] - theta0)) < 1e-12
    assert res["E"] < 1e-28 + 1e-14 * res["n1"]
    s, th = oracle.to_library_convention(res["m"], res["theta_paper"], n)
    assert s == s0 and abs(oracle.wrap_angle(th + theta0)) < 1e-12


def test_paper_validation_protocol():
    """Template = reference with its start moved from 0 to 0.25 and rotated by
    pi/3 (experiments of section 2).  Found: t0 = 0.75 and the clockwise pi/3
    that undoes the rotation, zero energy."""
    rng = np.random.default_rng(3)
    for n in (64, 256, 1024):
        z1 = random_curve(rng, n)
        z2 = np.exp(1j * np.pi / 3) * np.roll(z1, -(n // 4))
        res = oracle.align_pair(z1, z2)
        assert res["m"] / n == 0.75
        assert abs(res["theta_paper"] - np.pi / 3) < 1e-12
        assert res["E"] < 1e-14 * res["n1"]


@pytest.mark.parametrize("seed", range(5))
def test_swap_symmetry(seed):
    rng = np.random.default_rng(50 + seed)
    n = 96
    z1, z2 = random_curve(rng, n), random_curve(rng, n)
    a, b = oracle.align_pair(z1, z2), oracle.align_pair(z2, z1)
    assert b["m"] == (n - a["m"]) % n
    assert abs(oracle.wrap_angle(a["theta_paper"] + b["theta_paper"])) < 1e-12
    assert abs(a["E"] - b["E"]) < 1e-14


def test_energy_expansion_and_bounds():
    """E^h = ||b1||^2 + ||b2||^2 - 2 tr(RA^T)/n (rewrite of Eq. disc-energy0),
    0 <= E <= n1 + n2, and the optimum is below the energy at random (m, theta)."""
    rng = np.random.default_rng(11)
    n = 80
    z1, z2 = random_curve(rng, n), random_curve(rng, n) * 0.7
    res = oracle.align_pair(z1, z2)
    assert abs(res["E"] - (res["n1"] + res["n2"] - 2 * res["T"] / n)) < 1e-14
    assert 0.0 <= res["E"] <= res["n1"] + res["n2"]
    for _ in range(50):
        m, th = int(rng.integers(0, n)), rng.uniform(-np.pi, np.pi)
        assert oracle.energy(z1, z2, m, th) >= res["E"] - 1e-15


def test_scale_invariance():
    rng = np.random.default_rng(12)
    n = 64
    z1, z2 = random_curve(rng, n), random_curve(rng, n)
    a = oracle.align_pair(z1, z2)
    b = oracle.align_pair(3.0 * z1, 3.0 * z2)
    assert a["m"] == b["m"]
    assert abs(a["theta_paper"] - b["theta_paper"]) < 1e-12
    assert abs(b["E"] - 9.0 * a["E"]) < 1e-12


def test_circle_all_shifts_tie():
    """For a circle every start index is optimal; the angle moves by 2 pi / n per index."""
    n = 64
    z = np.exp(2j * np.pi * np.arange(n) / n)
    T, H = oracle.shift_scores(z, z)
    assert np.ptp(T) < 1e-12
    d = oracle.wrap_angle(np.diff(H))
    assert np.allclose(d, 2 * np.pi / n, atol=1e-12)


def test_k_fold_symmetry_gives_k_ties():
    n, k = 120, 3
    t = np.arange(n) * 2 * np.pi / n
    z = (1 + 0.3 * np.cos(k * t)) * np.exp(1j * t)
    T, _ = oracle.shift_scores(z, z)
    top = np.sort(np.argsort(-T)[:k])
    assert list(top) == [0, n // k, 2 * n // k]
    assert np.ptp(T[top]) < 1e-12
    rest = np.delete(T, top)
    assert rest.max() < T[0] * (1 - 1e-4)


def symmetric_curve(n, fold, a=0.3):
    """Nodes of r(t) = 1 + a cos(fold t), t = 2 pi l / n, with the fold-fold
    symmetry exact in floating point: the first n/fold nodes are computed and
    the others are copies turned by a quarter turn (fold 4, (x, y) -> (-y, x))
    or a half turn (fold 2, (x, y) -> (-x, -y)), both exact."""
    assert fold in (2, 4) and n % fold == 0
    q = n // fold
    t = 2 * np.pi * np.arange(q) / n
    r = 1.0 + a * np.cos(fold * t)
    x, y = r * np.cos(t), r * np.sin(t)
    xs, ys = [x], [y]
    for _ in range(fold - 1):
        if fold == 4:
            x, y = -y, x
        else:
            x, y = -x, -y
        xs.append(x)
        ys.append(y)
    z = np.empty(n, dtype=np.complex128)
    z.real = np.concatenate(xs)
    z.imag = np.concatenate(ys)
    return z


@pytest.mark.parametrize("n,fold,m0", [(64, 4, 11), (96, 4, 70), (50, 2, 7), (62, 2, 40)])
def test_exact_ties_go_to_the_smallest_shift(n, fold, m0):
    """Algorithm 2 keeps the highest value and is silent on exact ties; the
    oracle reports the tied start index whose shift s = (n - m) mod n is
    smallest.  A curve with exact fold-fold symmetry read from start index m0
    ties exactly (bit for bit) at m = -m0 + j n / fold, j = 0..fold-1: a turn
    by 2 pi / fold negates or swaps the sums of Eq. A-mtx term by term.  The
    expected index is worked out here by hand from that set; keeping the
    smallest m, or the last of the scan, picks another member."""
    z1 = symmetric_curve(n, fold)
    z2 = np.roll(z1, -m0)                      # z2[l] = z1[(l + m0) mod n]
    T, _ = oracle.shift_scores(z1, z2)
    ties = sorted(((-m0 + j * n // fold) % n) for j in range(fold))
    assert np.ptp(T[ties]) == 0.0              # exact ties
    assert np.delete(T, ties).max() < T[ties[0]] * (1 - 1e-6)
    shifts = [(n - m) % n for m in ties]
    expect_m = ties[int(np.argmin(shifts))]
    assert expect_m != min(ties)               # the two tie rules differ here
    res = oracle.align_pair(z1, z2)
    assert res["m"] == expect_m
    # at tie member m the copy is curve 1 turned by k turns of 2 pi / fold,
    # k = ((m + m0) mod n) / (n / fold), counter-clockwise; R(theta) of
    # section 2 turns it back clockwise by theta = 2 pi k / fold, and the
    # energy vanishes
    k = ((expect_m + m0) % n) // (n // fold)
    assert abs(oracle.wrap_angle(res["theta_paper"] - 2 * np.pi * k / fold)) < 1e-12
    assert res["E"] < 1e-28
    # the batch entry point applies the same rule
    m, _, _, _, _ = oracle.align_batch_f32(z1[None].astype(np.complex64), z2[None].astype(np.complex64))
    T32, _ = oracle.shift_scores(z1.astype(np.complex64), z2.astype(np.complex64))
    assert np.ptp(T32[ties]) == 0.0
    assert m[0] == expect_m
    # initializer hand-off: t0 = m / n with the same m
    t0, R, _ = oracle.initializer(z1, z2)
    assert t0 == expect_m / n
    assert np.allclose(R, R_paper(2 * np.pi * k / fold), atol=1e-12)


@pytest.mark.parametrize("n", [60, 64, 97])
def test_circle_through_align_pair(n):
    """A circle aligned to a turned, restarted copy of itself: every start
    index is optimal up to rounding (T constant, E = 0), and the angle at the
    returned index is the one that undoes the turn and the restart: the node
    at start index m sits 2 pi m / n further along the circle."""
    alpha, m0 = 0.9, 5
    l = np.arange(n)
    z1 = np.exp(2j * np.pi * l / n)
    z2 = np.exp(1j * alpha) * np.exp(2j * np.pi * ((l + m0) % n) / n)
    res = oracle.align_pair(z1, z2)
    T = res["T_all"]
    assert np.ptp(T) <= 1e-13 * T.max()
    m = res["m"]
    # R(theta) beta2(l + m) = beta1(l): clockwise by alpha + 2 pi (m + m0) / n
    expect = oracle.wrap_angle(alpha + 2 * np.pi * (m + m0) / n)
    assert abs(oracle.wrap_angle(res["theta_paper"] - expect)) < 1e-12
    assert res["E"] < 1e-26


@pytest.mark.parametrize("n", [60, 300, 301])
def test_three_fold_curve_through_align_pair(n):
    """r = 1 + 0.3 cos 3t against a restarted copy: three start indices tie
    mathematically (exactly when 3 | n, up to rounding of the node values
    otherwise the copy is only near them).  With 3 | n the returned index is
    one of the three, its energy vanishes and its angle is a multiple of
    2 pi / 3."""
    m0 = 17
    l = np.arange(n)
    t = 2 * np.pi * l / n
    z1 = (1 + 0.3 * np.cos(3 * t)) * np.exp(1j * t)
    z2 = np.roll(z1, -m0)
    res = oracle.align_pair(z1, z2)
    T = res["T_all"]
    top = np.argsort(-T)[:3]
    if n % 3 == 0:
        ties = sorted(((-m0 + j * n // 3) % n) for j in range(3))
        assert sorted(top) == ties
        assert res["m"] in ties
        assert np.ptp(T[ties]) <= 1e-13 * T.max()
        k = ((res["m"] + m0) % n) // (n // 3)
        assert abs(oracle.wrap_angle(res["theta_paper"] - 2 * np.pi * k / 3)) < 1e-12
        assert res["E"] < 1e-26
    else:
        # without 3 | n only the restart index itself matches exactly
        assert res["m"] == (-m0) % n
        assert res["E"] < 1e-26


def test_batch_matches_pairs():
    rng = np.random.default_rng(5)
    B, n = 6, 40
    z1 = np.stack([random_curve(rng, n) for _ in range(B)]).astype(np.complex64)
    z2 = np.stack([random_curve(rng, n) for _ in range(B)]).astype(np.complex64)
    m, th, e, t, used = oracle.align_batch_f32(z1, z2, nthreads=2)
    assert used >= 1
    for p in range(B):
        r = oracle.align_pair(z1[p].astype(np.complex128), z2[p].astype(np.complex128))
        assert m[p] == r["m"] and th[p] == r["theta_paper"] and e[p] == r["E"]


def test_check_batch_reads_the_slow_method_at_a_given_shift():
    """check_batch_f32 (the benchmark's full-batch accuracy leg) returns the
    slow method's optimum and, at any correlation shift s, the value, angle
    and energy of start index (n - s) mod n, the same numbers the per-pair
    functions give; T2 is the largest value over the other indices."""
    rng = np.random.default_rng(11)
    B, n = 5, 48
    z1 = np.stack([random_curve(rng, n) for _ in range(B)]).astype(np.complex64)
    z2 = np.stack([random_curve(rng, n) for _ in range(B)]).astype(np.complex64)
    shifts = np.array([0, 1, 17, n - 1, 30], dtype=np.int32)
    r = oracle.check_batch_f32(z1, z2, shifts, nthreads=2)
    for p in range(B):
        a, b = z1[p].astype(np.complex128), z2[p].astype(np.complex128)
        ref = oracle.align_pair(a, b)
        assert r["m"][p] == ref["m"] and r["E"][p] == ref["E"] and r["T"][p] == ref["T"]
        T = ref["T_all"]
        assert r["T2"][p] == np.max(np.delete(T, ref["m"]))
        ma = (n - int(shifts[p])) % n
        assert r["T_at"][p] == T[ma] and r["theta_paper_at"][p] == ref["theta_all"][ma]
        assert r["E_at"][p] == oracle.energy(a, b, ma, ref["theta_all"][ma])


def test_resampling_needed_for_nonuniform_sampling():
    """Analogue of the hippopede illustration: a copy of a curve sampled with
    nodes crowded in one part aligns badly as raw nodes and well after
    uniform arc-length resampling of both lists."""
    n = 256
    t1 = np.arange(n) * 2 * np.pi / n
    u = np.arange(n) / n
    t2 = 2 * np.pi * (u + 0.12 * np.sin(2 * np.pi * u) / (2 * np.pi) * 2)   # crowded nodes
    shape = lambda t: (1 + 0.3 * np.cos(2 * t)) * np.exp(1j * t)        # noqa: E731
    raw1 = shape(t1)
    raw2 = np.exp(1j * np.pi / 3) * shape(t2 + 0.25 * 2 * np.pi)
    to_xy = lambda z: np.stack([z.real, z.imag], 1)                      # noqa: E731
    L1 = np.sum(np.abs(np.diff(np.append(raw1, raw1[0]))))
    L2 = np.sum(np.abs(np.diff(np.append(raw2, raw2[0]))))
    bad = oracle.align_pair((raw1 - raw1.mean()) / L1, (raw2 - raw2.mean()) / L2)
    r1, _ = rr.resample(to_xy(raw1), n)
    r2, _ = rr.resample(to_xy(raw2), n)
    good = oracle.align_pair(r1, r2)
    assert good["E"] < 1e-4 * good["n1"]
    assert bad["E"] > 100 * good["E"]


def test_generator_template_truth():
    """single_pair's template is the raw curve rotated by theta0 and shifted by
    s0 vertices; aligning the raw vertex lists (no resampling) recovers both."""
    raw1, raw2, truth = curves.single_pair(4242, n_raw=200, sigma=0.0)
    z1 = raw1[:, 0].astype(np.float64) + 1j * raw1[:, 1]
    z2 = raw2[:, 0].astype(np.float64) + 1j * raw2[:, 1]
    res = oracle.align_pair(z1 - z1.mean(), z2 - z2.mean())
    s, th = oracle.to_library_convention(res["m"], res["theta_paper"], 200)
    assert s == truth["s0"]
    assert abs(oracle.wrap_angle(th + truth["theta0"])) < 1e-6


@pytest.mark.parametrize("n,m0,theta0", [(64, 16, 1.0), (200, 150, -2.2), (257, 1, 0.4)])
def test_initializer_reproduces_curve_in_matrix_form(n, m0, theta0):
    """Hand-off of section 3 in the matrix notation of section 2: with
    beta2 built so that R(theta0) beta2(t + t0) = beta1(t) at t0 = m0 / n,
    the oracle returns exactly that t0 and R, and applying them to the nodes
    of beta2 reproduces beta1."""
    rng = np.random.default_rng(n + m0)
    z1 = random_curve(rng, n)
    b1 = np.stack([z1.real, z1.imag], 1)
    R0 = R_paper(theta0)
    b2 = np.empty_like(b1)
    for l in range(n):
        b2[(l + m0) % n] = R0.T @ b1[l]
    t0, R, res = oracle.initializer(b1, b2)
    assert t0 == m0 / n
    assert np.max(np.abs(R - R0)) < 1e-12
    back = np.stack([R @ b2[(l + round(t0 * n)) % n] for l in range(n)])
    assert np.max(np.abs(back - b1)) < 1e-12
    assert res["E"] < 1e-24


@pytest.mark.parametrize("n", [11, 97, 250, 1009])
def test_zero_padded_correlation_identity(n):
    """The identity behind sizes with a prime factor above 7: for M >= 2n,
    a = z1 then zeros, b = (z2, z2) then zeros, the length-M transform of
    conj(A) B holds M conj(C(s)) at index M - n + s, with C the correlation
    whose magnitude and angle the slow method reports at every shift."""
    rng = np.random.default_rng(n)
    z1, z2 = random_curve(rng, n), random_curve(rng, n)
    M = 2 * n + 3                              # any length >= 2n works
    a = np.zeros(M, complex)
    b = np.zeros(M, complex)
    a[:n] = z1
    b[:2 * n] = np.concatenate([z2, z2])
    D = np.fft.fft(np.conj(np.fft.fft(a)) * np.fft.fft(b))
    C = np.conj(D[M - n:]) / M
    T, th, _, _ = oracle.per_shift_arrays(z1, z2)
    assert np.max(np.abs(np.abs(C) - T)) < 1e-12 * np.max(T)
    assert np.max(np.abs(oracle.wrap_angle(np.angle(C) - th))) < 1e-9
