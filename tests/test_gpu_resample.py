"""GPU parity of resample_arclength against the FP64 oracle resampler."""
import numpy as np
import pytest

from oracle import resample_ref as rr
from synth import curves

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# Node tolerance: FP32 chord lengths, spline solve and evaluation on curves of
# unit length; the positions carry a few FP32 ulps of the raw coordinates
# (|raw| ~ 1, perimeter ~ 6.5), i.e. ~1e-7 after scaling by 1/L.
TOL_POS = 2e-6


@pytest.fixture(scope="module")
def ca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_17779_amd as m
    m.default_context(0)
    return m


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def run(ca, polys, ns, mode):
    raw = np.concatenate([p[:, 0] + 1j * p[:, 1] for p in polys]).astype(np.complex64)
    roff = np.zeros(len(polys) + 1, np.int64)
    roff[1:] = np.cumsum([len(p) for p in polys])
    ooff = np.zeros(len(polys) + 1, np.int64)
    ooff[1:] = np.cumsum(ns)
    note(f"resample {len(polys)} curves mode={mode}")
    out, norms, flags = ca.resample_arclength(torch.from_numpy(raw).cuda(), torch.from_numpy(roff).cuda(),
                                              torch.from_numpy(ooff).cuda(), mode=mode)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ooff, norms.cpu().numpy(), flags.cpu().numpy()


@pytest.mark.parametrize("mode", ["spline", "linear"])
def test_resample_parity(ca, mode):
    d = curves.ragged_pairs(77, 40, 64, 4096)
    polys = [d["raw1"][d["off1"][b]:d["off1"][b + 1]] for b in range(40)]
    polys += [d["raw2"][d["off2"][b]:d["off2"][b + 1]] for b in range(40)]
    ns = np.concatenate([d["n"], d["n"]])
    out, ooff, norms, flags = run(ca, polys, ns, mode)
    m = rr.SPLINE if mode == "spline" else rr.LINEAR
    worst = 0.0
    for c, p in enumerate(polys):
        z, info = rr.resample(p.astype(np.float64), int(ns[c]), m)
        g = out[ooff[c]:ooff[c + 1]]
        err = np.max(np.abs(g - z))
        worst = max(worst, err)
        assert err <= TOL_POS, f"curve {c}: node error {err:.3g}"
        assert abs(norms[c] - np.mean(np.abs(g.astype(np.complex128)) ** 2)) < 1e-12
        assert flags[c] == 0
    note(f"resample {mode}: worst node error {worst:.3g}")


def test_resample_small_and_worked_example(ca):
    sq = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    tri = np.array([[0, 0], [3, 0], [3, 4]], np.float32)
    polys = [sq, sq, tri, sq * 7 + 2]
    ns = [8, 8, 30, 16]
    for mode in ("spline", "linear"):
        out, ooff, norms, flags = run(ca, polys, ns, mode)
        m = rr.SPLINE if mode == "spline" else rr.LINEAR
        for c, p in enumerate(polys):
            z, _ = rr.resample(p.astype(np.float64), ns[c], m)
            assert np.max(np.abs(out[ooff[c]:ooff[c + 1]] - z)) < 1e-6


def test_resample_cleaning_and_degenerate(ca):
    rng = np.random.default_rng(5)
    ang = np.sort(rng.uniform(0, 2 * np.pi, 50))
    P = np.stack([np.cos(ang), np.sin(ang)], 1).astype(np.float32)
    dup = np.vstack([P[:10], P[9:10], P[9:10], P[10:], P[:1], P[:1]])
    line = np.array([[0, 0], [1, 1], [1, 1], [0, 0]], np.float32)       # 2 distinct points
    point = np.array([[2, 2]] * 6, np.float32)
    nanp = P.copy()
    nanp[3, 0] = np.nan
    polys = [P, dup, line, point, nanp]
    ns = [64, 64, 16, 16, 16]
    out, ooff, norms, flags = run(ca, polys, ns, "spline")
    assert np.max(np.abs(out[0:64] - out[64:128])) < 1e-6
    assert flags[0] == 0 and flags[1] == 0
    assert flags[2] & 8 and flags[3] & 8 and flags[4] & 16
    assert np.all(out[128:] == 0)


def test_resample_full_size_sampled(ca):
    """The ragged workload's resampling launch (100,000 pairs, 200,000 curves)
    with sampled curves checked against the oracle."""
    B = 100000
    note("full-size resample: generating")
    d = curves.ragged_pairs_torch(17782, B, "cuda")
    raw = torch.cat([d["raw1"], d["raw2"]])
    roff = torch.cat([d["off1"], d["off2"][1:] + d["off1"][-1]])
    ns = torch.cat([d["n"], d["n"]]).long()
    ooff = torch.zeros(2 * B + 1, dtype=torch.int64, device="cuda")
    ooff[1:] = torch.cumsum(ns, 0)
    note("resample full size")
    out, _, flags = ca.resample_arclength(raw, roff, ooff)
    torch.cuda.synchronize()
    assert int((flags != 0).sum().item()) == 0
    roff_h, ooff_h, ns_h = roff.cpu().numpy(), ooff.cpu().numpy(), ns.cpu().numpy()
    worst = 0.0
    for c in np.random.default_rng(2).choice(2 * B, 40, replace=False):
        p = raw[roff_h[c]:roff_h[c + 1]].cpu().numpy()
        z, _ = rr.resample(np.stack([p.real, p.imag], 1).astype(np.float64), int(ns_h[c]))
        g = out[ooff_h[c]:ooff_h[c + 1]].cpu().numpy()
        err = np.max(np.abs(g - z))
        worst = max(worst, err)
        assert err <= TOL_POS
    note(f"full-size resample: worst sampled node error {worst:.3g}")


def test_clockwise_flag(ca):
    """CA_FLAG_CLOCKWISE follows the sign of the oracle's signed area, on the
    fast kernel and on the general one (a curve with repeated vertices), for
    curves far from the origin too; reversing a polygon reverses its nodes'
    orientation and sets the flag."""
    d = curves.ragged_pairs(78, 12, 64, 1024)
    polys = [d["raw1"][d["off1"][b]:d["off1"][b + 1]] for b in range(12)]
    polys = polys + [p[::-1].copy() for p in polys]
    far = polys[0] + np.float32([300.0, -200.0])
    polys += [far, far[::-1].copy()]
    dup = np.vstack([polys[1][:5], polys[1][4:5], polys[1][5:]])          # general kernel
    polys += [dup, dup[::-1].copy()]
    ns = [128] * len(polys)
    out, ooff, norms, flags = run(ca, polys, ns, "spline")
    for c, p in enumerate(polys):
        area = rr.resample(p.astype(np.float64), 128)[1]["area"]
        want = ca.FLAG_CLOCKWISE if area < 0 else 0
        assert flags[c] == want, (c, area, flags[c])
    assert sum(int(f) == ca.FLAG_CLOCKWISE for f in flags) == len(polys) // 2


def test_dense_tiles_and_mixed_node_placement(ca):
    """Upsampled curves (more nodes than raw vertices) over several tiles, and
    a curve whose first tile of knots holds few nodes per knot while its second
    holds hundreds: both node-placement paths inside one curve, against the
    oracle."""
    t = np.linspace(0.0, 2 * np.pi, 700, endpoint=False)
    up = np.stack([np.cos(t) * (1 + 0.2 * np.cos(3 * t)), np.sin(t) * (1 + 0.2 * np.cos(3 * t))], 1)
    dense = np.linspace(0.0, 0.6, 520, endpoint=False)             # 520 knots on a short arc
    sparse = np.linspace(0.6, 2 * np.pi, 40, endpoint=False)       # 40 knots on the rest
    tt = np.concatenate([dense, sparse])
    mixed = np.stack([np.cos(tt) * (1 + 0.1 * np.sin(2 * tt)), np.sin(tt) * (1 + 0.1 * np.sin(2 * tt))], 1)
    polys = [up.astype(np.float32), mixed.astype(np.float32), (mixed[::-1] * 3 + 1).astype(np.float32)]
    ns = [4000, 3000, 2048]
    for mode in ("spline", "linear"):
        out, ooff, norms, flags = run(ca, polys, ns, mode)
        m = rr.SPLINE if mode == "spline" else rr.LINEAR
        for c, p in enumerate(polys):
            z, info = rr.resample(p.astype(np.float64), ns[c], m)
            err = np.max(np.abs(out[ooff[c]:ooff[c + 1]] - z))
            note(f"dense/mixed curve {c} {mode}: node error {err:.3g}")
            assert err <= TOL_POS
            assert flags[c] == (ca.FLAG_CLOCKWISE if info["area"] < 0 else 0)


@pytest.mark.parametrize("mode", ["spline", "linear"])
def test_vertex_cap(ca, mode):
    """Raw curves of exactly CA_RESAMPLE_MAX_RAW vertices are resampled (the
    wave-per-curve kernel, and the general kernel when a duplicate vertex has
    to be dropped); one vertex more gives CA_FLAG_UNSUPPORTED_N and zero
    nodes."""
    cap = ca.RESAMPLE_MAX_RAW
    rng = np.random.default_rng(cap)
    n = 1000

    def ellipse(m):
        t = np.sort(rng.uniform(0, 2 * np.pi, m))
        return np.stack([1.3 * np.cos(t), 0.7 * np.sin(t)], -1).astype(np.float32)

    full = ellipse(cap)
    dup = full.copy()
    dup[500] = dup[499]                    # a consecutive duplicate, dropped by cleaning
    over = ellipse(cap + 1)
    polys = [full, dup, over]
    out, ooff, norms, flags = run(ca, polys, [n, n, n], mode)
    m = rr.SPLINE if mode == "spline" else rr.LINEAR
    for c in (0, 1):
        assert flags[c] & ca.FLAG_UNSUPPORTED_N == 0
        ref, _ = rr.resample(polys[c].astype(np.float64), n, m)
        err = np.abs(out[ooff[c]:ooff[c + 1]] - ref).max()
        note(f"cap {mode} curve {c}: max |dz| {err:.3g}")
        assert err <= TOL_POS
    assert flags[2] & ca.FLAG_UNSUPPORTED_N
    assert np.all(out[ooff[2]:ooff[3]] == 0)
