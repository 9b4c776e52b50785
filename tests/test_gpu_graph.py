"""Graph capture: the alignment and resampling launches recorded in a HIP
graph and replayed several times, with eager work in between, reproduce the
eager results bit for bit."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_17779_amd as m
    m.default_context(0)
    return m


def capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


@pytest.mark.parametrize("kind", ["team", "block", "bf16", "allpairs", "ragged", "ragged_any", "srv", "handoff"])
def test_graph_replays_match_eager(ca, kind):
    print(f"[gpu] graph replay {kind}", flush=True)
    if kind == "ragged_any":
        # padded sizes, a size above the limit (flagged by the binning kernel)
        rng = np.random.default_rng(12)
        sizes = [97, 5000, 64, 1009, 11, 256]
        offn = np.zeros(len(sizes) + 1, dtype=np.int64)
        offn[1:] = np.cumsum(sizes)
        a = (rng.normal(size=offn[-1]) + 1j * rng.normal(size=offn[-1])).astype(np.complex64)
        b = (rng.normal(size=offn[-1]) + 1j * rng.normal(size=offn[-1])).astype(np.complex64)
        z1, z2, off = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), torch.from_numpy(offn).cuda()
        out = ca.empty_results(len(sizes), "cuda")
        fn = lambda: ca.align_batch(z1, z2, offsets=off, out=out)  # noqa: E731
    elif kind == "srv":
        a, _ = inputs.batch(13, 9, 512)
        z = torch.from_numpy(a).cuda()
        q = torch.empty_like(z)
        out = q.view(torch.uint8)
        fn = lambda: ca.srv_transform(z, out=q)  # noqa: E731
    elif kind == "handoff":
        a, b = inputs.batch(14, 21, 256)
        rec = ca.align_batch(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        t0 = torch.empty(21, dtype=torch.float64, device="cuda")
        rot = torch.empty(21, 2, 2, dtype=torch.float64, device="cuda")
        out = torch.empty(21 * 40, dtype=torch.uint8, device="cuda")

        def fn():
            t, r = ca.to_initializer(rec, n=256)
            t0.copy_(t)
            rot.copy_(r)
            out.copy_(torch.cat([t0.view(torch.uint8), rot.view(torch.uint8).reshape(-1)]))
    elif kind == "allpairs":
        g_in = torch.from_numpy(inputs.gallery(8, 24, 256)).cuda()
        out = ca.empty_results(24 * 23 // 2, "cuda")
        fn = lambda: ca.align_all_pairs(g_in, out=out)          # noqa: E731
    elif kind == "ragged":
        d = inputs.ragged(9, 12)
        z1, z2 = torch.from_numpy(d["z1"]).cuda(), torch.from_numpy(d["z2"]).cuda()
        off = torch.from_numpy(d["off"]).cuda()
        out = ca.empty_results(12, "cuda")
        fn = lambda: ca.align_batch(z1, z2, offsets=off, out=out)  # noqa: E731
    else:
        n = {"team": 1024, "block": 1000, "bf16": 128}[kind]
        a, b = inputs.batch(10 + n, 37, n)
        z1, z2 = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        out = ca.empty_results(37, "cuda")
        prec = "split_bf16" if kind == "bf16" else "fp32"
        fn = lambda: ca.align_batch(z1, z2, precision=prec, out=out)  # noqa: E731
    fn()
    torch.cuda.synchronize()
    eager = out.clone()
    g = capture(fn)
    for r in range(4):
        out.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()           # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {r} differs"
        del junk


def test_graph_resample(ca):
    from synth import curves
    d = curves.ragged_pairs(11, 20)
    raw = torch.view_as_complex(torch.from_numpy(d["raw1"]).cuda()).contiguous()
    roff = torch.from_numpy(d["off1"]).cuda()
    n = torch.from_numpy(d["n"].astype(np.int64)).cuda()
    ooff = torch.zeros(21, dtype=torch.int64, device="cuda")
    ooff[1:] = torch.cumsum(n, 0)
    out = torch.empty(int(ooff[-1].item()), dtype=torch.complex64, device="cuda")
    fn = lambda: ca.resample_arclength(raw, roff, ooff, out=out, with_norms=False, with_flags=False)  # noqa: E731
    fn()
    torch.cuda.synchronize()
    eager = out.clone()
    g = capture(fn)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
