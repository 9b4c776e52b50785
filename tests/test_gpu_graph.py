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


@pytest.mark.parametrize("kind", ["ragged", "allpairs", "resample"])
def test_graph_survives_workspace_growth(ca, kind):
    """A graph captured on a fresh context, then a larger eager call that
    outgrows the context's workspace (size-class lists, spectra and norms,
    resampler curve list), then replays: the replays still match the eager
    result of the captured call, because the outgrown buffers are kept until
    the context is destroyed."""
    print(f"[gpu] graph after workspace growth {kind}", flush=True)
    ctx = ca.Context(0)
    if kind == "ragged":
        small, big = inputs.ragged(21, 10), inputs.ragged(22, 300)
        z1, z2, off = (torch.from_numpy(small[k]).cuda() for k in ("z1", "z2", "off"))
        out = ca.empty_results(10, "cuda")
        fn = lambda: ca.align_batch(z1, z2, offsets=off, out=out, ctx=ctx)  # noqa: E731
        b1, b2, boff = (torch.from_numpy(big[k]).cuda() for k in ("z1", "z2", "off"))
        grow = lambda: ca.align_batch(b1, b2, offsets=boff, ctx=ctx)  # noqa: E731
    elif kind == "allpairs":
        g_small = torch.from_numpy(inputs.gallery(23, 20, 256)).cuda()
        g_big = torch.from_numpy(inputs.gallery(24, 90, 256)).cuda()
        out = ca.empty_results(20 * 19 // 2, "cuda")
        fn = lambda: ca.align_all_pairs(g_small, out=out, ctx=ctx)  # noqa: E731
        grow = lambda: ca.align_all_pairs(g_big, ctx=ctx)  # noqa: E731
    else:
        from synth import curves
        d = curves.ragged_pairs(25, 8)
        raw = torch.view_as_complex(torch.from_numpy(d["raw1"]).cuda()).contiguous()
        roff = torch.from_numpy(d["off1"]).cuda()
        n = torch.from_numpy(d["n"].astype(np.int64)).cuda()
        ooff = torch.zeros(9, dtype=torch.int64, device="cuda")
        ooff[1:] = torch.cumsum(n, 0)
        out = torch.empty(int(ooff[-1].item()), dtype=torch.complex64, device="cuda")
        fn = lambda: ca.resample_arclength(raw, roff, ooff, out=out, ctx=ctx)  # noqa: E731
        d2 = curves.ragged_pairs(26, 400)
        raw2 = torch.view_as_complex(torch.from_numpy(d2["raw1"]).cuda()).contiguous()
        roff2 = torch.from_numpy(d2["off1"]).cuda()
        n2 = torch.from_numpy(d2["n"].astype(np.int64)).cuda()
        ooff2 = torch.zeros(401, dtype=torch.int64, device="cuda")
        ooff2[1:] = torch.cumsum(n2, 0)
        grow = lambda: ca.resample_arclength(raw2, roff2, ooff2, ctx=ctx)  # noqa: E731
    fn()
    torch.cuda.synchronize()
    eager = out.clone()
    g = capture(fn)
    grow()
    torch.cuda.synchronize()
    for r in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {r} after growth differs"
    del g
    torch.cuda.synchronize()
    ctx.close()


def _ragged_raw(seed, B):
    from synth import curves
    d = curves.ragged_pairs(seed, B)
    raw = torch.view_as_complex(torch.from_numpy(np.concatenate([d["raw1"], d["raw2"]])).cuda()).contiguous()
    off2 = d["off2"][1:] + d["off1"][-1]
    roff = torch.from_numpy(np.concatenate([d["off1"], off2])).cuda()
    n = np.concatenate([d["n"], d["n"]]).astype(np.int64)
    ooff = torch.zeros(2 * B + 1, dtype=torch.int64, device="cuda")
    ooff[1:] = torch.cumsum(torch.from_numpy(n).cuda(), 0)
    return raw, roff, ooff


def test_library_graph_ragged_pipeline(ca):
    """ca_graph_begin/end record GPU resampling of a ragged batch's raw
    polygons and its alignment as one library-owned graph; replays with eager
    work in between reproduce the eager nodes and records bit for bit."""
    print("[gpu] library graph: resample + ragged alignment", flush=True)
    B = 40
    raw, roff, ooff = _ragged_raw(31, B)
    total = int(ooff[-1].item())
    half = int(ooff[B].item())
    nodes = torch.empty(total, dtype=torch.complex64, device="cuda")
    off = ooff[: B + 1].contiguous()
    out = ca.empty_results(B, "cuda")

    def step(stream=None):
        ca.resample_arclength(raw, roff, ooff, out=nodes, with_norms=False, with_flags=False, stream=stream)
        ca.align_batch(nodes[:half], nodes[half:], offsets=off, out=out, stream=stream)

    step()
    torch.cuda.synchronize()
    want_nodes, want = nodes.clone(), out.clone()
    g = ca.capture(step)
    for r in range(4):
        nodes.zero_()
        out.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(nodes, want_nodes) and torch.equal(out, want), f"replay {r} differs"
        del junk
    g.close()


def test_library_graph_all_pairs_noalloc(ca):
    """The allocation-free all-pairs entry point recorded in a library graph
    (the use it is meant for) replays to the eager records of align_all_pairs."""
    print("[gpu] library graph: align_all_pairs_noalloc", flush=True)
    g_in = torch.from_numpy(inputs.gallery(32, 50, 512)).cuda()
    want = ca.align_all_pairs(g_in)
    out = torch.zeros_like(want)
    torch.cuda.synchronize()
    g = ca.capture(lambda st: ca.align_all_pairs_noalloc(g_in, out, stream=st))
    for r in range(3):
        out.zero_()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(out, want), f"replay {r} differs"
    g.close()


def test_library_graph_failed_call_discards_capture(ca):
    """A call that fails during a capture (here an unsupported n) makes
    ca_graph_end fail, and the context captures normally afterwards."""
    z = torch.zeros(4, 5000, dtype=torch.complex64, device="cuda")
    with pytest.raises(ca.CurveAlignError) as e:
        ca.capture(lambda st: ca.align_batch(z, z, stream=st))
    assert e.value.status in (ca.ERR_UNSUPPORTED_N, ca.ERR_INVALID_ARG)
    a, b = inputs.batch(33, 8, 256)
    z1, z2 = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    want = ca.align_batch(z1, z2)
    out = torch.zeros_like(want)
    torch.cuda.synchronize()
    g = ca.capture(lambda st: ca.align_batch(z1, z2, out=out, stream=st))
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    g.close()
