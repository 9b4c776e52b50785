"""Launch tuning on the GPU: ca_autotune installs one of its candidates,
choices survive a save/load round trip, and no choice changes what is
computed -- grid and tile choices give bit-identical records, radix schedules
give records that pass the oracle's acceptance rule (FP32 and FP64).

Tuning runs on contexts of its own, so the default context that the other
GPU tests share keeps its choices.
"""
import numpy as np
import pytest

import acceptance as acc
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


@pytest.fixture
def ctx(ca):
    c = ca.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def smooth7(m):
    for p in (2, 3, 5, 7):
        while m % p == 0:
            m //= p
    return m == 1


def transform_size(n):
    if smooth7(n):
        return n
    m = 2 * n
    while not smooth7(m):
        m += 1
    return m


@pytest.mark.parametrize("knob,key,allowed", [
    ("team_grid", 256, {(1,), (2,), (4,), (0,)}),
    ("team_grid", 1024, {(1,), (2,), (4,), (0,)}),
    ("allpairs_cols", 128, {(2,), (4,), (8,), (16,), (32,), (64,)}),
    ("block_grid", 1, {(1,), (2,), (4,), (0,)}),
    ("block_grid", 4, {(1,), (2,), (4,), (0,)}),
    ("block_threads", 3, {(256,), (512,)}),
    ("block_threads", 4, {(256,), (512,), (1024,)}),
])
def test_autotune_installs_a_candidate(ca, ctx, knob, key, allowed):
    note(f"autotune {knob} key={key}")
    ms = ca.autotune(knob, key, ctx=ctx)
    got = tuple(ca.tune_get(knob, key, ctx=ctx))
    note(f"{knob}[{key}] -> {got} at {ms:.4f} ms")
    assert ms > 0.0
    assert got in allowed


@pytest.mark.parametrize("M", [2048, 3000, 4096, 8192, 210])
def test_autotune_radix_schedule(ca, ctx, M):
    note(f"autotune block_plan M={M}")
    ms = ca.autotune("block_plan", M, ctx=ctx)
    r = ca.tune_get("block_plan", M, ctx=ctx)
    note(f"block_plan[{M}] -> {r} at {ms:.4f} ms")
    assert ms > 0.0
    assert int(np.prod(r)) == M and set(r) <= ({2, 3, 4, 5, 7, 8, 16} if M > 2048 else {2, 3, 4, 5, 7, 8})


def test_autotune_rejects_unused_transform_size(ca, ctx):
    # 7-smooth but above the zero-padded size of every n <= 4096 that maps near it
    used = {transform_size(n) for n in range(2049, 4097) if not smooth7(n)}
    bad = [m for m in range(4097, 8193) if smooth7(m) and m not in used][:1]
    if not bad:
        pytest.skip("every 7-smooth size in (4096, 8192] is used")
    with pytest.raises(ca.CurveAlignError) as ei:
        ca.autotune("block_plan", bad[0], ctx=ctx)
    assert ei.value.status == ca.ERR_UNSUPPORTED_N


def test_grid_and_tile_choices_are_bit_identical(ca, ctx):
    z1, z2 = inputs.batch(700, 300, 256)
    g1, g2 = gpu(z1), gpu(z2)
    base = ca.align_batch(g1, g2, ctx=ctx).cpu()
    for g in (2, 4, 8, 0):
        ca.tune_set("team_grid", 256, g, ctx=ctx)
        note(f"team_grid={g}")
        assert torch.equal(ca.align_batch(g1, g2, ctx=ctx).cpu(), base), g
    gal = gpu(inputs.gallery(701, 150, 128))
    ref = ca.align_all_pairs(gal, ctx=ctx).cpu()
    for cols in (1, 2, 8, 16, 32, 128, 256):
        ca.tune_set("allpairs_cols", 128, cols, ctx=ctx)
        note(f"allpairs_cols={cols}")
        assert torch.equal(ca.align_all_pairs(gal, ctx=ctx).cpu(), ref), cols
    d = inputs.ragged(702, 60, 64, 4096)
    r1, r2, off = gpu(d["z1"]), gpu(d["z2"]), gpu(d["off"])
    ref = ca.align_batch(r1, r2, offsets=off, ctx=ctx).cpu()
    for g in (2, 4, 0):
        for cls in range(5):
            ca.tune_set("block_grid", cls, g, ctx=ctx)
        note(f"block_grid={g} (all classes)")
        assert torch.equal(ca.align_batch(r1, r2, offsets=off, ctx=ctx).cpu(), ref), g


# (n, radix schedules of its transform size M); each product is M
PLANS = [
    (2000, [[8, 2, 5, 5, 5], [5, 5, 5, 8, 2], [4, 4, 5, 5, 5], [2, 8, 5, 5, 5]]),   # M = 2000
    (1031, [[4, 3, 5, 5, 7], [7, 5, 5, 3, 4], [2, 2, 3, 5, 5, 7]]),                  # M = 2100 (padded)
    (512, [[8, 8, 8], [4, 4, 4, 8], [2, 4, 4, 4, 4]]),                                # M = 512
]


@pytest.mark.parametrize("n,plans", PLANS)
def test_radix_schedules_pass_acceptance(ca, ctx, n, plans):
    M = transform_size(n)
    for r in plans:
        assert int(np.prod(r)) == M
    B = 24
    z1, z2 = inputs.batch(710 + n, B, n)
    g1, g2 = gpu(z1), gpu(z2)
    z1d, z2d = z1.astype(np.complex128), z2.astype(np.complex128)
    g1d, g2d = gpu(z1d), gpu(z2d)
    off = gpu(np.arange(B + 1, dtype=np.int64) * n)          # ragged form: always the block engine
    f1, f2 = g1.reshape(-1), g2.reshape(-1)
    for r in plans:
        ca.tune_set("block_plan", M, r, ctx=ctx)
        assert ca.tune_get("block_plan", M, ctx=ctx) == r
        note(f"n={n} M={M} plan {r}")
        rec = ca.to_numpy(ca.align_batch(f1, f2, offsets=off, ctx=ctx))
        st = acc.check_batch(rec, z1, z2)
        rec64 = ca.to_numpy(ca.align_batch(g1d, g2d, precision="fp64", ctx=ctx))
        st64 = acc.check_batch(rec64, z1d, z2d, theta_tol=1e-10, e_rtol=1e-10)
        note(f"  fp32 {st}\n  fp64 {st64}")


# radix 16 (transform sizes above 2048): n = 4096 in FP32 and FP64, and the
# zero-padded n = 4093 (M = 8192, FP32 only)
R16 = [
    (4096, [[16, 16, 16], [16, 16, 4, 4], [4, 16, 16, 4], [16, 8, 8, 4]], True),
    (3072, [[16, 16, 4, 3], [3, 16, 16, 4], [3, 4, 16, 16]], True),
    (4093, [[16, 16, 16, 2], [2, 16, 16, 16], [8, 16, 16, 4]], False),
]


@pytest.mark.parametrize("n,plans,fp64", R16)
def test_radix16_schedules_pass_acceptance(ca, ctx, n, plans, fp64):
    M = transform_size(n)
    B = 16
    z1, z2 = inputs.batch(760 + n % 97, B, n)
    g1, g2 = gpu(z1), gpu(z2)
    off = gpu(np.arange(B + 1, dtype=np.int64) * n)
    f1, f2 = g1.reshape(-1), g2.reshape(-1)
    z1d, z2d = z1.astype(np.complex128), z2.astype(np.complex128)
    g1d, g2d = gpu(z1d), gpu(z2d)
    for r in plans:
        assert int(np.prod(r)) == M
        ca.tune_set("block_plan", M, r, ctx=ctx)
        assert ca.tune_get("block_plan", M, ctx=ctx) == r
        note(f"n={n} M={M} plan {r}")
        rec = ca.to_numpy(ca.align_batch(f1, f2, offsets=off, ctx=ctx))
        note(f"  fp32 {acc.check_batch(rec, z1, z2)}")
        if fp64:
            rec64 = ca.to_numpy(ca.align_batch(g1d, g2d, precision="fp64", ctx=ctx))
            note(f"  fp64 {acc.check_batch(rec64, z1d, z2d, theta_tol=1e-10, e_rtol=1e-10)}")


def test_fp64_arena_built_after_plan_change(ca, ctx):
    """A schedule installed before the first FP64 call is used when the FP64
    twiddle arena is built."""
    n, r = 1000, [5, 5, 5, 8]
    ca.tune_set("block_plan", n, r, ctx=ctx)
    z1, z2 = inputs.batch(720, 12, n)
    z1d, z2d = z1.astype(np.complex128), z2.astype(np.complex128)
    rec = ca.to_numpy(ca.align_batch(gpu(z1d), gpu(z2d), precision="fp64", ctx=ctx))
    note(f"fp64 after plan change: {acc.check_batch(rec, z1d, z2d, theta_tol=1e-10, e_rtol=1e-10)}")


def test_save_load_round_trip(ca, ctx, tmp_path):
    ca.tune_set("team_grid", 512, 4, ctx=ctx)
    ca.tune_set("allpairs_cols", 64, 32, ctx=ctx)
    ca.tune_set("block_plan", 4096, [4, 4, 4, 8, 8], ctx=ctx)
    ca.tune_set("block_grid", 3, 2, ctx=ctx)
    path = str(tmp_path / "tune.json")
    ca.tune_save(path, ctx=ctx)
    text = open(path).read()
    note(text)
    other = ca.Context(0)
    try:
        assert ca.tune_load(path, ctx=other) == 4
        assert ca.tune_get("team_grid", 512, ctx=other) == [4]
        assert ca.tune_get("allpairs_cols", 64, ctx=other) == [32]
        assert ca.tune_get("block_plan", 4096, ctx=other) == [4, 4, 4, 8, 8]
        assert ca.tune_get("block_grid", 3, ctx=other) == [2]
        assert ca.tune_get("team_grid", 1024, ctx=other) == [1]          # untouched default
        # a file for another device installs nothing
        foreign = tmp_path / "foreign.json"
        foreign.write_text(text.replace('"num_cus": ', '"num_cus": 1'))
        ca.tune_set("team_grid", 512, 2, ctx=other)
        assert ca.tune_load(str(foreign), ctx=other) == 0
        assert ca.tune_get("team_grid", 512, ctx=other) == [2]
        # a malformed file is refused whole
        broken = tmp_path / "broken.json"
        broken.write_text(text.replace('"values": [32]', '"values": [0]'))
        with pytest.raises(ca.CurveAlignError):
            ca.tune_load(str(broken), ctx=other)
        assert ca.tune_get("team_grid", 512, ctx=other) == [2]
        # results with the loaded choices match the defaults
        z1, z2 = inputs.batch(730, 40, 512)
        a = ca.align_batch(gpu(z1), gpu(z2), ctx=other).cpu()
        b = ca.align_batch(gpu(z1), gpu(z2), ctx=ca.default_context(0)).cpu()
        assert torch.equal(a, b)
    finally:
        torch.cuda.synchronize()
        other.close()


def test_thread_counts_agree(ca, ctx):
    """The 256-, 512- and (class 4) 1024-thread kernels of classes 3 and 4
    run the same butterflies; only the order of the FP64 norm and re-scoring
    sums differs."""
    sizes = [2053, 2500, 3001, 3072, 4093, 4096, 2187, 3500]   # padded (class 4) and 7-smooth (class 3)
    z1s, z2s = [], []
    for k, n in enumerate(sizes):
        a, b = inputs.batch(740 + k, 5, n)
        z1s += list(a)
        z2s += list(b)
    offs = np.zeros(len(z1s) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(z) for z in z1s])
    d = {"z1": np.concatenate(z1s), "z2": np.concatenate(z2s), "off": offs}
    r1, r2, off = gpu(d["z1"]), gpu(d["z2"]), gpu(d["off"])
    recs = {}
    for t3, t4 in ((256, 256), (512, 512), (512, 1024)):
        ca.tune_set("block_threads", 3, t3, ctx=ctx)
        ca.tune_set("block_threads", 4, t4, ctx=ctx)
        note(f"block_threads={t3},{t4}")
        recs[t4] = ca.to_numpy(ca.align_batch(r1, r2, offsets=off, ctx=ctx))
    a = recs[256]
    for t in (512, 1024):
        b = recs[t]
        assert np.array_equal(a["shift"], b["shift"]) and np.array_equal(a["flags"], b["flags"])
        # theta is an FP32 arc tangent of the FP64 C, whose partial sums the
        # thread counts add in different orders: equal to FP32 rounding
        assert np.all(np.abs(np.angle(np.exp(1j * (a["theta"] - b["theta"])))) <= 1e-6)
        assert np.all(np.abs(a["e0"] - b["e0"]) <= 1e-12 * np.abs(a["e0"]) + 1e-15)
    for i in range(0, 40, 8):
        lo, hi = d["off"][i], d["off"][i + 1]
        acc.check_pair(b[i], d["z1"][lo:hi], d["z2"][lo:hi])


def test_corrupt_cache_falls_back_to_defaults(ca, tmp_path, monkeypatch):
    """default_context() with an unreadable tuning cache warns and keeps the
    default launch choices (checked on a fresh default context)."""
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    monkeypatch.setenv("CURVEALIGN_TUNE_FILE", str(bad))
    saved = dict(ca._contexts)
    ca._contexts.clear()
    try:
        with pytest.warns(UserWarning):
            c = ca.default_context(0)
        assert c.tune_applied == 0
        assert ca.tune_get("allpairs_cols", 512, ctx=c) == [64]
        z1, z2 = inputs.batch(750, 8, 256)
        rec = ca.to_numpy(ca.align_batch(gpu(z1), gpu(z2), ctx=c))
        acc.check_batch(rec, z1, z2)
    finally:
        torch.cuda.synchronize()
        for k, v in ca._contexts.items():
            v.close()
        ca._contexts.clear()
        ca._contexts.update(saved)


def test_create_with_tune_cache_path(ca, tmp_path):
    """ca_create loads a tuning file given by path (the C caller's route to the
    tuned launches); a broken file fails the call and creates no context; NULL
    keeps the defaults."""
    src = ca.Context(0)
    try:
        ca.tune_set("team_grid", 256, 4, ctx=src)
        ca.tune_set("block_plan", 2048, [4, 8, 8, 8], ctx=src)
        path = str(tmp_path / "tune.json")
        ca.tune_save(path, ctx=src)
    finally:
        src.close()
    loaded = ca.Context(0, tune_file=path)
    plain = ca.Context(0)
    try:
        assert ca.tune_get("team_grid", 256, ctx=loaded) == [4]
        assert ca.tune_get("block_plan", 2048, ctx=loaded) == [4, 8, 8, 8]
        assert ca.tune_get("team_grid", 256, ctx=plain) == [1]
        broken = tmp_path / "broken.json"
        broken.write_text(open(path).read().replace('"values": [4]', '"values": [-3]'))
        with pytest.raises(ca.CurveAlignError) as e:
            ca.Context(0, tune_file=str(broken))
        assert e.value.status == ca.ERR_INVALID_ARG
        with pytest.raises(ca.CurveAlignError):
            ca.Context(0, tune_file=str(tmp_path / "missing.json"))
        # the loaded radix schedule gives results within the acceptance rule
        z1, z2 = inputs.batch(731, 24, 2048)
        res = ca.to_numpy(ca.align_batch(gpu(z1), gpu(z2), ctx=loaded))
        acc.check_batch(res, z1, z2)
    finally:
        torch.cuda.synchronize()
        loaded.close()
        plain.close()
