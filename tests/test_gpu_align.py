"""GPU parity of the alignment entry points against the FP64 oracle.

Every case calls the HIP library through its C ABI (via the ctypes binding)
on seeded inputs that the oracle resampled, and checks each pair with the
acceptance rule in acceptance.py.
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


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def run_batch(ca, z1, z2, **kw):
    note(f"align_batch B={z1.shape[0]} n={z1.shape[1]} {kw}")
    res = ca.align_batch(gpu(z1), gpu(z2), **kw)
    torch.cuda.synchronize()
    return ca.to_numpy(res)


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("rescore", ["top2", "window"])
def test_team_engine_parity(ca, n, rescore):
    B = 203 if n <= 256 else 77            # several teams/waves and a ragged tail
    z1, z2 = inputs.batch(11 + n, B, n)
    res = run_batch(ca, z1, z2, rescore=rescore)
    st = acc.check_batch(res, z1, z2)
    note(f"n={n} {rescore}: {st}")
    assert np.all((res["flags"] & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE)) == 0)
    if rescore == "window":
        # the FP64 window leaves a shift mismatch only at exact ties
        assert st["shift_mismatch"] == 0


@pytest.mark.parametrize("n", [2, 3, 12, 300, 315, 1000, 2048, 2187, 4096])
def test_block_engine_parity(ca, n):
    B = 24 if n >= 2048 else 40
    if n < 16:
        rng = np.random.default_rng(n)
        z1 = (rng.normal(size=(B, n)) + 1j * rng.normal(size=(B, n))).astype(np.complex64)
        z2 = (rng.normal(size=(B, n)) + 1j * rng.normal(size=(B, n))).astype(np.complex64)
    else:
        z1, z2 = inputs.batch(500 + n, B, n)
    for rescore in ("top2", "window"):
        res = run_batch(ca, z1, z2, rescore=rescore)
        st = acc.check_batch(res, z1, z2)
        note(f"n={n} {rescore}: {st}")


@pytest.mark.parametrize("n", [11, 13, 97, 143, 1009, 2053, 4093])
def test_padded_transform_parity(ca, n):
    """n with a prime factor above 7: zero-padded correlation at M >= 2n."""
    B = 16 if n >= 2048 else 40
    if n < 16:
        rng = np.random.default_rng(n)
        z1 = (rng.normal(size=(B, n)) + 1j * rng.normal(size=(B, n))).astype(np.complex64)
        z2 = (rng.normal(size=(B, n)) + 1j * rng.normal(size=(B, n))).astype(np.complex64)
    else:
        z1, z2 = inputs.batch(700 + n, B, n)
    for rescore in ("top2", "window"):
        res = run_batch(ca, z1, z2, rescore=rescore)
        st = acc.check_batch(res, z1, z2)
        note(f"padded n={n} {rescore}: {st}")
        if rescore == "window":
            assert st["shift_mismatch"] == 0


@pytest.mark.parametrize("n", [11, 97, 1009, 2039])
def test_padded_transform_fp64(ca, n):
    z1, z2 = inputs.batch(800 + n, 12, max(n, 16)) if n >= 16 else (None, None)
    if z1 is None:
        rng = np.random.default_rng(n)
        z1 = rng.normal(size=(12, n)) + 1j * rng.normal(size=(12, n))
        z2 = rng.normal(size=(12, n)) + 1j * rng.normal(size=(12, n))
    z1, z2 = z1.astype(np.complex128), z2.astype(np.complex128)
    note(f"align_batch fp64 padded n={n}")
    res = ca.to_numpy(ca.align_batch(gpu(z1), gpu(z2), precision="fp64"))
    acc.check_batch(res, z1, z2, theta_tol=1e-10, e_rtol=1e-10)


def test_fp64_single_pair(ca):
    """The one-pair workload in FP64 (n = 256)."""
    z1, z2, truth = inputs.single(17779, 256)
    note("align_pair fp64 n=256")
    res = ca.align_pair(gpu(z1), gpu(z2), precision="fp64")
    torch.cuda.synchronize()
    r = ca.to_numpy(res)[0]
    acc.check_pair(r, z1, z2, theta_tol=1e-10, e_rtol=1e-10)
    # the template is the same curve restarted s0 vertices later and rotated by theta0
    assert abs(int(r["shift"]) - truth["s0"]) <= 2
    assert abs(float(acc.oracle.wrap_angle(float(r["theta"]) + truth["theta0"]))) < 0.05


def test_fp64_batch_block_sizes(ca):
    # one size per FP64 class: <= 512, <= 1024, <= 2048 (1500), <= 4096 (3000, 4096)
    for n in (128, 360, 1024, 1500, 3000, 4096):
        z1, z2 = inputs.batch(900 + n, 16 if n <= 1024 else 8, n)
        note(f"align_batch fp64 n={n}")
        res = ca.to_numpy(ca.align_batch(gpu(z1.astype(np.complex128)), gpu(z2.astype(np.complex128)),
                                         precision="fp64"))
        acc.check_batch(res, z1.astype(np.complex128), z2.astype(np.complex128),
                        theta_tol=1e-10, e_rtol=1e-10)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [300, 263, 1000])
def test_small_batch_kernels_agree(ca, precision, n):
    """A batch of at most one pair per CU runs size classes 0 and 1 with 256
    threads per pair; a larger batch with 64 or 128.  The two run the same
    butterflies; only the order of the FP64 norm and re-scoring sums
    differs.  n = 300 (class 0), 263 (zero-padded to 540: class 1), 1000
    (class 1)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    big = cus + 37
    z1, z2 = inputs.batch(960 + n, big, n)
    if precision == "fp64":
        z1, z2 = z1.astype(np.complex128), z2.astype(np.complex128)
    note(f"small vs large batch {precision} n={n}: {cus} and {big} pairs")
    small = ca.to_numpy(ca.align_batch(gpu(z1[:cus]), gpu(z2[:cus]), precision=precision))
    large = ca.to_numpy(ca.align_batch(gpu(z1), gpu(z2), precision=precision))[:cus]
    torch.cuda.synchronize()
    assert np.array_equal(small["shift"], large["shift"])
    assert np.array_equal(small["flags"], large["flags"])
    th = 1e-6 if precision == "fp32" else 1e-12
    assert np.all(np.abs(np.angle(np.exp(1j * (small["theta"] - large["theta"])))) <= th)
    assert np.all(np.abs(small["e0"] - large["e0"]) <= 1e-12 * np.abs(large["e0"]) + 1e-15)
    tol = 1e-10 if precision == "fp64" else 1e-5
    acc.check_batch(small[:16], z1[:16], z2[:16], theta_tol=tol, e_rtol=tol)
    # ragged: the same pairs, alone and inside a larger ragged batch
    off = np.arange(0, big + 1, dtype=np.int64) * n
    rs = ca.to_numpy(ca.align_batch(gpu(z1[:cus].reshape(-1)), gpu(z2[:cus].reshape(-1)),
                                    offsets=gpu(off[:cus + 1]), precision=precision))
    rl = ca.to_numpy(ca.align_batch(gpu(z1.reshape(-1)), gpu(z2.reshape(-1)), offsets=gpu(off),
                                    precision=precision))[:cus]
    torch.cuda.synchronize()
    assert np.array_equal(rs["shift"], rl["shift"]) and np.array_equal(rs["flags"], rl["flags"])
    assert np.array_equal(rs["shift"], small["shift"])


def test_ragged_batch(ca):
    d = inputs.ragged(31, 48)
    note(f"ragged align_batch B=48 n in [{d['n'].min()}, {d['n'].max()}]")
    res = ca.to_numpy(ca.align_batch(gpu(d["z1"]), gpu(d["z2"]), offsets=gpu(d["off"])))
    torch.cuda.synchronize()
    off = d["off"]
    for b in range(48):
        acc.check_pair(res[b], d["z1"][off[b]:off[b + 1]], d["z2"][off[b]:off[b + 1]])


def test_ragged_unsupported_sizes_are_flagged(ca):
    rng = np.random.default_rng(3)
    sizes = [64, 11, 1, 5000, 128, 4093]   # 11, 4093: padded; 1: too small; 5000: too large
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    z1 = (rng.normal(size=off[-1]) + 1j * rng.normal(size=off[-1])).astype(np.complex64)
    z2 = (rng.normal(size=off[-1]) + 1j * rng.normal(size=off[-1])).astype(np.complex64)
    note("ragged unsupported sizes")
    res = ca.to_numpy(ca.align_batch(gpu(z1), gpu(z2), offsets=gpu(off)))
    bad = (res["flags"] & ca.FLAG_UNSUPPORTED_N) != 0
    assert list(bad) == [False, False, True, True, False, False]
    for b in (0, 1, 4, 5):
        acc.check_pair(res[b], z1[off[b]:off[b + 1]], z2[off[b]:off[b + 1]])
    # FP64: a padded transform above 4096 does not fit the block engine's LDS
    note("ragged fp64 sizes")
    r64 = ca.to_numpy(ca.align_batch(gpu(z1.astype(np.complex128)), gpu(z2.astype(np.complex128)),
                                     offsets=gpu(off), precision="fp64"))
    bad = (r64["flags"] & ca.FLAG_UNSUPPORTED_N) != 0
    assert list(bad) == [False, False, True, True, False, True]
    for b in (0, 1, 4):
        acc.check_pair(r64[b], z1[off[b]:off[b + 1]].astype(np.complex128),
                       z2[off[b]:off[b + 1]].astype(np.complex128), theta_tol=1e-10, e_rtol=1e-10)


@pytest.mark.parametrize("n", [64, 256, 1000, 1024])
def test_exact_copy_and_paper_protocol(ca, n):
    """Template = reference restarted at t = 0.25 and rotated by pi/3."""
    z1 = inputs.batch(7, 1, n)[0][0].astype(np.complex128)
    z2 = np.exp(1j * np.pi / 3) * np.roll(z1, -(n // 4))
    a = np.stack([z1, z1]).astype(np.complex64)
    b = np.stack([z2, z1]).astype(np.complex64)
    res = run_batch(ca, a, b)
    assert res["shift"][0] == n // 4 and res["shift"][1] == 0
    assert abs(res["theta"][0] + np.pi / 3) < 1e-5 and abs(res["theta"][1]) < 1e-6
    acc.check_batch(res, a, b)


def test_swap_symmetry(ca):
    z1, z2 = inputs.batch(44, 64, 512)
    r12 = run_batch(ca, z1, z2)
    r21 = run_batch(ca, z2, z1)
    ok = (r12["flags"] & ca.FLAG_NEAR_TIE) == 0
    assert np.all(r21["shift"][ok] == (512 - r12["shift"][ok]) % 512)
    assert np.max(np.abs(acc.oracle.wrap_angle(r12["theta"][ok] + r21["theta"][ok]))) < 2e-5
    assert np.allclose(r12["e0"], r21["e0"], rtol=1e-9, atol=1e-14)


def test_degenerate_and_nonfinite(ca):
    z1, z2 = inputs.batch(45, 4, 256)
    z1 = z1.copy()
    z2 = z2.copy()
    z1[1] = 0
    z2[2, 17] = np.nan
    res = run_batch(ca, z1, z2)
    assert res["flags"][1] & ca.FLAG_DEGENERATE and res["shift"][1] == 0
    assert res["e0"][1] == pytest.approx(acc.oracle.sqnorm(z2[1]), rel=1e-12)
    assert res["flags"][2] & ca.FLAG_NONFINITE and np.isnan(res["e0"][2])
    acc.check_pair(res[0], z1[0], z2[0])
    acc.check_pair(res[3], z1[3], z2[3])


def test_invalid_arguments(ca):
    z = gpu(np.zeros((2, 4097), np.complex64))
    with pytest.raises(ca.CurveAlignError) as e:
        ca.align_batch(z, z)
    assert e.value.status == ca.ERR_UNSUPPORTED_N
    z = gpu(np.zeros((2, 2053), np.complex128))
    with pytest.raises(ca.CurveAlignError) as e:
        ca.align_batch(z, z, precision="fp64")
    assert e.value.status == ca.ERR_UNSUPPORTED_N
    z = gpu(np.zeros((0, 64), np.complex64))
    out = ca.align_batch(z, z)        # empty batch: no-op
    assert out.shape == (0, ca.RESULT_BYTES)
    z = gpu(np.zeros((2, 128), np.complex64))
    with pytest.raises(ValueError):
        ca.align_batch(z, z, precision="fp16")


def test_theta_from_fp64(ca):
    z1, z2 = inputs.batch(46, 64, 1024)
    res = run_batch(ca, z1, z2, theta_fp64=True)
    assert np.all(res["flags"] & ca.FLAG_THETA_FP64)
    acc.check_batch(res, z1, z2, theta_tol=1e-6)


@pytest.mark.parametrize("n", [128, 1024])
@pytest.mark.parametrize("rescore", ["top2", "window"])
def test_team_theta_from_rescored_c(ca, n, rescore):
    """The team kernels take theta as an FP32 arc tangent of the FP64 re-scored
    C at the chosen shift: same shift as the FP64-theta run, angle within FP32
    rounding of the FP64 arc tangent (C's parts rounded to FP32: ~6e-8 rad,
    atan2f's error a few ulps more)."""
    z1, z2 = inputs.batch(48 + n, 64, n)
    a = run_batch(ca, z1, z2, rescore=rescore)
    b = run_batch(ca, z1, z2, rescore=rescore, theta_fp64=True)
    assert np.array_equal(a["shift"], b["shift"])
    assert np.all(b["flags"] & ca.FLAG_THETA_FP64) and not np.any(a["flags"] & ca.FLAG_THETA_FP64)
    d = np.abs(np.angle(np.exp(1j * (a["theta"] - b["theta"]))))
    note(f"n={n} {rescore}: max |theta - theta_fp64| = {d.max():.3g}")
    assert d.max() < 5e-7
    assert np.array_equal(a["e0"], b["e0"])


def test_determinism(ca):
    z1, z2 = inputs.batch(47, 256, 1024)
    a = run_batch(ca, z1, z2)
    b = run_batch(ca, z1, z2)
    assert a.tobytes() == b.tobytes()


def test_full_size_batch_sampled(ca):
    """65,536 pairs at n = 1024 in the benchmark's launch configuration;
    sampled pairs checked against the oracle one by one."""
    from synth import curves
    B, n = 65536, 1024
    note("full-size batch: generating")
    r1, r2 = curves.batch_pairs_torch(17780, B, n, "cuda")
    z1 = torch.view_as_complex(r1).contiguous()
    z2 = torch.view_as_complex(r2).contiguous()
    note("full-size batch: align_batch B=65536 n=1024")
    out = ca.align_batch(z1, z2)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(B, 48, replace=False)
    it = torch.from_numpy(idx).cuda()
    res = ca.to_numpy(out[it])
    st = acc.check_batch(res, z1[it].cpu().numpy(), z2[it].cpu().numpy())
    note(f"full size sampled: {st}")
    fl = ca.unpack(out)["flags"]
    assert int(((fl & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE)) != 0).sum().item()) == 0


@pytest.mark.parametrize("snap", [True, False])
def test_full_size_ragged_sampled(ca, snap):
    """The ragged workload in the benchmark's launch configuration: 100,000
    raw polygon pairs (n log-uniform in [64, 4096]; snap=False keeps every
    integer n, so padded transforms run too) resampled on the GPU, then one
    ragged align_batch; sampled pairs, a third of them from the largest size
    classes, checked against the oracle on the GPU's own nodes."""
    from synth import curves
    B = 100000
    note(f"full-size ragged (snap={snap}): generating")
    d = curves.ragged_pairs_torch(17782, B, "cuda", snap=snap)
    raw = torch.cat([d["raw1"], d["raw2"]])
    roff = torch.cat([d["off1"], d["off2"][1:] + d["off1"][-1]])
    n = d["n"].long()
    ooff = torch.zeros(2 * B + 1, dtype=torch.int64, device="cuda")
    ooff[1:] = torch.cumsum(torch.cat([n, n]), 0)
    note("full-size ragged: resample_arclength")
    nodes, _, _ = ca.resample_arclength(raw, roff, ooff, with_norms=False, with_flags=False)
    off = ooff[: B + 1].contiguous()
    half = int(off[-1].item())
    note("full-size ragged: align_batch with offsets")
    out = ca.align_batch(nodes[:half], nodes[half:], offsets=off)
    torch.cuda.synchronize()
    fl = ca.unpack(out)["flags"]
    assert int(((fl & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE | ca.FLAG_UNSUPPORTED_N)) != 0).sum().item()) == 0
    n_h = n.cpu().numpy()
    rng = np.random.default_rng(5 if snap else 6)
    big = np.flatnonzero(n_h > 2048)
    idx = np.concatenate([rng.choice(B, 20, replace=False), rng.choice(big, 10, replace=False)])
    res = ca.to_numpy(out[torch.from_numpy(idx).cuda()])
    off_h = off.cpu().numpy()
    stats = []
    for r, b in zip(res, idx):
        z1 = nodes[off_h[b]:off_h[b + 1]].cpu().numpy()
        z2 = nodes[half + off_h[b]:half + off_h[b + 1]].cpu().numpy()
        stats.append(acc.check_pair(r, z1, z2))
    note(f"full-size ragged sampled: {len(stats)} pairs, n up to {int(n_h[idx].max())}, "
         f"theta err max {max(s['theta_err'] for s in stats):.3g}, "
         f"e0 rel err max {max(s['e0_rel_err'] for s in stats):.3g}")
