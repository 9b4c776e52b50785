"""GPU parity of the split-BF16 MFMA paths (n = 128 and n = 1024) against the
FP64 oracle.

Tolerances: theta within 1e-3 rad (split-BF16), e0 within 1e-5 relative
(e0 uses the FP64 C at the chosen shift), shift exact except at near-ties.
At n = 1024 the shift comes from an FP64 search around the vertex of a
parabola fitted to the split-BF16 |C|^2, and from FP64 searches started at
any other shift within the error window (curves with rotational symmetry).
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


def test_bf16_parity(ca):
    B = 203                                   # odd: the last pair group holds one pair
    z1, z2 = inputs.batch(128128, B, 128)
    note("split_bf16 align_batch B=203 n=128")
    res = ca.to_numpy(ca.align_batch(torch.from_numpy(z1).cuda(), torch.from_numpy(z2).cuda(),
                                     precision="split_bf16"))
    st = acc.check_batch(res, z1, z2, theta_tol=1e-3)
    note(f"split_bf16: {st}")
    assert st["shift_mismatch"] == 0
    assert np.all((res["flags"] & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE)) == 0)
    note(f"windows above the cap: {int(((res['flags'] & ca.FLAG_CAND_CAPPED) != 0).sum())}")
    # the window rule re-scores in FP64, so the chosen C(s*) and e0 are exact to FP64
    fp32 = ca.to_numpy(ca.align_batch(torch.from_numpy(z1).cuda(), torch.from_numpy(z2).cuda(),
                                      rescore="window"))
    assert np.array_equal(res["shift"], fp32["shift"])
    assert np.allclose(res["e0"], fp32["e0"], rtol=1e-12, atol=1e-16)


def test_bf16_theta_fp64_and_protocol(ca):
    z1 = inputs.batch(9, 1, 128)[0][0].astype(np.complex128)
    z2 = np.exp(1j * np.pi / 3) * np.roll(z1, -32)
    a = np.stack([z1, z1, z2]).astype(np.complex64)
    b = np.stack([z2, z1, z1]).astype(np.complex64)
    res = ca.to_numpy(ca.align_batch(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(),
                                     precision="split_bf16", theta_fp64=True))
    assert list(res["shift"]) == [32, 0, 96]
    acc.check_batch(res, a, b, theta_tol=1e-6)


def test_bf16_rejects_other_sizes(ca):
    for n in (256, 512, 2048):
        z = torch.zeros(4, n, dtype=torch.complex64, device="cuda")
        with pytest.raises(ca.CurveAlignError) as e:
            ca.align_batch(z, z, precision="split_bf16")
        assert e.value.status == ca.ERR_UNSUPPORTED_N


def test_bf16_1024_parity(ca):
    B = 301                                   # not a multiple of the four pairs per block
    z1, z2 = inputs.batch(1024, B, 1024)
    note("split_bf16 align_batch B=301 n=1024")
    res = ca.to_numpy(ca.align_batch(torch.from_numpy(z1).cuda(), torch.from_numpy(z2).cuda(),
                                     precision="split_bf16"))
    st = acc.check_batch(res, z1, z2, theta_tol=1e-3)
    note(f"split_bf16 n=1024: {st}")
    assert st["shift_mismatch"] == 0
    assert np.all((res["flags"] & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE | ca.FLAG_CAND_CAPPED)) == 0)
    assert np.all(res["flags"] & ca.FLAG_RESCORED)
    assert st["theta_err_max"] < 1e-4


def test_bf16_1024_exact_copies_protocol_and_flags(ca):
    z1 = inputs.batch(11, 1, 1024)[0][0].astype(np.complex128)
    z2 = np.exp(1j * np.pi / 3) * np.roll(z1, -256)         # start 0 -> 0.25, rotation pi/3
    zero = np.zeros(1024)
    nanz = z1.copy()
    nanz[17] = np.nan
    a = np.stack([z1, z1, z2, zero, nanz]).astype(np.complex64)
    b = np.stack([z2, z1, z1, z1, z1]).astype(np.complex64)
    res = ca.to_numpy(ca.align_batch(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(),
                                     precision="split_bf16", theta_fp64=True))
    assert list(res["shift"][:3]) == [256, 0, 768]
    acc.check_batch(res[:3], a[:3], b[:3], theta_tol=1e-6)
    assert res["flags"][3] & ca.FLAG_DEGENERATE
    assert res["flags"][4] & ca.FLAG_NONFINITE
    assert np.isnan(res["e0"][4])


@pytest.mark.parametrize("n", [128, 1024])
@pytest.mark.parametrize("shape", ["circle", "three_fold", "four_fold"])
def test_bf16_symmetric_curves(ca, shape, n):
    """Symmetric shapes: at n = 128 the pruned window keeps far peaks of
    nearly equal height (three- and four-fold) and handles a window wider
    than the candidate cap (the circle); at n = 1024 the separate-peak and
    segment searches."""
    import test_gpu_ties as ties
    z1, z2 = ties.pairs(shape, n, np.complex64)
    note(f"split_bf16 ties {shape} n={n}")
    res = ca.to_numpy(ca.align_batch(torch.from_numpy(z1).cuda(), torch.from_numpy(z2).cuda(),
                                     precision="split_bf16"))
    for b in range(len(res)):
        a64, b64 = z1[b].astype(np.complex128), z2[b].astype(np.complex128)
        orc = acc.oracle_pair(a64, b64)
        assert orc["T"][int(res["shift"][b])] >= (1 - acc.NEAR_TIE) * orc["T"].max()
        acc.check_pair(res[b], a64, b64, theta_tol=1e-3, orc=orc)
        assert res["flags"][b] & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE) == 0


def test_bf16_1024_full_size_sampled(ca):
    """65,536 pairs at n = 1024 (the batch workload, resampled on the GPU) in
    the benchmark's launch configuration; sampled pairs against the oracle."""
    from synth import curves
    B, n = 65536, 1024
    r1, r2 = curves.batch_pairs_torch(17780, B, n, "cuda")
    raw = torch.view_as_complex(torch.cat([r1, r2]).reshape(-1, 2)).contiguous()
    roff = torch.arange(0, 2 * B + 1, dtype=torch.int64, device="cuda") * n
    nodes, _, _ = ca.resample_arclength(raw, roff, roff)
    z1, z2 = nodes[: B * n].view(B, n), nodes[B * n:].view(B, n)
    note("split_bf16 n=1024 full size")
    out = ca.align_batch(z1, z2, precision="split_bf16")
    torch.cuda.synchronize()
    idx = np.random.default_rng(5).choice(B, 64, replace=False)
    it = torch.from_numpy(idx).cuda()
    st = acc.check_batch(ca.to_numpy(out[it]), z1[it].cpu().numpy(), z2[it].cpu().numpy(), theta_tol=1e-3)
    note(f"split_bf16 n=1024 full size sampled: {st}")
    fl = ca.unpack(out)["flags"]
    assert int(((fl & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE)) != 0).sum().item()) == 0
    note(f"capped: {int(((fl & ca.FLAG_CAND_CAPPED) != 0).sum().item())}")


def test_bf16_full_size_sampled(ca):
    """1,048,576 pairs at n = 128 in the benchmark's launch configuration."""
    from synth import curves
    B, n = 1 << 20, 128
    r1, r2 = curves.batch_pairs_torch(17783, B, n, "cuda", kmin=8, kmax=8, sigma_max=1e-3)
    z1 = torch.view_as_complex(r1).contiguous()
    z2 = torch.view_as_complex(r2).contiguous()
    note("split_bf16 full size")
    out = ca.align_batch(z1, z2, precision="split_bf16")
    torch.cuda.synchronize()
    idx = np.random.default_rng(3).choice(B, 64, replace=False)
    it = torch.from_numpy(idx).cuda()
    st = acc.check_batch(ca.to_numpy(out[it]), z1[it].cpu().numpy(), z2[it].cpu().numpy(), theta_tol=1e-3)
    note(f"split_bf16 full size sampled: {st}")
    fl = ca.unpack(out)["flags"]
    bad = int(((fl & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE)) != 0).sum().item())
    capped = int(((fl & ca.FLAG_CAND_CAPPED) != 0).sum().item())
    note(f"capped windows: {capped}")
    assert bad == 0
