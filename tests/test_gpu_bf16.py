"""GPU parity of the split-BF16 MFMA path (n = 128) against the FP64 oracle.

Tolerances: theta within 1e-3 rad (split-BF16), e0 within 1e-5 relative
(e0 uses the FP64 C at the chosen shift), shift exact except at near-ties.
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
    z = torch.zeros(4, 256, dtype=torch.complex64, device="cuda")
    with pytest.raises(ca.CurveAlignError) as e:
        ca.align_batch(z, z, precision="split_bf16")
    assert e.value.status == ca.ERR_UNSUPPORTED_N


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
