"""GPU parity of align_all_pairs (per-curve spectra + upper-triangle tiles)."""
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


def upper_index(i, j, m):
    return i * m - i * (i + 1) // 2 + (j - i - 1)


@pytest.mark.parametrize("M,n", [(70, 512), (37, 128), (9, 1024), (2, 64), (3, 256)])
def test_all_pairs_parity(ca, M, n):
    g = inputs.gallery(100 + n, M, n)
    note(f"align_all_pairs M={M} n={n}")
    res = ca.to_numpy(ca.align_all_pairs(torch.from_numpy(g).cuda()))
    torch.cuda.synchronize()
    assert len(res) == M * (M - 1) // 2
    for i in range(M):
        for j in range(i + 1, M):
            acc.check_pair(res[upper_index(i, j, M)], g[i], g[j])


def test_all_pairs_matches_batch_bits(ca):
    """The same pair through align_all_pairs and align_batch gives the same
    shift, flags, theta and gap bit for bit; e0 and err_est agree to rounding
    (the batch kernel sums curve 2's norm in its re-scoring pass, i.e. in the
    shifted order, the spectra kernel in node order)."""
    M, n = 40, 512
    g = inputs.gallery(5, M, n)
    gt = torch.from_numpy(g).cuda()
    note("all pairs vs batch bits")
    allp = ca.to_numpy(ca.align_all_pairs(gt))
    ii, jj = np.triu_indices(M, 1)
    bat = ca.to_numpy(ca.align_batch(gt[torch.from_numpy(ii).cuda()].contiguous(),
                                     gt[torch.from_numpy(jj).cuda()].contiguous()))
    for f in ("shift", "flags", "theta", "gap"):
        assert np.array_equal(allp[f], bat[f]), f
    assert np.all(np.abs(allp["e0"] - bat["e0"]) <= 1e-12 * np.abs(bat["e0"]) + 1e-15)
    assert np.all(np.abs(allp["err_est"] - bat["err_est"]) <= 1e-6 * np.abs(bat["err_est"]))


def test_all_pairs_full_size_sampled(ca):
    """M = 4096 curves at n = 512 (8,386,560 pairs) in the benchmark's launch
    configuration; sampled pairs checked one by one against the oracle."""
    from synth import curves
    M, n = 4096, 512
    gt = torch.view_as_complex(curves.gallery_torch(17781, M, n, "cuda")).contiguous()
    g = gt.cpu().numpy()
    note("align_all_pairs full size")
    out = ca.align_all_pairs(gt)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    rows = []
    for _ in range(40):
        i, j = sorted(rng.choice(M, 2, replace=False))
        rows.append((i, j, upper_index(i, j, M)))
    idx = torch.tensor([k for _, _, k in rows], device="cuda")
    res = ca.to_numpy(out[idx])
    for r, (i, j, _) in zip(res, rows):
        acc.check_pair(r, g[i], g[j])
    fl = ca.unpack(out)["flags"]
    assert int(((fl & (ca.FLAG_DEGENERATE | ca.FLAG_NONFINITE)) != 0).sum().item()) == 0
