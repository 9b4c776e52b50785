"""The allocation-free all-pairs entry point, align_all_pairs_noalloc,
against align_all_pairs through the C ABI.

- Two calls in a row on one context, the second with a smaller gallery
  (4096 x 512, the largest the static scratch holds at n = 512, then
  1500 x 256): every record equals the one align_all_pairs writes for the
  same gallery, bit for bit (the two entry points share their kernels), and
  sampled pairs meet the acceptance rule against the FP64 oracle.
- The calls leave the device's free memory unchanged (no workspace grows).
- A gallery whose spectra exceed CA_NOALLOC_SCRATCH_BYTES is refused with
  CA_ERR_TOO_LARGE before anything is enqueued.
"""
import ctypes

import numpy as np
import pytest

import acceptance as acc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_17779_amd as m
    return m


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def upper_index(i, j, m):
    return i * m - i * (i + 1) // 2 + (j - i - 1)


def gallery(seed, M, n):
    from synth import curves
    return torch.view_as_complex(curves.gallery_torch(seed, M, n, "cuda")).contiguous()


def test_noalloc_matches_all_pairs_on_two_calls(ca):
    sizes = [(4096, 512), (1500, 256)]
    assert ca.noalloc_scratch_bytes(4096, 512) <= ca.NOALLOC_SCRATCH_BYTES
    gals = [gallery(17790 + k, M, n) for k, (M, n) in enumerate(sizes)]
    ref_ctx = ca.Context(0)
    ctx = ca.Context(0)
    note("align_all_pairs (reference records) 4096x512 and 1500x256")
    want = [ca.align_all_pairs(g, ctx=ref_ctx) for g in gals]
    outs = [torch.zeros_like(w) for w in want]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    note("align_all_pairs_noalloc 4096x512 then 1500x256")
    for g, o in zip(gals, outs):
        ca.align_all_pairs_noalloc(g, o, ctx=ctx)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (1 << 20), f"device free memory fell by {free0 - free1} bytes"
    rng = np.random.default_rng(7)
    for (M, n), g, w, o in zip(sizes, gals, want, outs):
        assert torch.equal(o, w), f"records differ from align_all_pairs at {M}x{n}"
        gn = g.cpu().numpy()
        rows = [tuple(sorted(rng.choice(M, 2, replace=False))) for _ in range(24)]
        idx = torch.tensor([upper_index(i, j, M) for i, j in rows], device="cuda")
        res = ca.to_numpy(o[idx])
        for r, (i, j) in zip(res, rows):
            acc.check_pair(r, gn[i], gn[j])
    note("noalloc ok")


def test_noalloc_refuses_galleries_above_the_scratch(ca):
    ctx = ca.Context(0)
    buf = torch.zeros(16, dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    L = ca.lib()
    for M, n in [(16384, 128), (4097, 1024), (8193, 256)]:
        assert ca.noalloc_scratch_bytes(M, n) > ca.NOALLOC_SCRATCH_BYTES
        st = L.align_all_pairs_noalloc(ctx.handle, p, M, n, p, None, None)
        assert st == ca.ERR_TOO_LARGE, (M, n, st)
        assert "CA_NOALLOC_SCRATCH_BYTES" in L.ca_last_error().decode()
    # the largest galleries at the limit are accepted by the size check
    for M, n in [(8192, 256), (2048, 1024), (4096, 512)]:
        assert ca.noalloc_scratch_bytes(M, n) <= ca.NOALLOC_SCRATCH_BYTES
    torch.cuda.synchronize()
