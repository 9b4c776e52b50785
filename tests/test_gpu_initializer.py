"""GPU parity of to_initializer (the elastic-solver hand-off of section 3)
against the FP64 oracle's (t0, R(theta)) in the paper's notation."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_R = 1e-5        # FP32 path: |d theta| <= 1e-5 rad bounds every entry of R


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


def check_pair(z1, z2, t0, R, rec):
    """Oracle optimum outside near-ties; otherwise consistency with the record."""
    n = len(z1)
    t0o, Ro, res = oracle.initializer(z1.astype(np.complex128), z2.astype(np.complex128))
    T = np.sort(res["T_all"])
    gap = (T[-1] - T[-2]) / T[-1]
    # always: the conversion of the record itself
    assert t0 == ((n - int(rec["shift"])) % n) / n
    assert np.max(np.abs(R - oracle.R_paper(-float(rec["theta"])))) < 1e-12
    if gap >= 1e-6:
        assert t0 == t0o
        assert np.max(np.abs(R - Ro)) <= TOL_R
        return 0
    return 1


@pytest.mark.parametrize("n", [128, 1024])
def test_uniform_batch(ca, n):
    B = 61
    z1, z2 = inputs.batch(400 + n, B, n)
    note(f"align_batch + to_initializer B={B} n={n}")
    res = ca.align_batch(gpu(z1), gpu(z2), rescore="window")
    t0, R = ca.to_initializer(res, n=n)
    torch.cuda.synchronize()
    rec, t0, R = ca.to_numpy(res), t0.cpu().numpy(), R.cpu().numpy()
    near = sum(check_pair(z1[i], z2[i], t0[i], R[i], rec[i]) for i in range(B))
    note(f"n={n}: near-ties {near}/{B}")


def test_ragged_batch_with_flagged_pairs(ca):
    d = inputs.ragged(402, 40, 64, 1024)
    off = d["off"].copy()
    z1, z2 = d["z1"].copy(), d["z2"].copy()
    z2[off[3]:off[4]] = 0                       # degenerate pair: flagged, identity hand-off
    note(f"ragged align_batch + to_initializer B={len(off) - 1}")
    offs = gpu(off)
    res = ca.align_batch(gpu(z1), gpu(z2), offsets=offs)
    t0, R = ca.to_initializer(res, offsets=offs)
    torch.cuda.synchronize()
    rec, t0, R = ca.to_numpy(res), t0.cpu().numpy(), R.cpu().numpy()
    assert rec["flags"][3] & ca.FLAG_DEGENERATE
    assert t0[3] == 0.0 and np.array_equal(R[3], np.eye(2))
    for i in range(len(off) - 1):
        if i == 3:
            continue
        check_pair(z1[off[i]:off[i + 1]], z2[off[i]:off[i + 1]], t0[i], R[i], rec[i])


def test_empty_and_argument_errors(ca):
    res = ca.empty_results(0, "cuda:0")
    t0, R = ca.to_initializer(res, n=64)
    assert t0.shape == (0,) and R.shape == (0, 2, 2)
    with pytest.raises(ValueError):
        ca.to_initializer(ca.empty_results(4, "cuda:0"))
    with pytest.raises(ca.CurveAlignError):
        ca.to_initializer(ca.empty_results(4, "cuda:0"), n=0)
