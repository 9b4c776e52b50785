"""GPU parity of the SRV step of section 3 against the FP64 oracle.

Stage 1: srv_transform (FP32) against oracle.srv_ref.srv on the same FP32
nodes.  Stage 2: the (t0, R) step of Eq. (dist2-energy), align_batch on
(q2*, q1) + to_initializer, on SRV values computed by the oracle (rounded to
FP32), against the oracle's minimiser.  End to end (GPU SRV into GPU
alignment) is reported and only the clear shifts are gated.
"""
import numpy as np
import pytest

import acceptance as acc
import inputs
from oracle import srv_ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_Q = 1e-6       # |q_gpu - q| <= TOL_Q |q|: a few FP32 roundings per value


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


def check_q(qg, z):
    q = srv_ref.srv(z.astype(np.complex128))
    err = np.abs(qg.astype(np.complex128) - q)
    assert np.all(err <= TOL_Q * np.abs(q) + 1e-30), float(np.max(err / np.maximum(np.abs(q), 1e-30)))
    return float(np.max(err / np.maximum(np.abs(q), 1e-30)))


@pytest.mark.parametrize("n", [64, 1000, 1024])
def test_srv_uniform(ca, n):
    z1, _ = inputs.batch(600 + n, 37, n)
    note(f"srv_transform uniform count=37 n={n}")
    q = ca.srv_transform(gpu(z1)).cpu().numpy()
    worst = max(check_q(q[i], z1[i]) for i in range(len(z1)))
    note(f"n={n}: max relative error {worst:.3g}")


def test_srv_ragged_and_degenerate_segments(ca):
    rng = np.random.default_rng(5)
    sizes = [2, 3, 5, 1000, 4097, 77]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    z = (rng.normal(size=off[-1]) + 1j * rng.normal(size=off[-1])).astype(np.complex64)
    z[off[5] + 10] = z[off[5] + 9]              # zero-length segment 9 of curve 5
    note("srv_transform ragged")
    q = ca.srv_transform(gpu(z), gpu(off)).cpu().numpy()
    for c in range(len(sizes)):
        check_q(q[off[c]:off[c + 1]], z[off[c]:off[c + 1]])
    assert q[off[5] + 9] == 0


def test_srv_perimeter_identity(ca):
    """(1/n) sum |q|^2 equals the polygon's length."""
    z1, _ = inputs.batch(610, 8, 512)
    q = ca.srv_transform(gpu(z1)).cpu().numpy().astype(np.complex128)
    for i in range(8):
        z = z1[i].astype(np.complex128)
        per = np.sum(np.abs(np.roll(z, -1) - z))
        assert abs(np.mean(np.abs(q[i]) ** 2) - per) < 1e-6 * per


@pytest.mark.parametrize("n", [128, 1024])
def test_step_on_oracle_srv(ca, n):
    B = 33
    z1, z2 = inputs.batch(620 + n, B, n)
    q1 = np.stack([srv_ref.srv(z.astype(np.complex128)) for z in z1]).astype(np.complex64)
    q2 = np.stack([srv_ref.srv(z.astype(np.complex128)) for z in z2]).astype(np.complex64)
    note(f"SRV step B={B} n={n}: align_batch(q2, q1) + to_initializer")
    res = ca.align_batch(gpu(q2), gpu(q1), rescore="window")
    t0, R = ca.to_initializer(res, n=n)
    torch.cuda.synchronize()
    rec, t0, R = ca.to_numpy(res), t0.cpu().numpy(), R.cpu().numpy()
    st = acc.check_batch(rec, q2, q1)
    note(f"n={n}: {st}")
    for i in range(B):
        a, b = q1[i].astype(np.complex128), q2[i].astype(np.complex128)
        t0o, Ro, Eo = srv_ref.srv_step(a, b)
        if acc.oracle_pair(b, a)["gap"] >= 1e-6:
            assert t0[i] == t0o
            assert np.max(np.abs(R[i] - Ro)) <= 1e-5


def test_step_end_to_end(ca):
    n, B = 1024, 33
    z1, z2 = inputs.batch(630, B, n)
    qg1 = ca.srv_transform(gpu(z1))
    qg2 = ca.srv_transform(gpu(z2))
    rec = ca.to_numpy(ca.align_batch(qg2, qg1, rescore="window"))
    clear, agree = 0, 0
    for i in range(B):
        q1 = srv_ref.srv(z1[i].astype(np.complex128))
        q2 = srv_ref.srv(z2[i].astype(np.complex128))
        orc = acc.oracle_pair(q2, q1)
        if orc["gap"] >= 1e-4:
            clear += 1
            agree += int(rec["shift"][i]) == orc["s0"]
    note(f"end to end: {agree}/{clear} clear shifts agree")
    assert agree == clear
