"""Per-pair acceptance rule of the alignment results against the FP64 oracle.

Shift: exact when the oracle's top-2 relative gap g = (T(s0) - T2) / T(s0)
is at least 1e-6; at a near-tie (g < 1e-6) any shift with
T(shift) >= (1 - 1e-6) T(s0) is accepted (several answers are correct there).
theta: compared with the oracle's optimal angle at the shift the library
chose, modulo 2 pi.  e0: |e0 - E(shift)| <= rtol E(shift) + 1e-12 (n1 + n2),
with E(shift) the energy of Eq. disc-energy summed directly by the oracle.
"""
from __future__ import annotations

import numpy as np

import oracle

NEAR_TIE = 1e-6


def oracle_pair(z1: np.ndarray, z2: np.ndarray):
    """Oracle arrays for one pair (FP64, library convention, indexed by shift)."""
    n = len(z1)
    T, th, m, thp = oracle.per_shift_arrays(z1, z2)
    s0 = int(np.argmax(T))
    T2 = np.max(np.delete(T, s0)) if n > 1 else 0.0
    g = (T[s0] - T2) / T[s0] if T[s0] > 0 else 0.0
    return {"T": T, "theta": th, "m": m, "theta_paper": thp, "s0": s0, "gap": g,
            "n1": oracle.sqnorm(z1), "n2": oracle.sqnorm(z2)}


def check_pair(res, z1, z2, theta_tol=1e-5, e_rtol=1e-5, orc=None):
    """Return a dict of error figures; raise AssertionError when outside the rule."""
    orc = orc or oracle_pair(z1, z2)
    n = len(z1)
    s = int(res["shift"])
    assert 0 <= s < n, f"shift {s} out of range"
    T = orc["T"]
    s0 = orc["s0"]
    near = orc["gap"] < NEAR_TIE
    if near:
        assert T[s] >= (1 - NEAR_TIE) * T[s0], f"near-tie shift {s} below tolerance (s0 {s0})"
    else:
        assert s == s0, f"shift {s} != oracle {s0} (gap {orc['gap']:.3g})"
    dth = float(oracle.wrap_angle(float(res["theta"]) - orc["theta"][s]))
    assert abs(dth) <= theta_tol, f"theta error {dth:.3g} at shift {s}"
    E = oracle.energy(z1, z2, int(orc["m"][s]), float(orc["theta_paper"][s]))
    de = abs(float(res["e0"]) - E)
    tol = e_rtol * E + 1e-12 * (orc["n1"] + orc["n2"])
    assert de <= tol, f"e0 {float(res['e0'])!r} vs {E!r} (err {de:.3g} > {tol:.3g})"
    return {"near_tie": near, "exact_shift": s == s0, "theta_err": abs(dth),
            "e0_rel_err": de / max(E, 1e-300), "gap": orc["gap"]}


def check_batch(res_np, z1s, z2s, **kw):
    stats = [check_pair(res_np[i], z1s[i], z2s[i], **kw) for i in range(len(res_np))]
    return {"pairs": len(stats),
            "near_ties": int(sum(s["near_tie"] for s in stats)),
            "shift_mismatch": int(sum(not s["exact_shift"] for s in stats)),
            "theta_err_max": float(max(s["theta_err"] for s in stats)),
            "e0_rel_err_max": float(max(s["e0_rel_err"] for s in stats))}
