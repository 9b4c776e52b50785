"""FP64 CPU oracle for closed-curve alignment (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check in __graft_entry__ and the CPU-baseline leg of
bench.py may import this package.  It shares no code with the GPU library.

Two parts:
  * align_ref.c     -- the paper's slow method (every start index, optimal
                       rotation per index, Eq. disc-energy), built with gcc
                       into liboracle_align.so and called through ctypes;
  * resample_ref.py -- arc-length resampling in FP64.

Conventions.  The oracle reports in the paper's notation: a start index m
(t0 = m / n, curve 2 read as beta2[(l + m) mod n]) and a clockwise angle
theta_paper (R(theta) = [[cos, sin], [-sin, cos]]).  The GPU library reports
the shift s of the correlation C(s) = sum_n z1[n] conj(z2[n - s]) and the
counter-clockwise angle arg C(s) applied to curve 2.  `to_library_convention`
converts: s = (n - m) mod n, theta = -theta_paper (wrapped to (-pi, pi]).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import resample_ref  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "align_ref.c")
_LIB = os.path.join(_HERE, "liboracle_align.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile align_ref.c with gcc (no fast-math) into liboracle_align.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_shift_scores.argtypes = [dp, dp, ctypes.c_int, dp, dp]
        L.oracle_shift_scores.restype = None
        L.oracle_a_matrix.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.oracle_a_matrix.restype = None
        L.oracle_energy.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.oracle_energy.restype = ctypes.c_double
        L.oracle_sqnorm.argtypes = [dp, ctypes.c_int]
        L.oracle_sqnorm.restype = ctypes.c_double
        L.oracle_best_index.argtypes = [dp, ctypes.c_int]
        L.oracle_best_index.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_align_pair.argtypes = [dp, dp, ctypes.c_int, ip, dp, dp, dp, dp, dp]
        L.oracle_align_pair.restype = None
        L.oracle_align_batch_f32.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_align_batch_f32.restype = ctypes.c_int
        L.oracle_check_batch_f32.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_int, ctypes.c_int] + [ctypes.c_void_p] * 9
        L.oracle_check_batch_f32.restype = ctypes.c_int
        _lib = L
    return _lib


def _as_xy(z) -> np.ndarray:
    """complex array (n,) or real (n, 2) -> contiguous float64 (n, 2)."""
    z = np.asarray(z)
    if np.iscomplexobj(z):
        out = np.empty((z.shape[0], 2), dtype=np.float64)
        out[:, 0] = z.real
        out[:, 1] = z.imag
        return out
    return np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 2)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def shift_scores(z1, z2):
    """(T[m], theta_paper[m]) for every start index m (paper notation)."""
    b1, b2 = _as_xy(z1), _as_xy(z2)
    n = b1.shape[0]
    T = np.empty(n)
    H = np.empty(n)
    lib().oracle_shift_scores(_dp(b1), _dp(b2), n, _dp(T), _dp(H))
    return T, H


def a_matrix(z1, z2, m: int) -> np.ndarray:
    b1, b2 = _as_xy(z1), _as_xy(z2)
    a = np.empty(4)
    lib().oracle_a_matrix(_dp(b1), _dp(b2), b1.shape[0], int(m), _dp(a))
    return a.reshape(2, 2)


def energy(z1, z2, m: int, theta_paper: float) -> float:
    """Eq. disc-energy at start index m and paper-convention angle."""
    b1, b2 = _as_xy(z1), _as_xy(z2)
    return lib().oracle_energy(_dp(b1), _dp(b2), b1.shape[0], int(m), float(theta_paper))


def sqnorm(z) -> float:
    b = _as_xy(z)
    return lib().oracle_sqnorm(_dp(b), b.shape[0])


def align_pair(z1, z2):
    """The slow method on one pair.  Returns a dict in paper notation."""
    b1, b2 = _as_xy(z1), _as_xy(z2)
    n = b1.shape[0]
    T = np.empty(n)
    H = np.empty(n)
    m = ctypes.c_int()
    th, e, t = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().oracle_align_pair(_dp(b1), _dp(b2), n, ctypes.byref(m), ctypes.byref(th),
                            ctypes.byref(e), ctypes.byref(t), _dp(T), _dp(H))
    return {"m": m.value, "theta_paper": th.value, "E": e.value, "T": t.value,
            "T_all": T, "theta_all": H, "n1": sqnorm(b1), "n2": sqnorm(b2)}


def align_batch_f32(z1: np.ndarray, z2: np.ndarray, nthreads: int = 0):
    """Slow method over a batch of complex64 pairs [B, n] (upcast to FP64).

    Returns (m, theta_paper, E, T, threads_used).
    """
    z1 = np.ascontiguousarray(z1, dtype=np.complex64)
    z2 = np.ascontiguousarray(z2, dtype=np.complex64)
    B, n = z1.shape
    m = np.empty(B, dtype=np.int32)
    th = np.empty(B)
    e = np.empty(B)
    t = np.empty(B)
    used = lib().oracle_align_batch_f32(z1.ctypes.data, z2.ctypes.data, B, n, int(nthreads),
                                        m.ctypes.data, th.ctypes.data, e.ctypes.data,
                                        t.ctypes.data)
    return m, th, e, t, used


def check_batch_f32(z1: np.ndarray, z2: np.ndarray, shifts: np.ndarray, nthreads: int = 0):
    """Slow method over a batch of complex64 pairs [B, n], plus each pair read
    at a given correlation shift (start index (n - shift) mod n).

    Returns a dict of arrays: m, theta_paper, E, T (the optimum, paper
    notation), T2 (largest value over the other start indices), and at the
    given shift T_at, theta_paper_at, E_at; plus "threads".
    """
    z1 = np.ascontiguousarray(z1, dtype=np.complex64)
    z2 = np.ascontiguousarray(z2, dtype=np.complex64)
    B, n = z1.shape
    sh = np.ascontiguousarray(shifts, dtype=np.int32)
    assert sh.shape == (B,)
    out = {"m": np.empty(B, dtype=np.int32)}
    for k in ("theta_paper", "E", "T", "T2", "T_at", "theta_paper_at", "E_at"):
        out[k] = np.empty(B)
    used = lib().oracle_check_batch_f32(z1.ctypes.data, z2.ctypes.data, B, n, int(nthreads), sh.ctypes.data,
                                        out["m"].ctypes.data, out["theta_paper"].ctypes.data,
                                        out["E"].ctypes.data, out["T"].ctypes.data, out["T2"].ctypes.data,
                                        out["T_at"].ctypes.data, out["theta_paper_at"].ctypes.data,
                                        out["E_at"].ctypes.data)
    out["threads"] = used
    return out


def wrap_angle(a):
    """Wrap into (-pi, pi]."""
    a = np.asarray(a, dtype=np.float64)
    w = np.mod(a + np.pi, 2.0 * np.pi) - np.pi
    return np.where(w == -np.pi, np.pi, w)


def to_library_convention(m, theta_paper, n: int):
    """(start index m, clockwise angle) -> (correlation shift s, CCW angle)."""
    return (n - np.asarray(m)) % n, wrap_angle(-np.asarray(theta_paper))


def per_shift_arrays(z1, z2):
    """T, theta (library convention) and E indexed by the library shift s."""
    b1, b2 = _as_xy(z1), _as_xy(z2)
    n = b1.shape[0]
    T, H = shift_scores(b1, b2)
    s = np.arange(n)
    m = (n - s) % n
    return T[m], wrap_angle(-H[m]), m, H[m]


def R_paper(theta_paper: float) -> np.ndarray:
    """R(theta) of section 2: [[cos, sin], [-sin, cos]] (clockwise by theta)."""
    c, s = np.cos(theta_paper), np.sin(theta_paper)
    return np.array([[c, s], [-s, c]])


def initializer(z1, z2):
    """The rigid optimum handed to an elastic solver (section 3): the start
    parameter t0 = m / n at which curve 2 is read and R(theta_paper), the
    slow method's minimiser of Eq. disc-energy.  Returns (t0, R, align_pair dict)."""
    res = align_pair(z1, z2)
    n = _as_xy(z1).shape[0]
    return res["m"] / n, R_paper(res["theta_paper"]), res

