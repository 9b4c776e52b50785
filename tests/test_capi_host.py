"""Host-side checks of the C ABI (no GPU needed, no compute calls).

- libcurvealign.so loads and exports every function include/curvealign.h
  declares;
- the record and option layouts and the enum values the header fixes are
  the ones the Python binding marshals (checked with a C program compiled by
  gcc against the header itself);
- ca_n_supported is the predicate the header states (2 <= n <= CA_MAX_N,
  no prime factor above 7), checked by trial division;
- argument errors are reported on the host, before the context is used or
  any device work is enqueued: NULL context, NULL data pointers, negative
  counts, bad option values, unsupported n (the context handle passed in
  those checks is a dummy that the library must not dereference);
- on a machine with no GPU, ca_create reports CA_ERR_NO_DEVICE.
"""
import ctypes
import json
import os
import re
import subprocess

import pytest

import paper_2501_17779_amd as ca
from paper_2501_17779_amd import build as cabuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "curvealign.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ca.LIB_PATH):
        cabuild.build()
    return ca.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_bound_entry_points():
    assert set(declared_functions()) == set(ca.EXPORTED)


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", ca.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in exported, name
        assert getattr(L, name) is not None


_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "curvealign.h"
int main(void) {
    printf("{\"result_size\": %zu, \"result_align\": %zu, \"options_size\": %zu,\n",
           sizeof(ca_result_t), _Alignof(ca_result_t), sizeof(ca_options_t));
    printf("\"offsets\": [%zu, %zu, %zu, %zu, %zu, %zu],\n", offsetof(ca_result_t, shift),
           offsetof(ca_result_t, flags), offsetof(ca_result_t, theta), offsetof(ca_result_t, e0),
           offsetof(ca_result_t, err_est), offsetof(ca_result_t, gap));
    printf("\"status\": [%d, %d, %d, %d, %d, %d, %d, %d],\n", CA_OK, CA_ERR_INVALID_ARG, CA_ERR_UNSUPPORTED_N,
           CA_ERR_HIP, CA_ERR_OOM, CA_ERR_NO_DEVICE, CA_ERR_INTERNAL, CA_ERR_TOO_LARGE);
    printf("\"flags\": [%u, %u, %u, %u, %u, %u, %u, %u],\n", (unsigned)CA_FLAG_NEAR_TIE,
           (unsigned)CA_FLAG_RESCORED, (unsigned)CA_FLAG_CAND_CAPPED, (unsigned)CA_FLAG_DEGENERATE,
           (unsigned)CA_FLAG_NONFINITE, (unsigned)CA_FLAG_THETA_FP64, (unsigned)CA_FLAG_UNSUPPORTED_N,
           (unsigned)CA_FLAG_CLOCKWISE);
    printf("\"prec\": [%d, %d, %d], \"rescore\": [%d, %d], \"resample\": [%d, %d], \"max_n\": %d,\n",
           CA_PREC_FP32, CA_PREC_SPLIT_BF16, CA_PREC_FP64, CA_RESCORE_TOP2, CA_RESCORE_WINDOW,
           CA_RESAMPLE_SPLINE, CA_RESAMPLE_LINEAR, CA_MAX_N);
    printf("\"max_raw\": %d, \"noalloc_bytes\": %lld}\n", CA_RESAMPLE_MAX_RAW,
           (long long)CA_NOALLOC_SCRATCH_BYTES);
    return 0;
}
"""


def test_header_layout_matches_binding(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    h = json.loads(subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout)
    dt = ca.RESULT_DTYPE
    assert h["result_size"] == dt.itemsize == ca.RESULT_BYTES == 32
    assert h["result_align"] == 8
    assert h["offsets"] == [dt.fields[f][1] for f in ("shift", "flags", "theta", "e0", "err_est", "gap")]
    assert h["options_size"] == ctypes.sizeof(ca._Options) == 16
    assert h["status"] == [ca.OK, ca.ERR_INVALID_ARG, ca.ERR_UNSUPPORTED_N, ca.ERR_HIP, ca.ERR_OOM,
                           ca.ERR_NO_DEVICE, ca.ERR_INTERNAL, ca.ERR_TOO_LARGE]
    assert h["noalloc_bytes"] == ca.NOALLOC_SCRATCH_BYTES
    assert h["flags"] == [ca.FLAG_NEAR_TIE, ca.FLAG_RESCORED, ca.FLAG_CAND_CAPPED, ca.FLAG_DEGENERATE,
                          ca.FLAG_NONFINITE, ca.FLAG_THETA_FP64, ca.FLAG_UNSUPPORTED_N, ca.FLAG_CLOCKWISE]
    assert h["prec"] == [ca.PRECISION[k] for k in ("fp32", "split_bf16", "fp64")]
    assert h["rescore"] == [ca.RESCORE[k] for k in ("top2", "window")]
    assert h["resample"] == [ca.RESAMPLE[k] for k in ("spline", "linear")]
    assert h["max_n"] == ca.MAX_N
    assert h["max_raw"] == ca.RESAMPLE_MAX_RAW == 32768


# entry points that compute a step of the paper's method (the others create
# and destroy contexts, report status or tune launches)
COMPUTE_ENTRY_POINTS = ("align_pair", "align_batch", "align_all_pairs", "resample_arclength",
                        "to_initializer", "srv_transform")


def test_every_compute_declaration_cites_the_paper():
    """The comment block in front of each compute entry point names the
    passage that defines its operation: a section of the paper (sections 1-3;
    section 4 is the conclusions), an algorithm or an equation."""
    text = open(HEADER).read()
    for name in COMPUTE_ENTRY_POINTS:
        m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*ca_status_t\s+" + name + r"\s*\(", text, flags=re.S)
        assert m, f"no comment block in front of {name}"
        block = m.group(1)
        assert re.search(r"section [123]\b|Algorithm [12]\b|Eq\. ?\(?[a-z0-9-]+", block), name
        assert not re.search(r"section [4-9]", block), name
    assert not re.search(r"section [4-9]", text)


def _expected_support(n):
    if n < 2 or n > ca.MAX_N:
        return 0
    m = n
    for p in (2, 3, 5, 7):
        while m % p == 0:
            m //= p
    return 1 if m == 1 else 2


def test_n_supported_predicate(L):
    for n in list(range(-3, ca.MAX_N + 40)) + [2 ** 31 - 1, -(2 ** 31)]:
        assert L.ca_n_supported(n) == _expected_support(n), n
    explicit = {1: 0, 2: 1, 11: 2, 840: 1, 2187: 1, 4093: 2, 4095: 2, 4096: 1, 4100: 0}   # 4095 = 3^2 5 7 13
    for n, want in explicit.items():
        assert L.ca_n_supported(n) == want, n


def test_status_strings(L):
    seen = set()
    for st in (ca.OK, ca.ERR_INVALID_ARG, ca.ERR_UNSUPPORTED_N, ca.ERR_HIP, ca.ERR_OOM, ca.ERR_NO_DEVICE,
               ca.ERR_INTERNAL, ca.ERR_TOO_LARGE):
        s = L.ca_status_string(st).decode()
        assert s and s not in seen
        seen.add(s)
    assert L.ca_status_string(12345).decode() == "unknown status"


def _last(L):
    return L.ca_last_error().decode()


def test_null_context_is_rejected_on_host(L):
    dummy = ctypes.c_void_p(16)      # never dereferenced: validation fails first
    assert L.align_pair(None, dummy, dummy, 64, dummy, None, None) == ca.ERR_INVALID_ARG
    assert "NULL" in _last(L)
    assert L.align_batch(None, dummy, dummy, None, 64, 4, dummy, None, None) == ca.ERR_INVALID_ARG
    assert L.align_all_pairs(None, dummy, 8, 64, dummy, None, None) == ca.ERR_INVALID_ARG
    assert L.align_all_pairs_noalloc(None, dummy, 8, 64, dummy, None, None) == ca.ERR_INVALID_ARG
    assert L.resample_arclength(None, dummy, dummy, 4, dummy, dummy, None, None, 0, None) == ca.ERR_INVALID_ARG
    assert L.to_initializer(None, dummy, 64, None, 4, dummy, dummy, None) == ca.ERR_INVALID_ARG
    assert L.srv_transform(None, dummy, None, 64, 4, dummy, None) == ca.ERR_INVALID_ARG
    assert L.ca_create(None, 0, None) == ca.ERR_INVALID_ARG
    assert L.ca_destroy(None) == ca.OK
    h = ctypes.c_void_p()
    assert L.ca_graph_begin(None, ctypes.byref(h)) == ca.ERR_INVALID_ARG
    assert L.ca_graph_begin(dummy, None) == ca.ERR_INVALID_ARG
    assert L.ca_graph_end(None, ctypes.byref(h)) == ca.ERR_INVALID_ARG
    assert L.ca_graph_end(dummy, None) == ca.ERR_INVALID_ARG
    assert L.ca_graph_launch(None, None) == ca.ERR_INVALID_ARG
    assert L.ca_graph_destroy(None) == ca.OK


def test_create_without_gpu_reports_no_device(L):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible; covered by the GPU tests")
    h = ctypes.c_void_p()
    assert L.ca_create(ctypes.byref(h), 0, None) == ca.ERR_NO_DEVICE
    assert h.value is None
    assert _last(L)
    with pytest.raises(ca.CurveAlignError) as ei:
        ca.Context(0)
    assert ei.value.status == ca.ERR_NO_DEVICE


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rescore", ctypes.c_int32),
                ("theta_fp64", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def test_argument_errors_before_device_work(L):
    ctx = ctypes.c_void_p(0x1000)    # dummy handle: every case below must fail before using it
    p = ctypes.c_void_p(0x2000)      # dummy data pointer, never dereferenced on the host
    ok = _Opts(0, 0, 0, 0)
    bad = {"precision": _Opts(3, 0, 0, 0), "rescore": _Opts(0, 2, 0, 0), "reserved": _Opts(0, 0, 0, 1)}
    for what, o in bad.items():
        assert L.align_batch(ctx, p, p, None, 64, 4, p, ctypes.byref(o), None) == ca.ERR_INVALID_ARG
        assert what in _last(L)
        assert L.align_all_pairs(ctx, p, 8, 64, p, ctypes.byref(o), None) == ca.ERR_INVALID_ARG
    assert L.align_batch(ctx, p, p, None, 64, -1, p, None, None) == ca.ERR_INVALID_ARG
    assert L.align_batch(ctx, None, p, None, 64, 4, p, None, None) == ca.ERR_INVALID_ARG
    assert L.align_batch(ctx, p, p, None, 64, 4, None, None, None) == ca.ERR_INVALID_ARG
    assert L.align_batch(ctx, p, p, None, 64, 2 ** 31, p, None, None) == ca.ERR_INVALID_ARG
    for n in (0, 1, 4097, 8192):
        assert L.align_batch(ctx, p, p, None, n, 4, p, None, None) == ca.ERR_UNSUPPORTED_N, n
        assert L.align_pair(ctx, p, p, n, p, None, None) == ca.ERR_UNSUPPORTED_N, n
    for n in (0, 1, 11, 96, 2048, 4095, 8192):
        assert L.align_all_pairs(ctx, p, 8, n, p, None, None) == ca.ERR_UNSUPPORTED_N, n
    fp64 = _Opts(2, 0, 0, 0)
    for n in (2053, 4093, 4095):                  # padded size above the FP64 block engine's LDS
        assert L.align_batch(ctx, p, p, None, n, 4, p, ctypes.byref(fp64), None) == ca.ERR_UNSUPPORTED_N, n
    bf = _Opts(1, 0, 0, 0)
    assert L.align_batch(ctx, p, p, None, 256, 4, p, ctypes.byref(bf), None) == ca.ERR_UNSUPPORTED_N
    assert L.align_batch(ctx, p, p, p, 128, 4, p, ctypes.byref(bf), None) == ca.ERR_UNSUPPORTED_N
    assert L.align_all_pairs(ctx, p, 8, 128, p, ctypes.byref(bf), None) == ca.ERR_INVALID_ARG
    assert L.align_all_pairs(ctx, p, -1, 64, p, ctypes.byref(ok), None) == ca.ERR_INVALID_ARG
    assert L.align_all_pairs(ctx, None, 8, 64, p, None, None) == ca.ERR_INVALID_ARG
    assert L.align_all_pairs(ctx, p, 65537, 64, p, None, None) == ca.ERR_INVALID_ARG   # > 2^31 - 1 pairs
    # the allocation-free variant validates the same way, then checks the static scratch
    for what, o in bad.items():
        assert L.align_all_pairs_noalloc(ctx, p, 8, 64, p, ctypes.byref(o), None) == ca.ERR_INVALID_ARG
        assert what in _last(L)
    for n in (0, 96, 2048):
        assert L.align_all_pairs_noalloc(ctx, p, 8, n, p, None, None) == ca.ERR_UNSUPPORTED_N, n
    assert L.align_all_pairs_noalloc(ctx, None, 8, 64, p, None, None) == ca.ERR_INVALID_ARG
    assert L.align_all_pairs_noalloc(ctx, p, 65537, 64, p, None, None) == ca.ERR_INVALID_ARG
    for m, n in ((16384, 128), (4097, 1024), (65536, 64)):
        assert ca.noalloc_scratch_bytes(m, n) > ca.NOALLOC_SCRATCH_BYTES
        assert L.align_all_pairs_noalloc(ctx, p, m, n, p, None, None) == ca.ERR_TOO_LARGE, (m, n)
        assert "CA_NOALLOC_SCRATCH_BYTES" in _last(L)
    assert L.align_all_pairs_noalloc(ctx, None, 1, 64, None, None, None) == ca.OK
    assert L.resample_arclength(ctx, p, p, -1, p, p, None, None, 0, None) == ca.ERR_INVALID_ARG
    assert L.resample_arclength(ctx, p, p, 4, p, p, None, None, 2, None) == ca.ERR_INVALID_ARG
    assert L.resample_arclength(ctx, None, p, 4, p, p, None, None, 0, None) == ca.ERR_INVALID_ARG
    assert L.resample_arclength(ctx, p, p, 4, None, p, None, None, 0, None) == ca.ERR_INVALID_ARG
    assert L.resample_arclength(ctx, p, p, 2 ** 31, p, p, None, None, 0, None) == ca.ERR_INVALID_ARG
    assert L.to_initializer(ctx, p, 64, None, -1, p, p, None) == ca.ERR_INVALID_ARG
    assert L.to_initializer(ctx, p, 0, None, 4, p, p, None) == ca.ERR_INVALID_ARG
    assert L.to_initializer(ctx, p, 64, p, 4, p, p, None) == ca.ERR_INVALID_ARG
    assert L.to_initializer(ctx, p, 64, None, 4, None, p, None) == ca.ERR_INVALID_ARG
    assert L.to_initializer(ctx, p, 64, None, 4, p, None, None) == ca.ERR_INVALID_ARG
    assert L.srv_transform(ctx, p, None, 64, -1, p, None) == ca.ERR_INVALID_ARG
    assert L.srv_transform(ctx, p, None, 1, 4, p, None) == ca.ERR_INVALID_ARG
    assert L.srv_transform(ctx, p, p, 64, 4, p, None) == ca.ERR_INVALID_ARG
    assert L.srv_transform(ctx, None, None, 64, 4, p, None) == ca.ERR_INVALID_ARG
    assert L.srv_transform(ctx, p, None, 64, 4, None, None) == ca.ERR_INVALID_ARG
    # empty work is a no-op that touches nothing
    assert L.srv_transform(ctx, None, None, 64, 0, None, None) == ca.OK
    assert L.to_initializer(ctx, None, 64, None, 0, None, None, None) == ca.OK
    assert L.align_batch(ctx, None, None, None, 64, 0, None, None, None) == ca.OK
    assert L.align_all_pairs(ctx, None, 1, 64, None, None, None) == ca.OK
    assert L.resample_arclength(ctx, None, None, 0, None, None, None, None, 0, None) == ca.OK


def _tune_file(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p).encode()


def test_tuning_arguments_rejected_on_host(L):
    ctx = ctypes.c_void_p(0x1000)    # dummy handle: every case below must fail before using it
    i32 = ctypes.c_int32
    vals = (i32 * 16)(*([8] * 16))
    cnt = i32(16)
    assert L.ca_autotune(None, 0, 1024, None, None) == ca.ERR_INVALID_ARG
    assert L.ca_tune_get(None, 0, 1024, vals, ctypes.byref(cnt)) == ca.ERR_INVALID_ARG
    assert L.ca_tune_set(None, 0, 1024, vals, 1) == ca.ERR_INVALID_ARG
    assert L.ca_tune_save(None, b"/tmp/x.json") == ca.ERR_INVALID_ARG
    assert L.ca_tune_load(None, b"/tmp/x.json", None) == ca.ERR_INVALID_ARG
    for knob in (-1, 5):
        assert L.ca_autotune(ctx, knob, 1024, None, None) == ca.ERR_INVALID_ARG
        assert L.ca_tune_get(ctx, knob, 1024, vals, ctypes.byref(cnt)) == ca.ERR_INVALID_ARG
        assert L.ca_tune_set(ctx, knob, 1024, vals, 1) == ca.ERR_INVALID_ARG
    # keys the knobs do not serve
    for knob, key in ((0, 96), (1, 2048), (2, 11), (2, 16384), (2, 1)):
        assert L.ca_autotune(ctx, knob, key, None, None) == ca.ERR_UNSUPPORTED_N, (knob, key)
    assert L.ca_autotune(ctx, 3, 5, None, None) == ca.ERR_INVALID_ARG
    # (block_plan keys 0 and -8 once ran an endless default schedule: found by the sanitizer fuzz)
    for knob, key in ((0, 96), (1, 2048), (2, 11), (3, 5), (3, -1), (2, 0), (2, -8), (2, 1), (2, 16384)):
        assert L.ca_tune_get(ctx, knob, key, vals, ctypes.byref(cnt)) == ca.ERR_INVALID_ARG, (knob, key)
    # values outside the header's ranges
    def setv(knob, key, *v):
        arr = (i32 * max(1, len(v)))(*v)
        return L.ca_tune_set(ctx, knob, key, arr, len(v))
    assert setv(0, 1024, 9) == ca.ERR_INVALID_ARG
    assert setv(0, 1024, -1) == ca.ERR_INVALID_ARG
    assert setv(0, 1024, 1, 2) == ca.ERR_INVALID_ARG
    assert setv(1, 512, 0) == ca.ERR_INVALID_ARG
    assert setv(1, 512, 257) == ca.ERR_INVALID_ARG
    assert setv(2, 4096, 8, 8, 8) == ca.ERR_INVALID_ARG          # product 512
    assert setv(2, 2048, 16, 16, 8) == ca.ERR_INVALID_ARG        # radix 16 only above M = 2048
    assert setv(2, 3072, 6, 16, 32) == ca.ERR_INVALID_ARG        # 6 and 32 are not radices
    assert setv(2, 3000, 8, 3, 5, 5) == ca.ERR_INVALID_ARG       # product 600
    assert setv(3, 0, 9) == ca.ERR_INVALID_ARG
    assert setv(4, 2, 256) == ca.ERR_INVALID_ARG                  # classes 3 and 4 only
    assert setv(4, 3, 384) == ca.ERR_INVALID_ARG
    assert L.ca_autotune(ctx, 4, 2, None, None) == ca.ERR_INVALID_ARG
    assert L.ca_tune_set(ctx, 0, 1024, vals, 0) == ca.ERR_INVALID_ARG
    assert L.ca_tune_set(ctx, 2, 4096, vals, 17) == ca.ERR_INVALID_ARG
    assert L.ca_tune_set(ctx, 0, 1024, None, 1) == ca.ERR_INVALID_ARG
    assert L.ca_tune_get(ctx, 0, 1024, None, ctypes.byref(cnt)) == ca.ERR_INVALID_ARG
    assert L.ca_tune_save(ctx, None) == ca.ERR_INVALID_ARG
    assert L.ca_tune_load(ctx, None, None) == ca.ERR_INVALID_ARG


def test_tuning_file_rejections_on_host(L, tmp_path):
    """Every malformed cache is refused while reading, before the context is
    used (the handle is a dummy)."""
    ctx = ctypes.c_void_p(0x1000)
    applied = ctypes.c_int32(-7)
    assert L.ca_tune_load(ctx, str(tmp_path / "missing.json").encode(), ctypes.byref(applied)) == \
        ca.ERR_INVALID_ARG
    assert applied.value == 0
    head = '{"format": "curvealign-tune/1", "arch": "gfx950", "num_cus": 256, "entries": %s}'
    bad = {
        "not_json": "{format: 1}",
        "truncated": head[:40],
        "trailing": head % "[]" + " x",
        "array_root": "[]",
        "format": '{"format": "other/1", "arch": "gfx950", "num_cus": 256, "entries": []}',
        "no_arch": '{"format": "curvealign-tune/1", "num_cus": 256, "entries": []}',
        "no_entries": '{"format": "curvealign-tune/1", "arch": "gfx950", "num_cus": 256}',
        "knob": head % '[{"knob": "warp_size", "key": 64, "values": [1]}]',
        "key": head % '[{"knob": "team_grid", "key": 1.5, "values": [1]}]',
        "team_key": head % '[{"knob": "team_grid", "key": 96, "values": [1]}]',
        "value": head % '[{"knob": "team_grid", "key": 1024, "values": [9]}]',
        "cols": head % '[{"knob": "allpairs_cols", "key": 512, "values": [0]}]',
        "plan_product": head % '[{"knob": "block_plan", "key": 4096, "values": [8, 8, 8]}]',
        "plan_radix": head % '[{"knob": "block_plan", "key": 4096, "values": [32, 16, 8]}]',
        "plan_r16_small": head % '[{"knob": "block_plan", "key": 1024, "values": [16, 16, 4]}]',
        "plan_key": head % '[{"knob": "block_plan", "key": 4099, "values": [4099]}]',
        "class": head % '[{"knob": "block_grid", "key": 5, "values": [1]}]',
        "threads": head % '[{"knob": "block_threads", "key": 3, "values": [1024]}]',
        "values_type": head % '[{"knob": "block_grid", "key": 1, "values": ["2"]}]',
        "one_bad_of_two": head % ('[{"knob": "block_grid", "key": 1, "values": [2]}, '
                                  '{"knob": "block_grid", "key": 2, "values": [-2]}]'),
    }
    for name, text in bad.items():
        applied.value = -7
        st = L.ca_tune_load(ctx, _tune_file(tmp_path, name + ".json", text), ctypes.byref(applied))
        assert st == ca.ERR_INVALID_ARG, name
        assert applied.value == 0, name
        assert _last(L), name
