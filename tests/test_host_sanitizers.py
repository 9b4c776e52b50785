"""Host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only; no GPU needed).

capi.cpp and tune.hip are compiled with the sanitizers on their host code
only (each -fsanitize= behind -Xarch_host, so no device code is instrumented)
and linked with the ordinary objects of the kernel sources into
tests/sanitize/harness.cpp, which fuzzes the tuning-file parser (ca_tune_load)
with mutated documents, calls every entry point with random and invalid
arguments, and round-trips tuning choices through ca_tune_save/ca_tune_load.
Any sanitizer report aborts the harness; any failed check makes it exit
non-zero.
"""
import os
import subprocess

import pytest

from paper_2501_17779_amd import build as cabuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_17779_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
HIPFLAGS = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain not found")
    d = tmp_path_factory.mktemp("san")
    # ordinary objects of the kernel sources (built by the library build)
    plain = [os.path.join(cabuild.BUILD, f) for f in ("align.o", "resample.o", "bf16.o", "handoff.o", "srv.o")]
    if not all(os.path.exists(p) for p in plain):
        cabuild.build()
    objs = []
    procs = []
    for src in ("capi.cpp", "tune.hip", "../../tests/sanitize/harness.cpp"):
        obj = str(d / (os.path.basename(src) + ".o"))
        procs.append(subprocess.Popen([HIPCC, *HIPFLAGS, *SAN, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, f"{p.args}\n{out}\n{err}"
    exe = str(d / "harness")
    _run([CLANG, "-fsanitize=address,undefined", *objs, *plain, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    return exe, d


def test_host_code_under_asan_and_ubsan(harness):
    exe, d = harness
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""      # host code only, also on a machine with a GPU
    cache = os.path.join(ROOT, "paper_2501_17779_amd", "tune_cache.json")
    r = subprocess.run([exe, str(d), cache, "3000"], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, f"harness failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "all host checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
