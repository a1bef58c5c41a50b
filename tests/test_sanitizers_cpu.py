"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU (no GPU): the library's sources built with the sanitizers on their host
code only (device code is not instrumented), then
* tests/native/abi_check.cpp: option parsing, system validation, the
  clean-up of a plan whose device set-up fails, the tune-cache helpers, the
  autotuner's and every entry point's argument errors;
* tests/native/schedule_check.cpp: the pair schedules (every pair once,
  disjoint batches, screened schedules, plane maps).
A sanitizer report makes the run exit non-zero."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2309_00651_amd", "csrc")
# host-only instrumentation: every -fsanitize= goes to the host compiler
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
LIB_SOURCES = ["hfx_api.cpp", "autotune.cpp", "schedule.cpp", "exchange_common.hip",
               "exchange_f32.hip", "exchange_f64.hip", "gemm.hip", "ortho.hip", "ace.hip",
               "scdm.hip"]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        pytest.skip("hipcc not available")
    return h


def _compile(hipcc, src, out):
    cmd = [hipcc, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", *SAN,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-x", "hip", "-c", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    print(r.stdout[-2000:], r.stderr[-3000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "ALL OK" in r.stdout


@pytest.mark.slow
def test_abi_and_schedules_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    srcs = [os.path.join(CSRC, s) for s in LIB_SOURCES] + \
        [os.path.join(HERE, "native", "abi_check.cpp"),
         os.path.join(HERE, "native", "schedule_check.cpp")]
    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(hipcc, s, str(tmp_path / (os.path.basename(s) + ".o"))),
                           srcs))
    lib_objs, abi_obj, sched_obj = objs[:-2], objs[-2], objs[-1]
    abi_exe, sched_exe = str(tmp_path / "abi_check"), str(tmp_path / "schedule_check")
    for exe, main_obj in ((abi_exe, abi_obj), (sched_exe, sched_obj)):
        r = subprocess.run([hipcc, "--offload-arch=gfx950", *SAN, main_obj, *lib_objs, "-o", exe],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
    _run(abi_exe)
    _run(sched_exe)
