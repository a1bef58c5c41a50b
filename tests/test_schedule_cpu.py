"""Host checks of the pair schedules (tests/native/schedule_check.cpp over
paper_2309_00651_amd/csrc/schedule.cpp): every pair i <= j evaluated once
(every kept pair once when screened), disjoint orbitals inside a batch,
tile-pair shapes, slots and energy partials, for row tiles of 8-32 rows,
ragged orbital counts, batch caps, virtual groups and random screenings.
Compiled with hipcc as host code (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_schedule_host_checks(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "schedule_check")
    srcs = [os.path.join(HERE, "native", "schedule_check.cpp"),
            os.path.join(ROOT, "paper_2309_00651_amd", "csrc", "schedule.cpp")]
    cmd = [hipcc, "-std=c++17", "-O1", "--offload-arch=gfx950"]
    for s in srcs:
        cmd += ["-x", "hip", s]
    subprocess.run(cmd + ["-o", exe], check=True, capture_output=True, timeout=600)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-2000:]
    assert "ALL OK" in r.stdout
