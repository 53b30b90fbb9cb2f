"""Host check of the group kernel's tile plans and 64-bit tile descriptors
(tests/group_plan_check.hip, compiled here with hipcc; no GPU): every subset
covered once, descriptors decoding to the right first B, B count and T, every
lane's group walk landing on its B, and each tile within the kernel's group
and record bounds."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not found")
def test_group_plans_and_descriptors(tmp_path):
    exe = str(tmp_path / "group_plan_check")
    obj = exe + ".o"
    csrc = os.path.join(ROOT, "paper_2511_14923_amd", "csrc")
    flags = ["-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", csrc]
    subprocess.run([HIPCC] + flags + ["-c", os.path.join(HERE, "group_plan_check.hip"), "-o", obj],
                   check=True, capture_output=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-o", exe, obj], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "failures 0" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not found")
def test_tshard_work_decomposition(tmp_path):
    """The T-shared shard kernel's T list and tiles (tests/tshard_plan_check.hip):
    every rank of a range written exactly once, at the colex rank of the subset
    {a, b_0} + T the lane and loop name, within the kernel's bounds."""
    exe = str(tmp_path / "tshard_plan_check")
    obj = exe + ".o"
    csrc = os.path.join(ROOT, "paper_2511_14923_amd", "csrc")
    flags = ["-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", csrc]
    subprocess.run([HIPCC] + flags + ["-c", os.path.join(HERE, "tshard_plan_check.hip"), "-o", obj],
                   check=True, capture_output=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-o", exe, obj], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "failures 0" in r.stdout
