"""CPU model of the persistent traversal's queue claims (tests/claim_model.cpp): the kernel's
claim arithmetic (paper_2510_07868_amd/csrc/claim.hpp, shared by kernel and model) replayed
over random wave schedules, ray lengths, queue sizes (0 .. 300,001 entries, ragged slices),
claim chunks and refill thresholds, asserting that every index handed to a lane is in bounds,
comes from the pool or the slice it was claimed from, is handed out once, and that every entry
is handed out."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not installed")
def test_claim_indices_stay_in_bounds_and_cover_the_queue(tmp_path):
    exe = str(tmp_path / "claim_model")
    cc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    r = subprocess.run([cc, "--offload-host-only", "-O2", "-std=c++17", "-o", exe,
                        os.path.join(ROOT, "tests", "claim_model.cpp")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(out.stdout[-2000:])
    assert out.returncode == 0 and out.stdout.strip().startswith("claims ok"), out.stdout[-2000:]
