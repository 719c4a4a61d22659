"""Code-generation guard for the float push (the benchmark's hot kernel):
every instantiation of k_push_deposit<float, ...> keeps its state in
registers -- no private (scratch) segment and no call -- in the gfx950 code
that hipcc produces with the library's flags.  A helper that the inliner
leaves out of line turns the run parameters into scratch reads and slows the
push several times without changing a result, so the parity tests cannot
see it."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1511_08225_amd"))


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_float_push_has_no_scratch_and_no_calls(tmp_path):
    import build
    out = tmp_path / "k32.s"
    cmd = [build.HIPCC, *build.COMMON, "--offload-device-only", "-S", "-o", str(out),
           os.path.join(build.CSRC, "kernels_f32.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    kernels = 0
    for blk in re.findall(r"(- \.agpr_count.*?\.vgpr_spill_count:\s+\d+)", asm, re.S):
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        if "k_push_depositIf" not in name:
            continue
        kernels += 1
        scratch = int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", blk).group(1))
        assert scratch == 0, (name, scratch)
    assert kernels >= 20  # P in {1, 2, 4, 8, 16} x push/deposit x sheath/generic/profile
    assert "s_swappc" not in asm
