"""Resources of the step kernel as compiled for gfx950 (hipcc, device code
only, no GPU needed): both precisions must keep three 256-thread
workgroups per CU, which takes at most 168 VGPRs per lane without spills
and at most 53,344 bytes of LDS (54,112 bytes measured two workgroups per
CU on MI355X), and packed FP32 instructions must be absent."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    from paper_2507_12610_amd import build as B
    out = tmp_path_factory.mktemp("isa") / "kernels.s"
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2507_12610_amd", "csrc"),
           os.path.join(ROOT, "paper_2507_12610_amd", "csrc", "kernels.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out.read_text()


def kernel_meta(text, name_part):
    """(vgpr_count, vgpr_spill_count, group_segment_fixed_size) of the kernel
    whose mangled name contains name_part, from the code object metadata."""
    blocks = re.split(r"\n\s*- \.", text)
    for b in blocks:
        m = re.search(r"\.name:\s+(\S+)", b)
        if m and name_part in m.group(1):
            vg = int(re.search(r"\.vgpr_count:\s+(\d+)", b).group(1))
            sp = int(re.search(r"\.vgpr_spill_count:\s+(\d+)", b).group(1))
            lds = int(re.search(r"\.group_segment_fixed_size:\s+(\d+)", b).group(1))
            return vg, sp, lds
    raise AssertionError(f"kernel {name_part} not found")


@pytest.mark.parametrize("inst", ["k_stepIdE", "k_stepIfE"])
def test_step_kernel_fits_three_workgroups_per_cu(asm, inst):
    vgpr, spill, lds = kernel_meta(asm, inst)
    assert spill == 0, spill
    assert vgpr <= 168, vgpr
    assert lds <= 53_344, lds


def test_no_packed_fp32_instructions(asm):
    assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", asm)
