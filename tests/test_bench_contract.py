"""Host-side pieces of bench.py that need no GPU: the refusal of more than
one GPU, the algorithmic byte counts of the step kernel, and the committed
counter summaries it reads its traffic from."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_step_bytes_per_particle_and_contact():
    # state read 112 B, written 104 B, F and T 48 B; per contact the key and
    # the springs read and written: 8 + 56 + 8 + 48 (FP64), 8 + 28 + 8 + 24
    # with the springs kept as floats
    assert bench.step_bytes(1, 0) == 112 + 104 + 48
    assert bench.step_bytes(0, 1) == 8 + 56 + 8 + 48
    assert bench.step_bytes(0, 1, mixed=True) == 8 + 28 + 8 + 24
    assert bench.step_bytes(8_000_000, 43_887_015) == 264 * 8_000_000 + 120 * 43_887_015
    assert bench.step_bytes_formula() == "264 N + 120 C"
    assert bench.step_bytes_formula(True) == "264 N + 68 C"


@pytest.mark.parametrize("workload,key", [("packing_8M", "traffic"),
                                          ("packing_8M", "traffic_mixed"),
                                          ("column_200k", "traffic")])
def test_counter_summaries_are_well_formed(workload, key):
    """Each summary names the commands that made it (committed files only)
    and carries the figure bench.py reads and the source hash it checks."""
    name = bench.WORKLOADS[workload][key]
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    assert "python3 bench.py" in text and "_work" not in text
    m = re.search(r"^traffic_bytes_per_launch: (\d+)$", text, re.M)
    assert m and int(m.group(1)) > 0
    assert re.search(r"^kernel_source_sha256_16: [0-9a-f]{16}$", text, re.M)
