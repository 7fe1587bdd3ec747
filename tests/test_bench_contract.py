"""Host-side contract of bench.py: one GPU only, and the profile summaries
it reads its HBM traffic and utilisation from parse for the kernel source
they were taken on (no GPU needed)."""
import hashlib
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_profile_summaries_parse_for_their_kernel_source():
    sys.path.insert(0, ROOT)
    import bench
    src = os.path.join(ROOT, "paper_1301_0955_amd", "csrc", "lcd_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    text = open(os.path.join(ROOT, "profiles", "sweep_lfr3-10M-share64_kernels.md")).read()
    m = re.search(r"^kernels_sha256: ([0-9a-f]{64})", text, re.M)
    assert m
    caps = json.loads(re.search(r"^profiled_tier_capacities: (\[.*\])", text, re.M).group(1))
    t = bench.profiled_traffic("sweep_team_global_rec_kernel", caps, "xl64")
    u = bench.profiled_utilisation("sweep_team_global_rec_kernel", "xl64")
    if m.group(1) == sha:
        # taken on this source: both summaries give numbers for the dominant kernel
        assert t is not None and t > 0
        assert u is not None and 0 < u["valu_issue_frac"] < 1 and 0 < u["fp64_frac_upper"] < 1
    else:
        # a profile of another source is never reported
        assert t is None and u is None
    # other workloads or tier layouts never borrow the numbers
    assert bench.profiled_traffic("sweep_team_global_rec_kernel", caps, "large") is None
    assert bench.profiled_traffic("sweep_team_global_rec_kernel", [256] + list(caps[1:]), "xl64") is None


def test_kernel_names_follow_the_table_layout():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.kernel_of(3, 131072) == "sweep_team_global_rec_kernel"
    assert bench.kernel_of(3, 65536) == "sweep_team_global_rec_kernel"
    assert bench.kernel_of(3, 16384) == "sweep_team_global_kernel"
    assert bench.kernel_of(0, 512) == "sweep_lds_kernel"
    # the record layout starts where the library's does
    hdr = open(os.path.join(ROOT, "paper_1301_0955_amd", "csrc", "lcd_internal.h")).read()
    m = re.search(r"kRecordMinEntries = (\d+);", hdr)
    assert m and int(m.group(1)) == bench.RECORD_MIN_ENTRIES
