"""Host-side checks of bench.py (no GPU): the one-GPU rule and the
bookkeeping behind its traffic figure."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a configuration that was not run


def test_traffic_constant_matches_the_committed_profile():
    """bench.py reports PMC-measured traffic only for the sources it was
    profiled on; the constant and the profile summary must name the same
    sources and bytes."""
    import bench
    prof = open(os.path.join(ROOT, "profiles", "step_kernel_cube256.md")).read()
    sha = re.search(r"bench\.source_sha\(\)\): `([0-9a-f]+)`", prof).group(1)
    assert sha == bench.TRAFFIC_SOURCE_SHA
    # the traffic table's row: dispatches, raw fetch, scaled fetch, write, total (MiB)
    row = re.search(r"^\| `" + re.escape(bench.TRAFFIC_KERNEL) +
                    r"` \| ([0-9]+) \| ([0-9.]+) \| ([0-9.]+) \| ([0-9.]+) \| ([0-9.]+) \|$", prof,
                    flags=re.M)
    assert row is not None
    fetch_raw, fetch, write, total = (float(row.group(k)) for k in (2, 3, 4, 5))
    assert abs(fetch - 2.0 * fetch_raw) < 0.15 and abs(total - fetch - write) < 0.15
    assert abs(total * 2 ** 20 - bench.TRAFFIC_BYTES_F64) < 0.05 * 2 ** 20
