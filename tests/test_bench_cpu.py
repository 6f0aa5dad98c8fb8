"""The benchmark's contract on the host: more than one GPU is refused with a message, and the
per-unit work models behind the roofline objects are the stated sums."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_work_models():
    import bench
    st = dict(pixels=100, covered=60, samples=3840, shadow_rays=1000, shadow_nodes=30000, shadow_tris=5000,
              sec_rays=200, sec_nodes=7000, sec_tris=1200, sec_shadow_rays=500, sec_shadow_nodes=15000,
              sec_shadow_tris=2500)
    # a 4-wide node visit: four child slab tests of 25 lane operations, then 3 (any-hit: nearest
    # first) or 5 (closest hit: sorted) compare-exchanges of 4; 128 B per node, 48 B per triangle
    assert bench.kernel_lane_ops_per_step("trace_any", st) == (4 * 25 + 3 * 4) * (30000 + 15000) + 44 * (5000 + 2500)
    assert bench.kernel_lane_ops_per_step("trace_closest", st) == (4 * 25 + 5 * 4) * 7000 + 44 * 1200
    # 16 B ray record in and 1 B out per ray; one 16 B origin record per covered pixel
    assert bench.kernel_bytes_per_step("trace_any", st, None) == 17 * 1500 + 16 * 60 + 128 * 45000 + 48 * 7500
    assert bench.kernel_bytes_per_step("trace_closest", st, None) == 32 * 200 + 16 * 60 + 128 * 7000 + 48 * 1200
    assert abs(bench.VALU_PEAK_T - 39.3216) < 1e-9
