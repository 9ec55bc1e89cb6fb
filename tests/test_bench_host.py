"""The host side of bench.py, without a GPU: a request for more than one GPU
is refused with a message and no JSON line, and the oracle baseline leg
reports what the line's cpu_baseline object carries."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_cpu_baseline_reports_the_oracle():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench

    ns = 2 * bench.L * (bench.L - 1)
    res = bench.cpu_baseline(1, ns, workers=1, init="mwpm")
    assert res["kind"] == "oracle"
    assert res["unit"] == "syndromes/s"
    assert res["cores"] == 1 and res["host"]["cores_used"] == 1
    assert res["value"] > 0
    assert "exact enhanced-matching" in res["sample"]
    # one syndrome: 4 classes x chains x temperatures x (burn + sweeps) x stabilizers
    per = 4 * bench.CHAINS * bench.K * (bench.BURN + bench.SWEEPS) * ns
    assert abs(res["stabilizer_updates_per_s"] / res["value"] - per) < 1e-6 * per
