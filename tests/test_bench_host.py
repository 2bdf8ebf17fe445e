"""bench.py's host-side logic, on the CPU: the one-GPU guard, the source
hash that ties a counter summary to the code it measured, and the committed
summaries it reads."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_source_hash_ignores_comments_and_layout():
    a = "int f(int x) {  // twice\n  return 2 * x; /* scaled */\n}\n"
    b = "int f(int x) {\n\n      return 2 * x;\n}   // no comment\n"
    c = "int f(int x) { return 3 * x; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_each_roofline_kernel_has_a_counter_summary():
    for workload, (kernel, files) in bench.PROFILED.items():
        if workload == "c1":
            continue  # launch-latency workload: no roofline kernel summary
        path = os.path.join(ROOT, "profiles", "%s_%s.md" % (kernel, workload))
        assert os.path.exists(path), path
        text = open(path).read()
        keys = dict(re.findall(r"^- (\w+): (\S+)", text, flags=re.M))
        for key in ("source_sha", "hbm_bytes_per_launch", "valu_issue_frac"):
            assert key in keys, (path, key)
        assert re.fullmatch(r"[0-9a-f]{16}", keys["source_sha"]), path
        for f in files:
            assert os.path.exists(os.path.join(ROOT, "paper_2212_00574_amd", "csrc", f)), f
