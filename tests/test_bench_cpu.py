"""Host-side checks of the benchmark script: the one-GPU contract and the
stored HBM traffic keys."""

import ast
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_table_keys_name_a_shape_and_a_source():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    table = None
    for node in tree.body:
        if isinstance(node, ast.Assign) and getattr(node.targets[0], "id", "") == "MEASURED_TRAFFIC":
            table = ast.literal_eval(node.value)
    assert table
    for (workload, kernel, source, shape), value in table.items():
        assert workload in ("box20-p1", "pack512-p2", "batch256-p12", "pack256-p3")
        assert kernel.startswith("k_stage")
        assert len(source) == 16 and int(source, 16) >= 0
        assert len(shape) == 4 and all(isinstance(x, int) for x in shape)
        assert value > 0
