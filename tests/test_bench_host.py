"""Host checks of bench.py that need no GPU: the one-GPU guard and the
summary helpers' arithmetic."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_split_shares():
    sys.path.insert(0, ROOT)
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    s = b._split(np.array([1, 2, 3, 4]), np.array([2, 2, 1, 4]))
    assert s == {"fewer": 0.25, "more": 0.25, "equal": 0.5}
    # the aggregation's minimum bytes are below its per-pair gather bytes
    fwd, _ = b.agg_bytes(1000, 100, 8, 16, 500, 4)
    assert fwd == 500 * (64 + 12) + 4 * 8 * 100 + 16 * 100 + 64 * 100
