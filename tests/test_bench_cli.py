"""The benchmark's command-line contract that holds without a GPU: more than
one GPU is refused with a message and exit status 2, and the configurations
build the workloads they describe."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_multi_gpu_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_configs_build_their_workloads():
    import bench
    A = bench.make_matrix(bench.CONFIGS["c1"])
    assert A.n == 2500 and A.nnz == 12300
    assert set(bench.CONFIGS) >= {"c1", "c2", "c3", "c4"}
    c2 = bench.CONFIGS["c2"]
    assert (c2["d"], c2["m"], c2["nev"], c2["precision"]) == (50, 50, 20, "f64")
    c3 = bench.CONFIGS["c3"]
    assert c3["d"] == (10, 20) and c3["precision"] == "mixed"
    assert bench.HBM_PEAK_GBS == 8000.0


def test_default_headline_is_the_3d_operator_in_fp64():
    # the 424 MB FP64 pass of the 160^3 operator exceeds the 256 MB last-level
    # cache, so the default line measures HBM; the mixed solve runs beside it
    import bench
    a = bench.parse_args([])
    assert a.config == "c3" and a.precision == "f64" and a.gpus == 1
    A = bench.make_matrix(bench.CONFIGS[a.config])
    assert A.n == 160 ** 3 and A.nnz == 28_518_400
    assert A.nnz * 12 + 4 * (A.n + 1) + 16 * A.n > 256 * 2 ** 20
