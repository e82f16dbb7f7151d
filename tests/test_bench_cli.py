"""The benchmark's command-line contract that holds without a GPU: more than
one GPU is refused with a message and exit status 2, and the configurations
build the workloads they describe."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("config,variant,alg_mb,slack", [("c3", "plain", 428.9, 1.05),
                                                          ("c4", "ring", 695.7, 1.10)])
def test_traffic_entries_match_the_kernel_source(config, variant, alg_mb, slack):
    """The HBM traffic a line reports was counted for the kernel source as
    it stands: its key carries the hash of the source the variant is built
    from (the shared part of spmv.hip up to the windowed variant, plus the
    sliding-window kernel for that variant), so any edit there makes the
    entry stale (reported as null) until the counters are taken again.  The
    counted bytes sit at or a little above the algorithmic bytes per launch
    (for the sliding window, each segment's first column range on top)."""
    import hashlib
    import bench
    src = open(os.path.join(ROOT, "paper_1806_08020_amd", "csrc", "spmv.hip")).read()
    part = src[:src.index("// Windowed variant:")]
    if variant == "ring":
        part += src[src.index("// Sliding-window variant"):src.index("// A Y for K columns")]
    h = hashlib.sha256(part.encode()).hexdigest()[:16]
    assert bench.kernel_source_hash(variant) == h
    keys = [k for k in bench.MEASURED_TRAFFIC if k[0] == config and k[1] == "f64" and k[2] == variant]
    assert keys and all(k[3] == h for k in keys), (h, keys)
    for k in keys:
        assert bench.traffic_key(config, "f64", variant, *k[4:]) == k
        e = bench.MEASURED_TRAFFIC[k]
        mb = 1024 * (e["fetch_kib"] * e["fetch_factor"] + e["write_kib"] * e["write_factor"]) / 1e6
        assert alg_mb <= mb <= slack * alg_mb


def test_reference_probe_flags():
    """--bw-probe runs only the bandwidth reference kernels; the default run
    carries them as hbm_reference beside the headline."""
    import bench
    assert bench.parse_args(["--bw-probe"]).bw_probe
    assert not bench.parse_args([]).bw_probe
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'line["hbm_reference"] = bw_probe(torch)' in src


def test_cpu_baseline_fields_on_the_small_configuration():
    """The CPU baseline leg (the oracle, bounded) returns the reported rate
    with its unit, cores and kind, the per-step timings and the per-solve
    estimate, and the host description, on the 2-D Laplacian 50 x 50."""
    import bench
    import oracle as O
    cfg = bench.CONFIGS["c1"]
    csr = bench.make_matrix(cfg)
    from paper_1806_08020_amd import workloads as W
    b, _ = W.start_vectors(csr.n, cfg["seed"])
    roots, _ = O.gmres_poly(O.csr_matvec(csr), b, cfg["d"])
    bpa = cfg["d"] * (csr.nnz * 12 + 4 * (csr.n + 1) + 16 * csr.n)
    cb = bench.cpu_baseline(csr, roots, bpa, 0.2, cfg, 2, b)
    assert cb["unit"] == "GB/s" and cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0
    for k in ("s_per_pi_apply", "s_polynomial_build", "s_per_cycle_estimate", "s_per_solve_estimate",
              "eigenpairs_per_s_estimate", "host", "sample"):
        assert k in cb, k
    assert cb["s_per_solve_estimate"] >= cb["s_polynomial_build"]


def test_every_spmv_variant_names_its_kernel():
    """The roofline block names the kernel of whichever SpMV variant the
    matrix runs, and each variant's traffic key hashes a different source."""
    import bench
    from paper_1806_08020_amd import ppa
    assert set(bench.KERNEL_OF_VARIANT) == set(ppa.Matrix.SPMV_VARIANTS)
    src = open(os.path.join(ROOT, "paper_1806_08020_amd", "csrc", "spmv.hip")).read()
    for v, k in bench.KERNEL_OF_VARIANT.items():
        assert f"void {k}(" in src, k
    hashes = {bench.kernel_source_hash(v) for v in bench.KERNEL_OF_VARIANT}
    assert len(hashes) == len(bench.KERNEL_OF_VARIANT)
