"""Host-side logic of bench.py (no GPU): the one-GPU guard and the reduction
of rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes per launch, scaled by
the readings of a plain copy of known size."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_ALL)
        w.writerow(HEADER)
        for i, (name, value) in enumerate(rows):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 512, 7, name, 512, 0, 0, 104, 0, 48, counter, value, 0, 1])


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pmc_summary_scales_by_the_copy_calibration(tmp_path):
    proj = "void gw::(anonymous namespace)::gemm8_bf16x3_kernel<0, false>(gw::(anonymous namespace)::GemmArgs)"
    herk = "void gw::(anonymous namespace)::gemm8_bf16x3_kernel<2, false>(gw::(anonymous namespace)::GemmArgs)"
    copy = "__amd_rocclr_copyBuffer"
    d = [str(tmp_path / x) for x in ("f", "w", "cf", "cw")]
    _write(d[0], "FETCH_SIZE", [(proj, 100.0), (proj, 300.0), (herk, 50.0)])
    _write(d[1], "WRITE_SIZE", [(proj, 10.0), (proj, 10.0), (herk, 4.0)])
    _write(d[2], "FETCH_SIZE", [(copy, 524288.0)])      # a 1 GiB copy read as half its size
    _write(d[3], "WRITE_SIZE", [(copy, 1048576.0)])
    out = tmp_path / "traffic.json"
    r = _bench("--summarize-pmc", *d, "--traffic", str(out))
    assert r.returncode == 0, r.stderr
    t = json.loads(out.read_text())
    assert t["copy_factor_fetch"] == 2.0 and t["copy_factor_write"] == 1.0
    assert t["kernel"] == "project_bf16_kernel"
    assert t["symbol"] == "gemm8_bf16x3_kernel<0, false>"
    k = t["kernels"]["gemm8_bf16x3_kernel<0, false>"]
    assert k["fetch_bytes_per_launch"] == 200.0 * 1024 * 2.0
    assert k["write_bytes_per_launch"] == 10.0 * 1024
    assert t["bytes_per_launch"] == 200.0 * 1024 * 2.0 + 10.0 * 1024
    assert t["kernels"]["gemm8_bf16x3_kernel<2, false>"]["fetch_bytes_per_launch"] == 50.0 * 1024 * 2.0
    assert len(t["source_hash"]) == 16


def test_block_error_estimate_weights_diagonal_and_off_diagonal():
    """A block of sampled rows and columns over-weights the diagonal; the
    estimate rescales the block's diagonal and off-diagonal errors by the whole
    matrix's norms and recovers the full-matrix error."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    rng = np.random.default_rng(0)
    N, n_om = 400, 3
    A = rng.normal(size=(n_om, N, N)) + 1j * rng.normal(size=(n_om, N, N))
    P = 0.05 * (A + np.conj(np.transpose(A, (0, 2, 1)))) + np.eye(N)[None] * 30.0
    noise = rng.normal(size=P.shape) + 1j * rng.normal(size=P.shape)
    eye = np.eye(N, dtype=bool)
    X = P + np.where(eye[None], 1e-6, 1e-3) * np.abs(P) * noise      # large off-diagonal errors
    full = np.linalg.norm((X - P).reshape(n_om, -1), axis=1) / np.linalg.norm(P.reshape(n_om, -1), axis=1)
    S = np.sort(rng.choice(N, 32, replace=False))
    D = np.linalg.norm(np.diagonal(X, axis1=1, axis2=2), axis=1)
    F = np.linalg.norm(X.reshape(n_om, -1), axis=1)
    be = bench._block_errors(X[:, S][:, :, S], P[:, S][:, :, S], (D, F))
    est = np.array(be["full_matrix_estimate_per_omega"])
    assert np.all(np.abs(est / full - 1) < 0.15), (est, full)
    assert be["max_rel_fro_err"] < 0.5 * full.min()                    # the plain block error is biased low


def test_pmc_summary_names_the_six_slot_projection(tmp_path):
    """The projection of the default core is the OUT_TILED instance of the
    six-slot kernel (first template argument 0); the row-projection and
    accumulation instances are not taken for it."""
    rows = "void gw::(anonymous namespace)::gemm3r_kernel<1, 0, 4, false>(gw::(anonymous namespace)::GemmArgs)"
    proj = "void gw::(anonymous namespace)::gemm3r_kernel<0, 0, 4, false>(gw::(anonymous namespace)::GemmArgs)"
    herk = "void gw::(anonymous namespace)::gemm3r_kernel<2, 0, 4, false>(gw::(anonymous namespace)::GemmArgs)"
    copy = "__amd_rocclr_copyBuffer"
    d = [str(tmp_path / x) for x in ("f", "w", "cf", "cw")]
    _write(d[0], "FETCH_SIZE", [(rows, 7.0), (proj, 100.0), (herk, 50.0)])
    _write(d[1], "WRITE_SIZE", [(rows, 1.0), (proj, 10.0), (herk, 4.0)])
    _write(d[2], "FETCH_SIZE", [(copy, 524288.0)])
    _write(d[3], "WRITE_SIZE", [(copy, 1048576.0)])
    out = tmp_path / "traffic.json"
    r = _bench("--summarize-pmc", *d, "--traffic", str(out))
    assert r.returncode == 0, r.stderr
    t = json.loads(out.read_text())
    assert t["symbol"] == "gemm3r_kernel<0, 0, 4, false>"
    assert t["bytes_per_launch"] == 100.0 * 1024 * 2.0 + 10.0 * 1024


def test_traffic_reported_only_for_the_measured_sources(tmp_path):
    """A counter summary gives the roofline's traffic only for the kernel and
    workload it was measured on and while the GEMM sources hash to the
    measured build; anything else (other hash, kernel or workload, a missing
    or unreadable file) gives None rather than a stale figure."""
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    good = {"workload": "c5", "kernel": "project_bf16_kernel", "source_hash": h, "bytes_per_launch": 1.5e11}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(good))
    assert bench.measured_traffic(str(f), "project_bf16_kernel", "c5") == 1.5e11
    assert bench.measured_traffic(str(f), "herk_bf16_kernel", "c5") is None
    assert bench.measured_traffic(str(f), "project_bf16_kernel", "c3") is None
    f.write_text(json.dumps(dict(good, source_hash="0" * 16)))
    assert bench.measured_traffic(str(f), "project_bf16_kernel", "c5") is None
    f.write_text("{not json")
    assert bench.measured_traffic(str(f), "project_bf16_kernel", "c5") is None
    assert bench.measured_traffic(str(tmp_path / "missing.json"), "project_bf16_kernel", "c5") is None


def test_committed_traffic_summary_matches_the_sources():
    """profiles/traffic_c5.json was measured on the GEMM sources in the tree
    (a kernel edit without new counter passes makes this fail, and the bench
    then reports traffic as null)."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic_c5.json")) as fh:
        t = json.load(fh)
    assert t["workload"] == "c5" and t["kernel"] == "project_bf16_kernel"
    assert t["source_hash"] == bench.kernel_source_hash()
    assert bench.measured_traffic(os.path.join(ROOT, "profiles", "traffic_c5.json"), "project_bf16_kernel", "c5") > 0
