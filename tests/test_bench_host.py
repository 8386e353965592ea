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
