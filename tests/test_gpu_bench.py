"""bench.py's output contract on small workloads: one JSON line with the keys
the measurement is read from, a roofline object for the dominant kernel, the
oracle's CPU baseline, per-frequency parity and the W check (config 2 shapes);
and on the learned path (config 4: config 3 shapes, band sum cut at 300) the
judge report, the correction step's parity and the model error against the
all-band sum beside the truncation error."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    print("bench", *args, flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       timeout=900, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    return json.loads(lines[0])


def test_bench_json_contract_small_workload():
    d = _bench("--workload", "c2", "--cpu-seconds", "2")
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["higher_is_better"] is False and d["value"] > 0
    assert d["config"]["workload"].startswith("c2")
    rf = d["roofline"]
    assert rf["bound"] in ("mfma", "hbm", "alu")
    assert rf["unit"] in ("TFLOP/s", "GB/s")
    assert rf["achieved"] > 0 and rf["peak"] > 0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert "traffic" in rf
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
    par = d["parity"]
    assert par["max_rel_fro_err"] < 1e-4
    assert len(par["explicit_bands"]["per_omega"]) == 13 and max(par["explicit_bands"]["per_omega"]) < 1e-4
    assert par["explicit_bands"]["full_matrix_estimate_max"] < 1e-4
    assert len(par["explicit_bands"]["offdiag_per_omega"]) == 13
    assert len(par["w_residual_per_omega"]) == 13 and par["w_residual_max"] < 1e-8
    assert d["screening_ok"] is True and d["rel_err_bar_met"]["numeric_parity_vs_oracle"] is True
    assert d["model_error"] is None
    print(f"c2 bench line: {d['value']} {d['unit']}, dominant kernel {rf['kernel']} at {rf['achieved']} {rf['unit']}; "
          f"cpu baseline {cb}")


def test_bench_learned_path_reports_model_error():
    d = _bench("--workload", "c4", "--steps", "1", "--warmup", "1", "--no-compare", "--cpu-seconds", "2")
    assert d["config"]["workload"].startswith("c4") and d["config"]["surrogate"] is True
    j = d["config"]["surrogate_judge"]
    assert "judge_err" in j and len(j["judge_err"]) == 16 and "used_fallback" in j
    m = d["model_error"]
    assert len(m["corrected_vs_all_bands_per_omega"]) == 16 and len(m["truncation_per_omega"]) == 16
    if not j["used_fallback"]:
        # the correction removes most of what truncation leaves (A19 ii: reported, not gated at 1e-4)
        assert m["corrected_vs_all_bands_mean"] < 0.5 * m["truncation_mean"]
        assert d["parity"]["correction_step"]["max_rel_fro_err"] < 1e-4
    assert d["parity"]["explicit_bands"]["max_rel_fro_err"] < 1e-4
    assert d["parity"]["left_out_bands"]["max_rel_fro_err"] < 1e-4
    assert d["rel_err_bar_met"]["model_vs_all_bands"] == m["meets_1e-4"]
    print(f"c4 bench line: {d['value']} s/q-point, judge {j.get('judge_err_max')}, model error mean "
          f"{m['corrected_vs_all_bands_mean']:.4f} vs truncation {m['truncation_mean']:.4f}")
