#!/usr/bin/env python
"""Benchmark: seconds per q-point of P(q, i w) (plus W) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5]

A step is one pass of the whole hot path over the workload, inputs resident in
HBM: split of U into BF16 hi/lo words, fused product + projection, transition
weights, weighted Hermitian accumulation over all k-points and frequencies
(split-BF16 on MFMA, unoccupied bands up to the cutoff), the learned high-band
correction when a trained model is present, and the FP64 screening
W = (1 - vP)^-1 v.  Inputs are synthetic (seeded, shaped like the paper's
supercell workload: N_k=4, N=6000, R=65536, 256 occupied + 6000 unoccupied
bands, 16 imaginary frequencies, cutoff at 1500 unoccupied bands).

Also reported on the same JSON line:
  * the plain FP32 MFMA path on all 6000 unoccupied bands, timed on a sample of
    occupied bands of one k-point and scaled linearly to a whole q-point;
  * parity of sampled outputs at full size against the FP64 oracle;
  * "roofline" for the dominant kernel (HIP-event timing inside the timed
    region) and "cpu_baseline" (the oracle timed on a bounded sample, scaled).
"""
from __future__ import annotations

import argparse
import json
import re
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2516.6, "fp16": 2516.6, "fp32": 157.3, "fp64": 78.6}
HBM_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c5", "c4", "c3", "c2"])
    ap.add_argument("--precision", default="split_bf16", choices=["split_bf16", "split_fp16", "fp32", "fp16"],
                    help="fp16: the single-FP16 ablation (misses the 1e-4 bar)")
    ap.add_argument("--cutoff", type=int, default=None, help="explicit unoccupied bands (default: workload's)")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 plain-path comparison")
    ap.add_argument("--fp32-full", action="store_true",
                    help="time the FP32 plain path over every pair of the q-point instead of a sample")
    ap.add_argument("--no-model-error", action="store_true",
                    help="skip the all-band reference pass (model error of the learned correction)")
    ap.add_argument("--sample-occ", type=int, default=2, help="judge sample: occupied bands per k-point")
    ap.add_argument("--chunk-pairs", type=int, default=0, help="transition pairs per chunk (0: library default)")
    ap.add_argument("--judge-tol", type=float, default=0.25, help="judge tolerance of the learned correction")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target oracle time for cpu_baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for HBM traffic counters)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE csv outputs (bench run, then the copy "
                         "calibration) into the traffic file")
    ap.add_argument("--sigma", action="store_true",
                    help="measure the correlation self-energy instead (supercell workload: W for every momentum "
                         "transfer, then Sigma_c(i w) of the highest occupied and lowest unoccupied state)")
    ap.add_argument("--real", action="store_true",
                    help="measure the real-input (inversion-symmetric) path instead: the largest workload's shapes "
                         "with real U and wave functions, explicit bands to the cutoff, against the complex path "
                         "on the same pairs")
    ap.add_argument("--mpb", action="store_true",
                    help="basis optimization study instead: Sigma_c and time against the Coulomb-eigenvalue "
                         "threshold v_min on the training-run shapes")
    ap.add_argument("--spectral", action="store_true",
                    help="spectral route (transition-energy nodes + Hilbert transform) against the direct sum: time "
                         "and error for 32..256 nodes at 64 imaginary frequencies, one k-point of the supercell "
                         "workload")
    ap.add_argument("--surrogate-ablation", action="store_true",
                    help="ablation of the high-band correction on held-out training-run seeds: truncation, "
                         "missing diagonal only, congruence (learned and exact), and a rank-8 term in the "
                         "leading eigenvectors of -P_ret with coefficients fitted to the true residual")
    ap.add_argument("--ablation-seeds", type=int, default=4, help="held-out seeds for --surrogate-ablation")
    ap.add_argument("--tuning", action="append", default=[], metavar="KEY=VALUE",
                    help="kernel selection switch passed to gw_set_tuning before the run (repeatable)")
    ap.add_argument("--traffic", default=None,
                    help="measured per-launch HBM traffic of the dominant kernel (from rocprofv3 --pmc; default "
                         "profiles/traffic_<workload>.json)")
    return ap.parse_args()


def copy_calibration() -> int:
    """A plain copy of 2^30 bytes: its FETCH_SIZE / WRITE_SIZE counters give
    the factor between the counter readings and bytes moved."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}))
    return 0


def spectral_bench(a) -> int:
    """The spectral route against the direct sum on one k-point of the
    supercell-shaped workload (N=3000, R=32768, 128 occupied x 2000 unoccupied
    bands, split BF16): the direct sum at the 16-frequency mesh and at 64
    frequencies, and the spectral route at the 64 frequencies with 32, 64, 128
    and 256 log-spaced nodes over the transition energies; time of each call
    and the relative Frobenius difference from the direct sum per frequency.
    One JSON line."""
    import numpy as np
    import torch

    import gwsynth
    from paper_1003_0316_amd import binding as gw
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shp = gwsynth.SHAPES["c3"]
    inp = gwsynth.generate_torch(shp, dev, k_subset=[0, 1], log=log)
    n_occ = shp.n_occ
    om16 = np.asarray(inp.omega, dtype=np.float64)
    om64 = np.concatenate([[0.0], np.geomspace(0.01, 20.0, 63)])
    x_lo = inp.eps[1, n_occ:].min() - inp.eps[0, :n_occ].max()
    x_hi = inp.eps[1, n_occ:].max() - inp.eps[0, :n_occ].min()

    def timed(omega, nodes=None):
        call = gw.PolarizationCall(inp.U, inp.psi, inp.eps, omega, n_occ, precision="split_bf16", k_list=[0],
                                   nodes=nodes)
        ws = torch.empty(call.workspace_size(), dtype=torch.uint8, device=dev)
        call.run(ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        P = call.run(ws)
        e1.record()
        torch.cuda.synchronize()
        del ws
        return P, e0.elapsed_time(e1) / 1e3

    _, t16 = timed(om16)
    log(f"direct sum, 16 frequencies: {t16:.3f} s")
    Pd, t64 = timed(om64)
    log(f"direct sum, 64 frequencies: {t64:.3f} s")
    nd = torch.linalg.norm(Pd.reshape(om64.size, -1), dim=1)
    rows = []
    for B in (32, 64, 128, 256):
        nodes = np.geomspace(x_lo, x_hi, B)
        Ps, t = timed(om64, nodes)
        err = (torch.linalg.norm((Ps - Pd).reshape(om64.size, -1), dim=1) / nd).cpu().numpy()
        del Ps
        torch.cuda.empty_cache()
        rows.append({"nodes": B, "s": round(t, 3), "max_rel_diff": float(err.max()), "rel_diff_w0": float(err[0]),
                     "rel_diff_wmax": float(err[-1])})
        log(f"spectral route, {B} nodes: {t:.3f} s, max rel diff from the direct sum {err.max():.2e}")
    print(json.dumps({"metric": "spectral route vs direct sum, s per k-point and relative difference of P",
                      "unit": "s", "direct_16_freq_s": round(t16, 3), "direct_64_freq_s": round(t64, 3),
                      "spectral_64_freq": rows, "transition_energy_range": [float(x_lo), float(x_hi)],
                      "config": {"workload": "c3 shapes, k = 0 (unoccupied bands of set 1): N=3000, R=32768, "
                                             "128 x 2000 pairs", "precision": "split_bf16",
                                 "nodes": "log-spaced over the transition energies"}}))
    return 0


def surrogate_ablation(a) -> int:
    """Which part of the proposed correction carries the gain (training-run
    shapes: N=1000, R=8192, 64 + 1500 bands, 4 k-sets, 16 frequencies; the
    shipped model; held-out seeds; cutoffs 300 and 375).  Relative Frobenius
    error against the full-band P, per frequency, for
      truncation           P_ret
      diag_learned         P_ret - diag(d_hat)            d_hat = |P_ret,II| e^y
      diag_exact           P_ret - diag(d)                d the true missing diagonal
      congruence_learned   P_ret + D P_ret D              (the shipped surrogate, library kernels)
      congruence_exact     the same with D from d
      rank8_fitted         congruence_learned - X diag(c) X^H, X the 8 leading
                           eigenvectors of -P_ret, c >= 0 fitted to the true
                           residual (the best any learned rank-8 term of this form
                           can do)
      best_rank8           congruence_learned + the best rank-8 approximation of
                           the residual itself (the best any rank-8 term can do)
    The GPU computes P (split BF16) and the learned correction; the analysis
    (eigenvectors, fits) is FP64 NumPy on the host.  One JSON line."""
    import numpy as np
    import torch

    import gwsynth
    from paper_1003_0316_amd import binding as gw
    from paper_1003_0316_amd.surrogate import Surrogate
    from paper_1003_0316_amd.train_surrogate import SEED0, run_partials
    dev = torch.device("cuda:0")
    sur = Surrogate.load_default(dev)
    shp = gwsynth.SHAPES["c4train"]
    cuts = (300, 375)
    names = ["truncation", "diag_learned", "diag_exact", "congruence_learned", "congruence_exact", "rank8_fitted",
             "best_rank8"]
    errs = {c: {v: [] for v in names} for c in cuts}
    seeds = [gwsynth.BASE_SEED + SEED0 + 200 + i for i in range(a.ablation_seeds)]
    for s in seeds:
        inp, eps_dev, parts, P_full = run_partials(s, dev, cuts=cuts)
        Pf_all = P_full.cpu().numpy()
        n_om, N = Pf_all.shape[0], Pf_all.shape[1]
        for c in cuts:
            Pr_t = parts[c]
            Y, _ = sur.predict(Pr_t, eps_dev, inp.omega, shp.n_occ, c, inp.kq)
            y = Y[:, 0].double().clamp(-30.0, 30.0).cpu().numpy().reshape(n_om, N)
            Pc_t = Pr_t.clone()
            gw.gw_surrogate_apply(Pc_t, Y, sur.mlp.n_out)
            Pr_all, Pc_all = Pr_t.cpu().numpy(), Pc_t.cpu().numpy()
            rows = {v: [] for v in names}
            for j in range(n_om):
                pr, pf, pc = Pr_all[j], Pf_all[j], Pc_all[j]
                nf = np.linalg.norm(pf)
                err = lambda X: float(np.linalg.norm(X - pf) / nf)
                dr = np.real(np.diag(pr))
                d = dr - np.real(np.diag(pf))
                d_hat = np.abs(dr) * np.exp(y[j])
                Dx = np.sqrt(np.maximum(d, 0.0) / np.abs(dr))
                rows["truncation"].append(err(pr))
                rows["diag_learned"].append(err(pr - np.diag(d_hat)))
                rows["diag_exact"].append(err(pr - np.diag(d)))
                rows["congruence_learned"].append(err(pc))
                rows["congruence_exact"].append(err(pr + Dx[:, None] * pr * Dx[None, :]))
                Rs = pf - pc
                _, V = np.linalg.eigh(-pr)
                X = V[:, -8:]
                cf = np.maximum(-np.real(np.einsum("ia,ij,ja->a", X.conj(), Rs, X)), 0.0)
                rows["rank8_fitted"].append(err(pc - (X * cf) @ X.conj().T))
                er, Vr = np.linalg.eigh(Rs)
                idx = np.argsort(-np.abs(er))[:8]
                rows["best_rank8"].append(err(pc + (Vr[:, idx] * er[idx]) @ Vr[:, idx].conj().T))
            for v in names:
                errs[c][v].append(rows[v])
        log(f"seed {s}: cut 300 congruence {np.mean(errs[300]['congruence_learned'][-1]):.4f}, "
            f"rank8_fitted {np.mean(errs[300]['rank8_fitted'][-1]):.4f}, best_rank8 "
            f"{np.mean(errs[300]['best_rank8'][-1]):.4f}")
        del parts, P_full
        torch.cuda.empty_cache()
    out = {}
    for c in cuts:
        out[str(c)] = {v: {"mean": round(float(np.mean(e)), 5), "max": round(float(np.max(e)), 5),
                           "per_omega_mean": [round(float(x), 5) for x in np.mean(e, axis=0)]}
                       for v, e in errs[c].items()}
    print(json.dumps({"surrogate_ablation": out, "seeds": seeds,
                      "config": {"workload": "N_k=4, N=1000, R=8192, 64 occ + 1500 unocc bands, 16 imaginary "
                                             "frequencies (training-run shapes), held-out seeds",
                                 "precision": "split_bf16"}}))
    return 0


def mpb_bench(a) -> int:
    """Optimization of the product basis (keep v_mu >= v_min) on the
    training-run shapes (N_k=4, N=1000, R=8192, 64 + 1500 bands, 16
    frequencies): for each threshold, W for all 4 momentum transfers and
    Sigma_c(i w) of the highest occupied and lowest unoccupied band of set 0,
    split BF16 throughout; errors against the full basis.  One JSON line."""
    import numpy as np
    import torch

    import gwsynth
    from paper_1003_0316_amd import binding as gw
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shp = gwsynth.SHAPES["c4train"]
    inp = gwsynth.generate_torch(shp, dev, log=log)
    v_full = torch.from_numpy(inp.v).to(dev)
    mesh = inp.omega
    n_k = shp.n_k
    mu = 0.5 * (inp.eps[:, :shp.n_occ].max() + inp.eps[:, shp.n_occ:].min())
    states = [(0, shp.n_occ - 1), (0, shp.n_occ)]
    v_sorted = np.sort(inp.v)[::-1]
    rows = []
    ref = None
    # warm-up: one full-basis pass (library set-up and workspaces outside the timings)
    Ws = []
    for t in range(n_k):
        kq = (np.arange(n_k) + t) % n_k
        P = gw.gw_polarization(inp.U, inp.psi, inp.eps, mesh, shp.n_occ, precision="split_bf16", kq=kq)
        Ws.append(gw.gw_screen(P, v_full)[0])
        del P
    gw.gw_sigma_c(inp.U, inp.psi, inp.eps, Ws, v_full, mesh, mesh, states, mu, precision="split_bf16")
    torch.cuda.synchronize()
    del Ws
    for frac in (1.0, 0.8, 0.6, 0.45, 0.3, 0.2):
        n_keep = max(1, int(round(frac * shp.N)))
        v_min = 0.0 if frac == 1.0 else float(v_sorted[n_keep - 1])
        torch.cuda.synchronize()
        t0 = time.time()
        U, v, _ = gw.gw_basis_select(inp.U, v_full, v_min)
        Ws = []
        for t in range(n_k):
            kq = (np.arange(n_k) + t) % n_k
            P = gw.gw_polarization(U, inp.psi, inp.eps, mesh, shp.n_occ, precision="split_bf16", kq=kq)
            W, info = gw.gw_screen(P, v)
            del P
            Ws.append(W)
        sig = gw.gw_sigma_c(U, inp.psi, inp.eps, Ws, v, mesh, mesh, states, mu, precision="split_bf16")
        torch.cuda.synchronize()
        dt = time.time() - t0
        s = sig.cpu().numpy()
        if ref is None:
            ref = s
        err = float(np.max(np.abs(s - ref)) / np.max(np.abs(ref)))
        gap = float((s[1, 0] - s[0, 0]).real - (ref[1, 0] - ref[0, 0]).real)
        rows.append({"v_min": v_min, "sqrt_4pi_over_v_min": (float(np.sqrt(4 * np.pi / v_min)) if v_min > 0 else None),
                     "rank": int(U.shape[0]), "seconds": round(dt, 3), "sigma_rel_err": err,
                     "gap_sigma_change_Ha": gap, "gap_sigma_change_eV": gap * 27.211386})
        log(f"v_min {v_min:.3f}: rank {U.shape[0]}, {dt:.2f} s, Sigma rel err {err:.2e}, gap change {gap * 27.211:.4f} eV")
        del Ws, sig, U, v
        torch.cuda.empty_cache()
    out = {"metric": "Sigma_c(i w) error and time vs the Coulomb-eigenvalue threshold v_min",
           "unit": "s per (W for all transfers + Sigma_c of 2 states)", "n_gpus": 1,
           "data": "synthetic (seeded; training-run shapes)",
           "config": {"workload": "N_k=4, N=1000, R=8192, 64 occ + 1500 unocc bands, 16 imaginary frequencies",
                      "states": states, "precision": "split_bf16"},
           "rows": rows}
    print(json.dumps(out))
    return 0


def real_bench(a) -> int:
    """Real inputs (the inversion-symmetric case): the largest workload's shapes
    (N_k=4, N=6000, R=65536, 256 occupied bands, unoccupied bands 0..1499, 16
    frequencies) with U and the wave functions replaced by their real parts.
    Times one step of P (real split-BF16 path) + W, and the complex path on the
    same inputs and pairs; prints one JSON line."""
    import numpy as np
    import torch

    import gwsynth
    from paper_1003_0316_amd import binding as gw
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shp = gwsynth.SHAPES[a.workload]
    cutoff = a.cutoff or shp.n_unocc_cut or shp.n_unocc
    nb = shp.n_occ + cutoff
    inp = gwsynth.generate_torch(shp, dev, band_limit=nb, log=log)
    eps = np.ascontiguousarray(inp.eps[:, :nb])
    U_r = inp.U.real.contiguous()
    psi_r = inp.psi.real.contiguous()
    U_c = U_r.to(torch.complex64)
    psi_c = psi_r.to(torch.complex64)
    v = torch.from_numpy(inp.v).to(dev)
    mesh = inp.omega

    def run(real):
        call = gw.PolarizationCall(U_r if real else U_c, psi_r if real else psi_c, eps, mesh, shp.n_occ,
                                   precision="split_bf16", real=real)
        ws = gw.workspace(call.workspace_size(), dev, "real_bench")
        for _ in range(a.warmup):
            call.run(ws)
            gw.gw_screen(call.P, v)
        torch.cuda.synchronize()
        gw.gw_profile_reset()
        gw.gw_profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            call.run(ws)
            W, info = gw.gw_screen(call.P, v)
        e1.record()
        torch.cuda.synchronize()
        gw.gw_profile_enable(False)
        ms = e0.elapsed_time(e1) / a.steps
        kern = {k: gw.gw_profile_query(k) for k in ("project_bf16_kernel", "herk_bf16_kernel")}
        P = call.P
        return ms, kern, P

    ms_r, kern_r, P_r = run(True)
    imag_zero = bool(float(P_r.imag.abs().max()) == 0.0)
    sym_err = float((P_r - P_r.transpose(1, 2)).abs().max())
    del P_r
    torch.cuda.empty_cache()
    log(f"real path: {ms_r / 1e3:.3f} s/step")
    ms_c, kern_c, P_c = run(False)
    del P_c
    log(f"complex path on the same inputs: {ms_c / 1e3:.3f} s/step")
    T = shp.n_k * shp.n_occ * cutoff
    n_pr, t_pr = kern_r["project_bf16_kernel"]
    flops_real = 2.0 * shp.N * shp.R * T * a.steps          # one real multiply-add per (I, r, pair)
    achieved = flops_real / (t_pr * 1e-3) / 1e12
    out = {"metric": "P(q,iw) s/q-point, real inputs (inversion-symmetric), explicit bands to the cutoff",
           "value": round(ms_r / 1e3, 4), "unit": "s/q-point", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": round(ms_r, 2), "higher_is_better": False, "dtype": "bf16x3 (split hi/lo) real, fp32 acc",
           "data": "synthetic (seeded; paper-shaped; real parts of the generated U and wave functions)",
           "config": {"workload": f"{a.workload} shapes, real inputs, unoccupied bands 0..{cutoff - 1}",
                      "pairs": T, "step": "P (projection + accumulation) + W"},
           "complex_path_same_inputs_s": round(ms_c / 1e3, 4), "speedup_vs_complex": round(ms_c / ms_r, 2),
           "kernels_ms_per_step": {"real": {k: round(v[1] / a.steps, 1) for k, v in kern_r.items()},
                                   "complex": {k: round(v[1] / a.steps, 1) for k, v in kern_c.items()}},
           "roofline": {"bound": "mfma", "kernel": "project_bf16_kernel (real)", "achieved": round(achieved, 2),
                        "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_TFLOPS["bf16"], 4), "traffic": None,
                        "avg_launch_ms": round(t_pr / max(1, n_pr), 4), "launches": n_pr},
           "p_imag_exactly_zero": imag_zero, "p_symmetry_max_abs": sym_err}
    print(json.dumps(out))
    return 0


def sigma_bench(a) -> int:
    """Correlation self-energy (Eq. SEc_AC) on the supercell-shaped workload
    (N_k=8, N=3000, R=32768, 128 + 2000 bands, 16 imaginary frequencies):
    W(t) for all 8 momentum transfers (split-BF16 polarization, FP64
    screening), then Sigma_c(i w) at the 16 mesh frequencies for the highest
    occupied and the lowest unoccupied band of set 0, split BF16.  Prints one
    JSON line; the timed region is the self-energy call."""
    import numpy as np
    import torch

    import gwsynth
    from paper_1003_0316_amd import binding as gw
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shp = gwsynth.SHAPES["c3"]
    inp = gwsynth.generate_torch(shp, dev, log=log)
    v = torch.from_numpy(inp.v).to(dev)
    mesh = inp.omega
    n_k = shp.n_k
    t0 = time.time()
    Ws = []
    for t in range(n_k):
        kq = (np.arange(n_k) + t) % n_k
        P = gw.gw_polarization(inp.U, inp.psi, inp.eps, mesh, shp.n_occ, precision="split_bf16", kq=kq)
        W, info = gw.gw_screen(P, v)
        torch.cuda.synchronize()
        del P
        if int(info.abs().sum()) != 0:
            log(f"WARNING: screening reported non-positive pivots for transfer {t}")
        Ws.append(W)
        log(f"W for transfer {t} done")
    t_w = time.time() - t0
    mu = 0.5 * (inp.eps[:, :shp.n_occ].max() + inp.eps[:, shp.n_occ:].min())
    states = [(0, shp.n_occ - 1), (0, shp.n_occ)]
    call = gw.SigmaCall(inp.U, inp.psi, inp.eps, Ws, v, mesh, mesh, states, mu, precision="split_bf16")
    for _ in range(a.warmup):
        call.run()
    torch.cuda.synchronize()
    gw.gw_profile_reset()
    gw.gw_profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        sig = call.run()
    e1.record()
    torch.cuda.synchronize()
    gw.gw_profile_enable(False)
    ms = e0.elapsed_time(e1) / a.steps
    s_np = sig.cpu().numpy()
    n_wm, t_wm = gw.gw_profile_query("sigma_wm_kernel")
    n_pr, t_pr = gw.gw_profile_query("sigma_project_kernel")
    nb = shp.n_bands
    n_st = len(states)
    flops_wm = 8.0 * shp.N * shp.N * nb * len(mesh) * n_k * n_st * a.steps
    flops_pr = 8.0 * shp.N * shp.R * nb * n_k * n_st * a.steps
    achieved = flops_wm / (t_wm * 1e-3) / 1e12
    props = {"sigma_at_0_is_real": bool(np.all(np.abs(s_np[:, 0].imag) <= 1e-9 * np.abs(s_np[:, 0]))),
             "im_negative_for_w_gt_0": bool(np.all(s_np[:, 1:].imag < 0))}
    out = {"metric": "Sigma_c(i w) s/state (Eq. SEc_AC, all 8 momentum transfers, all 2128 bands, 16 frequencies)",
           "value": round(ms / 1e3 / n_st, 4), "unit": "s/state", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": round(ms, 2), "higher_is_better": False, "dtype": "bf16x3 (split hi/lo), fp32 acc, fp64 weights",
           "data": "synthetic (seeded; paper-shaped)",
           "config": {"workload": "c3: N_k=8, N=3000, R=32768, 128 occ + 2000 unocc bands, 16 imaginary frequencies",
                      "states": states, "mu": mu},
           "w_all_transfers_s": round(t_w, 2),
           "kernels_ms_per_step": {"sigma_wm_kernel": round(t_wm / a.steps, 2),
                                   "sigma_project_kernel": round(t_pr / a.steps, 2)},
           "roofline": {"bound": "mfma", "kernel": "sigma_wm_kernel", "achieved": round(achieved, 2),
                        "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_TFLOPS["bf16"], 4), "traffic": None,
                        "avg_launch_ms": round(t_wm / max(1, n_wm), 4),
                        "alg_flops_per_launch": flops_wm / max(1, n_wm), "launches": n_wm},
           "projection_tflops": round(flops_pr / (t_pr * 1e-3) / 1e12, 2) if t_pr > 0 else None,
           "sigma": [[[float(x.real), float(x.imag)] for x in row] for row in s_np],
           "properties": props}
    print(json.dumps(out))
    return 0


def _pmc_means(d: str, counter: str) -> dict:
    """mean counter value per dispatch, by kernel name, from rocprofv3 csv output"""
    import csv
    import glob
    acc = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "").replace("gw::(anonymous namespace)::", "")
                if name.startswith("void "):
                    name = name[len("void "):]
                key = name.split("(")[0]
                acc.setdefault(key, []).append(float(row["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize_pmc(a) -> int:
    fd, wd, cfd, cwd = a.summarize_pmc
    fetch, write = _pmc_means(fd, "FETCH_SIZE"), _pmc_means(wd, "WRITE_SIZE")
    cf, cw = _pmc_means(cfd, "FETCH_SIZE"), _pmc_means(cwd, "WRITE_SIZE")
    copy_f = max(cf.values()) if cf else None
    copy_w = max(cw.values()) if cw else None
    n = 1 << 30
    kf = n / (copy_f * 1024.0) if copy_f else None   # bytes per reported KiB
    kw = n / (copy_w * 1024.0) if copy_w else None
    out = {"workload": a.workload, "source_hash": kernel_source_hash(), "copy_factor_fetch": kf,
           "copy_factor_write": kw, "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        fb = fetch.get(k, 0.0) * 1024.0 * (kf or 1.0)
        wb = write.get(k, 0.0) * 1024.0 * (kw or 1.0)
        out["kernels"][k] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb}
    # the projection runs as the OUT_TILED instance (first template argument 0)
    # of the split-BF16 GEMM core: three-multiplication (gemm3r_: six plane
    # slots, gemm3m_: two stage buffers), or 4-wave (gemm_) / 8-wave (gemm8_)
    # four-product
    dom = next((k for k in out["kernels"] if re.match(r"(gemm3[rm]|gemm8?_bf16x3)_kernel<0[,>]", k)), None)
    if dom:
        out["kernel"] = "project_bf16_kernel"
        out["symbol"] = dom
        out["bytes_per_launch"] = out["kernels"][dom]["fetch_bytes_per_launch"] + \
            out["kernels"][dom]["write_bytes_per_launch"]
    with open(a.traffic or os.path.join(ROOT, "profiles", f"traffic_{a.workload}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
    return 0


def measured_traffic(traffic_file: str, kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from a counter summary written by
    --summarize-pmc, or None unless the summary is for this kernel and
    workload and was measured on the current GEMM sources (source hash)."""
    try:
        with open(traffic_file) as fh:
            tr = json.load(fh)
        if tr.get("kernel") == kernel and tr.get("source_hash") == kernel_source_hash() and \
                tr.get("workload") == workload:
            return float(tr["bytes_per_launch"])
    except (OSError, ValueError, KeyError, TypeError):
        pass
    return None


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("k_mfma.hip", "k_tiled.hip"):
        with open(os.path.join(ROOT, "paper_1003_0316_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _pairs_and_flops(shp, cutoff, n_om, sample_rows, fallback):
    """Algorithmic flops of one step: projection 8 N R per pair, Hermitian
    accumulation 4 N (N + 1) per pair and frequency, FP64 screening N^3 / 2
    complex multiply-adds per frequency; the judge's sample pairs are projected
    only."""
    N = shp.N
    T_main = shp.n_k * shp.n_occ * cutoff
    if fallback:
        T_main += shp.n_k * shp.n_occ * (shp.n_unocc - cutoff)
    T_sample = sample_rows * (shp.n_unocc - cutoff) if cutoff < shp.n_unocc else 0
    return T_main, T_sample, {
        "proj": 8.0 * N * shp.R * T_main, "acc": 4.0 * N * (N + 1) * T_main * n_om,
        "sample": 8.0 * N * shp.R * T_sample, "screen": 0.5 * N ** 3 * 8.0 * n_om}


def _block(P, S):
    """P[:, S][:, :, S] as a host array (S a device index tensor)."""
    return P[:, S][:, :, S].cpu().numpy()


def _norms(P):
    """Per frequency (||diag P||, ||P||_F) of a device [n_om][N][N] array."""
    import torch
    d = torch.linalg.vector_norm(torch.diagonal(P, dim1=1, dim2=2), dim=1)
    f = torch.stack([torch.linalg.vector_norm(P[j]) for j in range(P.shape[0])])
    return d.cpu().numpy(), f.cpu().numpy()


def _block_errors(x, ref, norms=None):
    """Relative errors of a sampled block [n_om][m][m] (rows = columns = the
    sampled basis functions): over the block, over its diagonal entries and
    over its off-diagonal entries; with the GPU matrix's own per-frequency
    diagonal and Frobenius norms, the estimate of the full-matrix relative
    Frobenius error sqrt(e_d^2 ||diag||^2 + e_o^2 ||off||^2) / ||P||, which
    weights diagonal and off-diagonal errors as the whole matrix does (a block
    alone over-weights the diagonal)."""
    import numpy as np
    m = x.shape[1]
    eye = np.eye(m, dtype=bool)
    d = x - ref
    blk = np.linalg.norm(d.reshape(d.shape[0], -1), axis=1) / np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    ed = np.linalg.norm(d[:, eye], axis=1) / np.linalg.norm(ref[:, eye], axis=1)
    eo = np.linalg.norm(d[:, ~eye], axis=1) / np.linalg.norm(ref[:, ~eye], axis=1)
    out = {"max_rel_fro_err": float(blk.max()), "per_omega": [float(v) for v in blk],
           "diag_per_omega": [float(v) for v in ed], "offdiag_per_omega": [float(v) for v in eo]}
    if norms is not None:
        D, F = norms
        O2 = np.maximum(F ** 2 - D ** 2, 0.0)
        est = np.sqrt(ed ** 2 * D ** 2 + eo ** 2 * O2) / F
        out["full_matrix_estimate_per_omega"] = [float(v) for v in est]
        out["full_matrix_estimate_max"] = float(est.max())
    return out


def _rel_per_omega(x, ref):
    """Relative Frobenius error per frequency of device arrays [n_om][..]."""
    import torch
    d = torch.linalg.vector_norm((x - ref).reshape(x.shape[0], -1), dim=1)
    r = torch.linalg.vector_norm(ref.reshape(ref.shape[0], -1), dim=1)
    return (d / r).cpu().numpy()


def _w_residual(P, W, v, S):
    """Per frequency ||W[S,:] - diag(v_S) P[S,:] W - diag(v)[S,:]||_F / ||v_S||:
    the sampled rows of (1 - vP) W = v (Eq. W_Dyson in matrix form)."""
    import torch
    out = []
    vs = v[S]
    for j in range(P.shape[0]):
        lhs = W[j][S] - vs[:, None] * (P[j][S].contiguous() @ W[j])
        lhs[torch.arange(S.numel(), device=S.device), S] -= vs
        out.append(float(torch.linalg.vector_norm(lhs) / torch.linalg.vector_norm(vs)))
    return out


def _diag_view(d):
    """A [n_om][N][N] read-only view whose (j, i, i) element is d[j, i] (no
    N x N storage): the oracle's feature function reads only the diagonal."""
    import numpy as np
    d = np.ascontiguousarray(d)
    return np.lib.stride_tricks.as_strided(d, shape=(d.shape[0], d.shape[1], d.shape[1]),
                                           strides=(d.strides[0], d.strides[1], 0), writeable=False)


def main() -> int:
    a = parse()
    if a.copy_calibration:
        return copy_calibration()
    if a.summarize_pmc:
        return summarize_pmc(a)
    if a.tuning:
        from paper_1003_0316_amd import binding as gw
        for kv in a.tuning:
            key, _, value = kv.partition("=")
            gw.gw_set_tuning(key, int(value))
            log(f"tuning {key} = {int(value)}")
    if a.sigma:
        return sigma_bench(a)
    if a.real:
        return real_bench(a)
    if a.mpb:
        return mpb_bench(a)
    if a.surrogate_ablation:
        return surrogate_ablation(a)
    if a.spectral:
        return spectral_bench(a)
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} is not supported: this build runs on one GPU only "
              f"(the k-point / occupied-band shards and the reduce-scatter of P over frequencies are "
              f"described in the design notes but not built)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import gwsynth
    from paper_1003_0316_amd import binding as gw

    shp = gwsynth.SHAPES[a.workload]
    cutoff = a.cutoff or shp.n_unocc_cut or shp.n_unocc
    learned_path = cutoff < shp.n_unocc
    surrogate = None
    if learned_path:
        from paper_1003_0316_amd import surrogate as sg
        if not os.path.exists(sg.DEFAULT_MODEL):
            print(f"bench.py: workload {a.workload} cuts the band sum at {cutoff} and needs the trained model "
                  f"{sg.DEFAULT_MODEL}, which is missing (no silent truncation)", file=sys.stderr)
            return 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"workload {a.workload}: N_k={shp.n_k} N={shp.N} R={shp.R} occ={shp.n_occ} unocc={shp.n_unocc} "
        f"cutoff={cutoff} precision={a.precision}")
    t0 = time.time()
    inp = gwsynth.generate_torch(shp, dev, log=log)
    torch.cuda.synchronize()
    log(f"inputs generated in {time.time() - t0:.1f} s")
    U, psi = inp.U, inp.psi
    eps_dev = torch.from_numpy(inp.eps).to(dev)
    v_dev = torch.from_numpy(inp.v).to(dev)
    n_om = inp.omega.shape[0]
    N = shp.N

    # ------------------------------------------------------------------ the step
    W = torch.empty((n_om, N, N), dtype=torch.complex128, device=dev)
    info = torch.empty(n_om, dtype=torch.int32, device=dev)
    sur_report = {}
    n_sample_occ = a.sample_occ
    if learned_path:
        surrogate = sg.Surrogate.load_default(dev, judge_tol=a.judge_tol)
        learned = surrogate.learned_call(U, psi, inp.eps, eps_dev, inp.omega, shp.n_occ, cutoff, inp.kq,
                                         precision=a.precision, n_sample_occ=n_sample_occ)
        learned.pol.desc.chunk_pairs = a.chunk_pairs
        P = learned.pol.P
        ws = torch.empty(learned.workspace_size(), dtype=torch.uint8, device=dev)

        def run_p():
            _, rep = learned.run(ws)
            sur_report.update(rep)
    else:
        pol = gw.PolarizationCall(U, psi, inp.eps, inp.omega, shp.n_occ, precision=a.precision, eps_dev=eps_dev,
                                  kq=inp.kq, unocc_range=(0, cutoff), chunk_pairs=a.chunk_pairs)
        P = pol.P
        ws = torch.empty(pol.workspace_size(), dtype=torch.uint8, device=dev)

        def run_p():
            pol.run(ws)

    def step():
        run_p()
        gw.gw_screen(P, v_dev, W=W, info=info)

    for i in range(a.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i} done")
    gw.gw_profile_reset()
    gw.gw_profile_enable(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tw0 = time.time()
    e0.record()
    for i in range(a.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.time() - tw0
    gw.gw_profile_enable(False)
    ms = e0.elapsed_time(e1) / a.steps
    log(f"timed {a.steps} step(s): {ms / 1e3:.3f} s/step (wall {wall:.1f} s)")
    info_h = info.cpu().numpy()
    screening_ok = bool(np.all(info_h == 0))
    if not screening_ok:
        log(f"ERROR: screening met non-positive pivots (eps not positive definite): info {info_h.tolist()}")
    fallback = bool(sur_report.get("used_fallback", False))

    pre = {"split_bf16": "bf16", "split_fp16": "f16", "fp16": "f16s", "fp32": "f32"}[a.precision]
    kernels = {}
    for name in (f"project_{pre}_kernel", f"herk_{pre}_kernel", "pair_product_kernel", "scale_split_kernel",
                 "update_kernel", "apply_kernel", "project_rows_bf16_kernel"):
        n, tot = gw.gw_profile_query(name)
        kernels[name] = {"launches": n, "total_ms": tot}
    sample_rows = shp.n_k * n_sample_occ if learned_path else 0
    T_main, T_sample, fl = _pairs_and_flops(shp, cutoff, n_om, sample_rows, fallback)
    per_step = {f"project_{pre}_kernel": fl["proj"], f"herk_{pre}_kernel": fl["acc"], "update_kernel": fl["screen"],
                "project_rows_bf16_kernel": fl["sample"] if a.precision == "split_bf16" else 0.0,
                "pair_product_kernel": 0.0, "scale_split_kernel": 0.0, "apply_kernel": 0.0}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dk = kernels[dom]
    avg_ms = dk["total_ms"] / max(1, dk["launches"])
    alg_per_launch = per_step[dom] * a.steps / max(1, dk["launches"])
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e12
    peak_dtype = "fp64" if dom == "update_kernel" else {"bf16": "bf16", "f16": "fp16", "f16s": "fp16", "f32": "fp32"}[pre]
    traffic = measured_traffic(a.traffic or os.path.join(ROOT, "profiles", f"traffic_{a.workload}.json"), dom,
                               a.workload)
    roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": PEAK_TFLOPS[peak_dtype],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[peak_dtype], 4), "traffic": traffic,
                "avg_launch_ms": round(avg_ms, 4), "alg_flops_per_launch": alg_per_launch,
                "launches": dk["launches"]}
    if traffic is not None:
        roofline["hbm_gbs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
        roofline["hbm_frac"] = round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_GBS, 4)
    if pre in ("bf16", "f16") and dom != "update_kernel":
        # a split product executes three 16-bit MFMA products per algorithmic
        # one; the three-multiplication core forms a complex product from 3
        # real products where the algorithmic count has 4
        xf = 3.0
        if pre == "bf16" and gw.gw_get_tuning("complex_product") == 3:
            xf *= 0.75
            roofline["complex_product"] = "three real products per complex product"
        roofline["executed_tflops"] = round(xf * achieved, 2)
        roofline["executed_frac"] = round(xf * achieved / PEAK_TFLOPS[peak_dtype], 4)
    breakdown = {k: round(v["total_ms"] / a.steps / 1e3, 4) for k, v in kernels.items()}
    log(f"kernels (s/step): {breakdown}; dominant {dom} at {achieved:.1f} TFLOP/s")

    # ----------------------------------------------------------- W check (a7)
    # 32 sampled basis functions spread over the basis (rows and columns of the checked blocks)
    S = np.array(sorted(set([0, 1, 2, 17, N // 3, N // 2, N - 2, N - 1] + list(range(100, 108)) +
                            [3, 5, 33, 64, 200, N // 7, N // 5, N // 4, (2 * N) // 5, (3 * N) // 5, (2 * N) // 3,
                             (3 * N) // 4, (4 * N) // 5, (6 * N) // 7, N - 9, N - 3])))
    S = S[S < N]
    Sg = torch.from_numpy(S).to(dev)
    w_res = _w_residual(P, W, v_dev, Sg)
    log(f"W residual of (1 - vP) W = v on {S.size} sampled rows: max {max(w_res):.2e}")
    P_step_blk = _block(P, Sg)
    step_norms = _norms(P)

    # --------------------------------------------- learned path: model error (A19 ii)
    model = None
    P_ret_blk = None
    y_gpu_free = None
    if learned_path and not a.no_model_error:
        tm = time.time()
        pret = gw.PolarizationCall(U, psi, inp.eps, inp.omega, shp.n_occ, precision=a.precision, eps_dev=eps_dev,
                                   kq=inp.kq, unocc_range=(0, cutoff))
        wsr = torch.empty(pret.workspace_size(), dtype=torch.uint8, device=dev)
        C = pret.run(wsr)
        rest = gw.PolarizationCall(U, psi, inp.eps, inp.omega, shp.n_occ, precision=a.precision, eps_dev=eps_dev,
                                   kq=inp.kq, unocc_range=(cutoff, shp.n_unocc))
        del wsr
        wsr = torch.empty(rest.workspace_size(), dtype=torch.uint8, device=dev)
        B = rest.run(wsr)
        torch.cuda.synchronize()
        del wsr
        t_all = time.time() - tm
        P_ret_blk = _block(C, Sg)
        p_ret_diag = torch.diagonal(C, dim1=1, dim2=2).real.cpu().numpy()
        B.add_(C)                                    # the all-band sum, same path
        trunc = _rel_per_omega(C, B)
        corr = _rel_per_omega(P, B) if not fallback else np.zeros(n_om)
        del C
        P_all_blk = _block(B, Sg)
        del B
        torch.cuda.empty_cache()
        model = {"corrected_vs_all_bands_per_omega": [float(x) for x in corr],
                 "corrected_vs_all_bands_max": float(corr.max()), "corrected_vs_all_bands_mean": float(corr.mean()),
                 "truncation_per_omega": [float(x) for x in trunc], "truncation_max": float(trunc.max()),
                 "truncation_mean": float(trunc.mean()),
                 "reference": f"explicit sum over all {shp.n_unocc} unoccupied bands on the same {a.precision} "
                              f"path, outside the timed region ({t_all:.0f} s)",
                 "meets_1e-4": bool(corr.max() <= 1e-4)}
        log(f"model error vs all bands: max {corr.max():.4f} mean {corr.mean():.4f} (truncation alone: max "
            f"{trunc.max():.4f} mean {trunc.mean():.4f}); all-band pass {t_all:.0f} s")

    # ------------------------------------------------- FP32 plain path, all bands
    compare = None
    if not a.no_compare:
        if a.fp32_full:
            # every pair of the q-point, one k-point per call (the sum accumulates), each call timed
            occ_s, scale = shp.n_occ, 1.0
            sample_txt = "all k-points, all occupied x all unoccupied bands (not extrapolated)"
            cms = 0.0
            P32 = torch.empty((n_om, N, N), dtype=torch.complex128, device=dev)
            for k in range(shp.n_k):
                call_k = gw.PolarizationCall(U, psi, inp.eps, inp.omega, shp.n_occ, precision="fp32",
                                             eps_dev=eps_dev, kq=inp.kq, k_list=[k], P=P32, accumulate=k > 0)
                cws = torch.empty(call_k.workspace_size(), dtype=torch.uint8, device=dev)
                c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                c0.record()
                call_k.run(cws)
                c1.record()
                torch.cuda.synchronize()
                cms += c0.elapsed_time(c1)
                log(f"fp32 plain path, k-point {k}: {c0.elapsed_time(c1) / 1e3:.1f} s")
                del cws, call_k
            del P32
        else:
            occ_s = 4 if a.workload == "c5" else 8
            cmp_call = gw.PolarizationCall(U, psi, inp.eps, inp.omega, shp.n_occ, precision="fp32", eps_dev=eps_dev,
                                           kq=inp.kq, k_list=[0], occ_range=(0, occ_s))
            scale = shp.n_k * shp.n_occ / occ_s
            sample_txt = f"k=0, occupied 0..{occ_s - 1}, all {shp.n_unocc} unoccupied, scaled x{scale:g}"
            cws = torch.empty(cmp_call.workspace_size(), dtype=torch.uint8, device=dev)
            cmp_call.run(cws)
            torch.cuda.synchronize()
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record()
            cmp_call.run(cws)
            c1.record()
            torch.cuda.synchronize()
            cms = c0.elapsed_time(c1)
            del cws, cmp_call
        pairs = (shp.n_k if a.fp32_full else 1) * occ_s * shp.n_unocc
        fl32 = 8.0 * N * shp.R * pairs + 4.0 * N * (N + 1) * pairs * n_om
        fp32_s = cms / 1e3 * scale
        compare = {"fp32_plain_all_bands_s_per_qpoint": round(fp32_s, 2), "sample": sample_txt,
                   "fp32_tflops": round(fl32 / cms / 1e9, 1),
                   "fp32_frac_of_fp32_mfma_peak": round(fl32 / cms / 1e9 / PEAK_TFLOPS["fp32"], 4),
                   "speedup_vs_fp32_plain": round(fp32_s / (ms / 1e3), 2)}
        log(f"fp32 plain path: {fp32_s:.1f} s/q-point ({'measured in full' if a.fp32_full else 'extrapolated'}), "
            f"{fl32 / cms / 1e9:.1f} TFLOP/s")
        torch.cuda.empty_cache()

    # ------------------------------------------------------------ oracle legs
    parity = {"w_residual_per_omega": w_res, "w_residual_max": max(w_res),
              "w_check": f"rows S of (1 - vP) W = v, |S|={S.size}, relative to ||v_S||"}
    cpu = None
    if not a.no_cpu:
        from oracle import polarization as orc
        kk = int(inp.kq[0])
        occ_p = 2
        U_S = U[Sg].cpu().numpy().astype(np.complex128)
        # explicit bands, 2 occupied bands of k = 0: GPU pass vs oracle on the sampled block
        par = gw.PolarizationCall(U, psi, inp.eps, inp.omega, shp.n_occ, precision=a.precision, eps_dev=eps_dev,
                                  kq=inp.kq, k_list=[0], occ_range=(0, occ_p), unocc_range=(0, cutoff))
        pws = torch.empty(par.workspace_size(), dtype=torch.uint8, device=dev)
        Pk = par.run(pws)
        Pblk = _block(Pk, Sg)
        nrm = _norms(Pk)
        del pws, par, Pk
        psi_h = np.zeros((shp.n_k, shp.n_bands, shp.R), dtype=np.complex64)  # only the needed rows are filled
        psi_h[0, :occ_p] = psi[0, :occ_p].cpu().numpy()
        psi_h[kk, shp.n_occ:] = psi[kk, shp.n_occ:].cpu().numpy()
        tp = time.time()
        Pref = orc.polarization(U_S, psi_h, inp.eps, inp.omega, shp.n_occ, kq=inp.kq, k_list=[0],
                                occ_range=(0, occ_p), unocc_range=(0, cutoff))
        be = _block_errors(Pblk, Pref, nrm)
        parity["explicit_bands"] = {**be, "sample": f"P[I,J] for |S|={S.size} sampled I,J, k=0, occupied 0..{occ_p - 1}, "
                                                    f"unoccupied 0..{cutoff - 1}, all {n_om} frequencies",
                                    "oracle_s": round(time.time() - tp, 1)}
        parity["max_rel_fro_err"] = max(be["max_rel_fro_err"], be["full_matrix_estimate_max"])
        log(f"sampled parity vs oracle (explicit bands): block {be['max_rel_fro_err']:.2e}, off-diagonal "
            f"{max(be['offdiag_per_omega']):.2e}, full-matrix estimate {be['full_matrix_estimate_max']:.2e}")
        if learned_path:
            # the left-out bands on the same block (the all-band reference's other part)
            par = gw.PolarizationCall(U, psi, inp.eps, inp.omega, shp.n_occ, precision=a.precision,
                                      eps_dev=eps_dev, kq=inp.kq, k_list=[0], occ_range=(0, occ_p),
                                      unocc_range=(cutoff, shp.n_unocc))
            pws = torch.empty(par.workspace_size(), dtype=torch.uint8, device=dev)
            Pk = par.run(pws)
            Pblk = _block(Pk, Sg)
            nrm = _norms(Pk)
            del pws, par, Pk
            Pref = orc.polarization(U_S, psi_h, inp.eps, inp.omega, shp.n_occ, kq=inp.kq, k_list=[0],
                                    occ_range=(0, occ_p), unocc_range=(cutoff, shp.n_unocc))
            be = _block_errors(Pblk, Pref, nrm)
            parity["left_out_bands"] = {**be, "sample": f"as above, unoccupied {cutoff}..{shp.n_unocc - 1}"}
            parity["max_rel_fro_err"] = max(parity["max_rel_fro_err"], be["max_rel_fro_err"],
                                            be["full_matrix_estimate_max"])
            log(f"sampled parity vs oracle (left-out bands): block {be['max_rel_fro_err']:.2e}, full-matrix "
                f"estimate {be['full_matrix_estimate_max']:.2e}")
            if not fallback and P_ret_blk is not None:
                # the correction step on the GPU's own P_ret (A19 (i)): oracle features from its
                # diagonal, FP64 perceptron with the same BF16-valued weights, congruence on the block
                from oracle import mlp as omlp
                from oracle import surrogate as osg
                from oracle.precision import round_bf16
                prm = surrogate.mlp.to_dict()
                for k in ("W1", "W2", "W3"):
                    prm[k] = round_bf16(prm[k]).astype(np.float64)
                X = osg.features(_diag_view(p_ret_diag.astype(np.complex128)), inp.eps, inp.omega, shp.n_occ,
                                 cutoff, inp.kq, n_in=surrogate.mlp.n_in)
                y = omlp.forward(prm, X)[:, 0].reshape(n_om, N)
                ref = osg.apply(P_ret_blk, y[:, S].reshape(-1))
                be = _block_errors(P_step_blk, ref, step_norms)
                err = np.array([be["max_rel_fro_err"], be["full_matrix_estimate_max"]])
                parity["correction_step"] = {**be,
                                             "sample": "the step's corrected P on the block against the oracle's "
                                                       "features, FP64 perceptron and congruence applied to the "
                                                       "GPU's explicit-band P"}
                parity["max_rel_fro_err"] = max(parity["max_rel_fro_err"], float(err.max()))
                log(f"correction step vs oracle: max rel err {err.max():.2e}")
        # cpu baseline: the oracle on one occupied band x m unoccupied bands (full basis)
        U_h = U.cpu().numpy().astype(np.complex128)
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        blas = "unknown BLAS"
        try:   # the oracle's products run in NumPy's BLAS: report its thread count
            import threadpoolctl
            pools = [p for p in threadpoolctl.threadpool_info() if p.get("user_api") == "blas"]
            if pools:
                cores = max(int(p["num_threads"]) for p in pools)
                blas = f"{pools[0].get('internal_api')} BLAS, {cores} threads"
        except ImportError:
            pass

        def oracle_time(m):
            tc = time.time()
            orc.polarization(U_h, psi_h, inp.eps, inp.omega, shp.n_occ, kq=inp.kq, k_list=[0], occ_range=(0, 1),
                             unocc_range=(0, m))
            return time.time() - tc
        ta, tb = oracle_time(4), oracle_time(16)
        per_pair = max((tb - ta) / 12.0, 1e-4)
        want = max(16, int((a.cpu_seconds - ta) / per_pair))
        o2 = int(min(occ_p, max(1, -(-want // cutoff))))     # occupied bands in the sample
        m2 = int(min(cutoff, max(16, -(-want // o2))))       # unoccupied bands per occupied band
        tc = time.time()
        orc.polarization(U_h, psi_h, inp.eps, inp.omega, shp.n_occ, kq=inp.kq, k_list=[0], occ_range=(0, o2),
                         unocc_range=(0, m2))
        dt2 = time.time() - tc
        T_pairs = shp.n_k * shp.n_occ * cutoff
        scale = T_pairs / (o2 * m2)
        cpu = {"value": round(dt2 * scale, 1), "unit": "s/q-point", "cores": cores, "kind": "oracle",
               "sample": f"k=0, occupied 0..{o2 - 1} x unoccupied 0..{m2 - 1} ({o2 * m2} pairs, full basis, all "
                         f"{n_om} frequencies) in {dt2:.1f} s ({blas}), scaled x{scale:.0f} to the {T_pairs} "
                         f"explicit pairs of a q-point"}
        log(f"cpu oracle: {dt2:.1f} s for {o2 * m2} pairs -> {dt2 * scale:.0f} s/q-point extrapolated")
        del U_h

    numeric_ok = (None if "max_rel_fro_err" not in parity
                  else parity["max_rel_fro_err"] <= 1e-4 and max(w_res) <= 1e-8 and screening_ok)
    out = {
        "metric": "P(q,iw) s/q-point: split-BF16+surrogate vs FP32 plain @ rel err<=1e-4",
        "value": round(ms / 1e3, 4),
        "unit": "s/q-point",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 2),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": {"split_bf16": "bf16x3 (split hi/lo), fp32 acc, fp64 P/W", "split_fp16": "fp16x3 (split), fp32 acc",
                  "fp16": "fp16 (single, ablation), fp32 acc", "fp32": "fp32"}[a.precision],
        "data": "synthetic (seeded; paper-shaped)",
        "config": {"workload": f"{a.workload}: N_k={shp.n_k}, N={N}, R={shp.R}, {shp.n_occ} occ + {shp.n_unocc} "
                               f"unocc bands, {n_om} imaginary frequencies, explicit bands to {cutoff}",
                   "precision": a.precision, "surrogate": learned_path,
                   "surrogate_judge": ({**sur_report, "n_sample_occ": n_sample_occ, "judge_tol": a.judge_tol}
                                       if learned_path else None),
                   "step": ("P (explicit bands, learned correction, judge sample) + W (FP64 screening)"
                            if learned_path else "P (all bands) + W (FP64 screening)"),
                   **({"tuning": a.tuning} if a.tuning else {}),
                   **({"chunk_pairs": a.chunk_pairs} if a.chunk_pairs else {})},
        "pairs_per_step": {"explicit": T_main, "judge_sample_projected": T_sample},
        "kernels_s_per_step": breakdown,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp32_compare": compare,
        "parity": parity,
        "model_error": model,
        "rel_err_bar_met": {"numeric_parity_vs_oracle": numeric_ok,
                            "model_vs_all_bands": (model["meets_1e-4"] if model else None)},
        "screening_ok": screening_ok,
    }
    print(json.dumps(out))
    return 0 if screening_ok else 3


if __name__ == "__main__":
    sys.exit(main())
