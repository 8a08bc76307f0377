"""Precision study of the phase estimators (paper section 4.2).

Runs QPE for every eigenvector of one target matrix as a batch of instances,
for a list of measurement-register sizes, and reports how far each estimator
lands from the true eigenphases: the max-norm estimator (argmax / 2^n), the
weighted average as the paper states it, and the circular mean. Everything
runs on the device through the C ABI (qpe_run, then qpe_estimate); only the
final error table is formed on the host.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np
import torch

from . import qpe


def circular_distance(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Distance of phases on the unit circle, in [0, 1/2]."""
    e = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) % 1.0
    return np.minimum(e, 1.0 - e)


def precision_study(U: torch.Tensor, psis: Sequence[torch.Tensor], phis: np.ndarray, n_list: Sequence[int],
                    form="mixed", flags: int = 0) -> List[Dict]:
    """One row per n: mean and max error of each estimator over the inputs.

    U: device complex128 (d, d); psis: device complex128 (d,) inputs whose
    exact eigenphases are phis (same order)."""
    phis = np.asarray(phis, dtype=np.float64)
    rows = []
    for n in n_list:
        probs = qpe.run_batch([(U, psi, int(n)) for psi in psis], form=form, flags=flags)
        est = qpe.estimate(probs)
        e_arg = circular_distance(est["argmax_phase"], phis)
        e_wgt = np.abs(est["weighted_phase"] - phis)  # the paper's plain |difference|
        e_wgt_c = circular_distance(est["weighted_phase"], phis)
        e_cir = circular_distance(est["circular_phase"], phis)
        rows.append({
            "n_meas": int(n),
            "instances": len(psis),
            "argmax_mean": float(e_arg.mean()), "argmax_max": float(e_arg.max()),
            "weighted_mean": float(e_wgt.mean()), "weighted_max": float(e_wgt.max()),
            "weighted_circular_mean": float(e_wgt_c.mean()),
            "circular_mean": float(e_cir.mean()), "circular_max": float(e_cir.max()),
            "prob_sum_min": float(est["prob_sum"].min()), "prob_sum_max": float(est["prob_sum"].max()),
        })
        del probs
    return rows


def halving_slope(rows: List[Dict], key: str = "argmax_mean") -> float:
    """Least-squares slope of log2(error) against n: -1 means the error
    halves per extra measurement qubit."""
    n = np.array([r["n_meas"] for r in rows], dtype=np.float64)
    e = np.log2(np.array([r[key] for r in rows], dtype=np.float64))
    A = np.vstack([n, np.ones_like(n)]).T
    return float(np.linalg.lstsq(A, e, rcond=None)[0][0])


def scaling_sweep(cases: Sequence[Dict], forms=("mixed", "fp64"), flags: int = 0, reps: int = 3) -> List[Dict]:
    """Time per circuit and memory against the total qubit count (the paper's
    section 4.1 sweeps, which use matrices with known eigenphases).

    cases: dicts with keys U, psi (device complex128), n (measurement
    qubits) and, optionally, peak (the outcome index that must carry all the
    probability). One row per (case, form): median time of `reps` circuits
    after one warm-up, the exact workspace the library asked for, the peak
    device memory the process held during the run, and the double-precision
    statevector size 16 * 2^(n + t) the paper plots as the lower bound."""
    rows = []
    for c in cases:
        U, psi, n = c["U"], c["psi"], int(c["n"])
        t = U.shape[0].bit_length() - 1
        for form in forms:
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats()
            base = torch.cuda.memory_allocated()
            need = qpe.workspace_bytes([(n, t)], form, flags)
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=U.device)
            P = qpe.run_batch([(U, psi, n)], form=form, flags=flags, workspace=ws)[0]
            torch.cuda.synchronize()
            times = []
            for _ in range(reps):
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record()
                P = qpe.run_batch([(U, psi, n)], form=form, flags=flags, workspace=ws)[0]
                ev1.record()
                torch.cuda.synchronize()
                times.append(ev0.elapsed_time(ev1))
            peak = torch.cuda.max_memory_allocated() - base
            row = {"n_total": n + t, "n_meas": n, "n_mat": t, "form": form,
                   "ms_per_circuit": round(float(np.median(times)), 4),
                   "workspace_bytes": int(need), "peak_device_bytes": int(peak),
                   "fp64_statevector_bytes": int(16 << (n + t)),
                   "peak_over_fp64_statevector": round(peak / float(16 << (n + t)), 4)}
            if c.get("peak") is not None:
                Ph = P.cpu().numpy()
                k = int(c["peak"])
                row["prob_at_peak"] = float(Ph[k])
                Ph[k] -= 1.0
                row["max_abs_err_vs_exact"] = float(np.abs(Ph).max())
            rows.append(row)
            del ws, P
    return rows
