"""QPE throughput benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config c2] [--no-cpu-baseline]

A step is one QPE circuit (Hadamard layer, FP64 powers with Newton-Schulz,
controlled products, inverse QFT, readout) through libqpe's qpe_run, with
U, psi and the workspace already resident in HBM. Workload (default):
N_meas = 16, N_mat = 10, a seeded 1024 x 1024 Haar unitary with a uniform
eigenphase and its eigenvector as input (2^26 amplitudes), in the mixed form
(complex64 state, split-FP16 matrix-core products with FP32 accumulation,
FP64 powers); the plain FP64 form is timed beside it.

Prints one JSON line. `value` = mixed-form circuits/s. `roofline` covers the
dominant kernel (the controlled-product GEMM): algorithmic flops per launch
8 * (N/2) * d^2 over its average launch time measured with HIP events on
the stream it runs on, against the dense FP16/BF16 matrix-core peak. Beside
it: the FP64 form, the prefix-doubling form, the split-BF16 scheme, and
`batched_c4`, the 512-instance batch (graph-replayed) in the mixed and FP64
forms. The CPU baseline is the oracle (numpy/scipy, complex128) on one full
circuit of the same workload, which also yields the run's max
|P_gpu - P_oracle|.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_F16_TFLOPS = 2500.0  # dense FP16 and BF16 matrix cores
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3  # FP32 vector ALUs
PEAK_HBM_GBS = 8000.0

# "dtype" is the matrix-core type of the dominant kernel; the whole path:
DTYPE_DETAIL = ("split-FP16 x3 products (two FP16 pieces per operand, FP32 accumulate) for the state GEMMs, "
                "FP32 QFT, FP64 powers, target rotation and readout")
# executed matrix-core flops per algorithmic flop of each split scheme
EXECUTED = {"split_fp16x3": 3, "split_bf16x6": 6}

# HBM bytes per launch of the controlled-product kernel at n = 16, t = 10,
# from two rocprofv3 --pmc passes (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, the
# factors a plain 1 GiB copy gives), keyed by the first 16 hex digits of the
# SHA-256 of the kernel source the counters were taken on. A changed kernel
# reports traffic null until it is measured again.
TRAFFIC = {
    "b0319bf79149ce9f": {"fetch_bytes": 262303.6 * 2.0 * 1024, "write_bytes": 262144.0 * 1024,
                         "profile": "profiles/ctrl_f16x3_qpe_n16_t10_hbm.md"},
}
CTRL_SRC = os.path.join(ROOT, "paper_2507_17175_amd", "csrc", "k_ctrl_mixed.hip")
# variants of the split-FP16 controlled product that run the kernel whose
# counters TRAFFIC holds at n = 16, t = 10 (the persistent wide ping-pong
# kernel: the built-in choice there, variant 9, and the BF16-only designs
# 3-6, which fall back to it)
TRAFFIC_VARIANTS = (0, 3, 4, 5, 6, 9)
CTRL_KERNELS = {1: "k_ctrl_f16x3<128,128>", 2: "k_ctrl_f16x3_db<128,128>", 7: "k_ctrl_f16x3_pp2<128,128>",
                8: "k_ctrl_f16x3_pp2<128,256>"}
CTRL_DEFAULT = "k_ctrl_f16x3_pp2p<128,256>"


def traffic_for_current_kernel():
    import hashlib
    try:
        h = hashlib.sha256(open(CTRL_SRC, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    rec = TRAFFIC.get(h)
    if rec is None:
        return None
    return {"bytes_per_launch": rec["fetch_bytes"] + rec["write_bytes"], "fetch_bytes": rec["fetch_bytes"],
            "write_bytes": rec["write_bytes"], "source": rec["profile"]}


CONFIGS = {
    "c1": "qpe-n8-t2 (Haar 4x4, exact-bit eigenphase k/256, eigenvector input)",
    "c2": "qpe-n16-t10 (Haar 1024x1024, uniform eigenphase, eigenvector input)",
    "c3": "qpe-n20-t8 (Haar 256x256, 3 eigenphases within 2^-18, superposed eigenvectors)",
    "c4": "qpe-batch-512 (512 instances, t uniform in 3..8, n uniform in 8..16, Haar, eigenvector inputs)",
    "c5": "qpe-n18-t14 (Haar 16384x16384, uniform eigenphase, eigenvector input; 2^32 amplitudes)",
}


def measure_batch(qpe, torch, probs, steps, warmup, autotune=True):
    """A batched workload: all instances in one qpe_run (grouped launches),
    the batch autotuner first (a few batched runs per variant, outside the
    timed region), then timed eagerly and as a replayed HIP graph; the same
    batch in the FP64 form beside it (replayed graph). Each instance's P is
    checked against the Fejer closed form of its eigenphase (eigenvector
    inputs)."""
    import oracle.qpe_oracle as O
    items = [(torch.from_numpy(p.U).cuda(), torch.from_numpy(p.psi).cuda(), p.n_meas) for p in probs]
    run = qpe.Runner(items, form="mixed")
    tuned = run.autotune(reps=2) if autotune else None
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    run.ctx.enable_timing(400 * steps + 512)
    run.ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    timing = run.ctx.read_timing()
    run.ctx.reset_timing()
    graph = qpe.CapturedRun(run)
    t0 = time.perf_counter()
    for _ in range(steps):
        graph()
    torch.cuda.synchronize()
    el_g = time.perf_counter() - t0
    rep = run.reports()
    P_mixed = [P.cpu().numpy() for P in run.probs]
    run64 = qpe.Runner(items, form="fp64")
    run64()
    torch.cuda.synchronize()
    graph64 = qpe.CapturedRun(run64)
    steps64 = max(2, steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps64):
        graph64()
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t0
    P64 = [P.cpu().numpy() for P in run64.probs]
    dP = max(float(np.abs(a - b).max()) for a, b in zip(P64, P_mixed))
    err_mixed = max(float(np.abs(Pm - O.fejer(p.phis[0], p.n_meas)).max()) for p, Pm in zip(probs, P_mixed))
    err_fp64 = max(float(np.abs(Pf - O.fejer(p.phis[0], p.n_meas)).max()) for p, Pf in zip(probs, P64))
    count = len(probs)
    flops = sum(4.0 * p.n_meas * (1 << p.n_meas) * (1 << p.n_mat) ** 2 for p in probs)
    g_cnt, g_ms = timing["ctrl_gemm"]
    mixed_cps = count * steps / el_g
    fp64_cps = count * steps64 / el64
    del graph, graph64, run, run64, items
    return {
        "instances": count, "steps": steps,
        "circuits_per_s": round(mixed_cps, 2), "ms_per_batch": round(1e3 * el_g / steps, 3),
        "eager_ms_per_batch": round(1e3 * el / steps, 3),
        "fp64_form": {"circuits_per_s": round(fp64_cps, 2), "ms_per_batch": round(1e3 * el64 / steps64, 3),
                      "steps": steps64, "max_abs_err_vs_fejer": err_fp64},
        "mixed_over_fp64": round(mixed_cps / fp64_cps, 3),
        "max_abs_err_mixed_vs_fejer": err_mixed,
        "max_abs_dP_mixed_vs_fp64": dP,
        "ctrl_gemm": {"algorithmic_flops_per_batch": flops, "ms_per_batch": round(g_ms / steps, 3),
                      "achieved_tflops": round(flops / (g_ms / steps / 1e3) / 1e12, 2),
                      "frac_of_f16_peak": round(flops / (g_ms / steps / 1e3) / 1e12 / PEAK_F16_TFLOPS, 4),
                      "launches_per_batch": g_cnt // steps},
        "breakdown": {k: {"launches": c // steps, "ms_per_batch": round(ms / steps, 4)}
                      for k, (c, ms) in timing.items()},
        "reports": {"flags_nonzero": int(np.count_nonzero(rep["flags"])),
                    "max_abs_prob_sum_minus_1": float(np.abs(rep["prob_sum"] - 1.0).max()),
                    "max_input_peak": float(rep["input_peak"].max())},
        "autotune": tuned,
        "graph": True,
    }


def bench_batch(a, qpe, torch, config_problems):
    """--config c4: the batched workload as the headline line."""
    probs = config_problems(a.config)
    b = measure_batch(qpe, torch, probs, a.steps, a.warmup, autotune=not a.no_autotune)
    out = {
        "metric": "QPE circuits/s (mixed form, batched)",
        "value": b["circuits_per_s"],
        "unit": "circuits/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": b["ms_per_batch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp16", "dtype_detail": DTYPE_DETAIL,
        "data": "synthetic (seeded Haar unitaries, eigenvector inputs)",
        "config": {"workload": CONFIGS[a.config], "instances": b["instances"], "form": "mixed", "graph": True},
        "batched": b,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_c5(a, qpe, torch):
    """The VRAM-scale workload (2^32 amplitudes, 32 GiB complex64 state,
    ~80 GiB of workspace): one mixed-form circuit takes tens of seconds, so
    it runs --steps circuits (default 1) without the autotuner, the FP64 form
    or the CPU oracle, plus one prefix-doubling circuit."""
    from workloads import config5_device

    t0 = time.perf_counter()
    U, psi, phi0, n, t = config5_device()
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    print(json.dumps({"progress": "c5 inputs generated", "seconds": round(gen_s, 1)}), file=sys.stderr, flush=True)
    N, d = 1 << n, 1 << t
    prob = {"U": U, "psi": psi, "n": n}
    steps = a.steps
    el, timing, rep, P = time_form(qpe, torch, prob, "mixed", steps, a.warmup)
    print(json.dumps({"progress": "c5 gate route timed", "seconds": round(el, 1)}), file=sys.stderr, flush=True)
    flops_per_launch = 8.0 * (N // 2) * d * d
    g_cnt, g_ms = timing["ctrl_gemm"]
    avg_s = (g_ms / g_cnt) / 1e3
    achieved = flops_per_launch / avg_s / 1e12
    el_d, timing_d, rep_d, P_dbl = time_form(qpe, torch, prob, "mixed", 1, 0, flags=qpe.PREFIX_DOUBLING)
    out = {
        "metric": "QPE circuits/s (mixed form)",
        "value": round(steps / el, 5), "unit": "circuits/s", "n_gpus": 1, "steps": steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * el / steps, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16", "dtype_detail": DTYPE_DETAIL,
        "data": "synthetic (seeded Haar unitary generated on the device, eigenvector input)",
        "config": {"workload": CONFIGS["c5"], "n_meas": n, "n_mat": t, "amplitudes": N * d, "form": "mixed",
                   "workspace_bytes": qpe.workspace_bytes([(n, t)], "mixed")},
        "roofline": {"kernel": CTRL_DEFAULT + " (controlled product, split-FP16 x3 on MFMA)", "bound": "mfma",
                     "achieved": round(achieved, 2), "peak": PEAK_F16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_F16_TFLOPS, 4),
                     "executed_frac": round(EXECUTED["split_fp16x3"] * achieved / PEAK_F16_TFLOPS, 4),
                     "flops_per_launch": flops_per_launch, "avg_launch_ms": round(avg_s * 1e3, 3),
                     "launches": g_cnt, "traffic": None},
        "breakdown_mixed": {k: {"launches": c, "ms_per_circuit": round(ms / steps, 2)} for k, (c, ms) in timing.items()},
        "report_mixed": {"prob_sum": float(rep["prob_sum"]), "unitarity_defect": float(rep["unitarity_defect"]),
                         "flags": int(rep["flags"])},
        "prefix_doubling_form": {"seconds_per_circuit": round(el_d, 2),
                                 "bitwise_equal_to_gate_route": bool(np.array_equal(P_dbl, P)),
                                 "breakdown": {k: {"launches": c, "ms_per_circuit": round(ms, 2)}
                                               for k, (c, ms) in timing_d.items()}},
        "input_generation_seconds": round(gen_s, 1),
        "target_phase": phi0,
        "argmax_outcome": int(np.argmax(P)),
    }
    print(json.dumps(out), flush=True)
    return 0


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed circuits (default 20; 1 for c5)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed circuits first (default 3; 0 for c5)")
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--fp64-steps", type=int, default=0, help="timed FP64-form circuits (default steps//2, >=3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (by default it picks the tile variants first, outside the timed "
                         "region; the timed kernels are the ones it picks)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched c4 leg of the default run")
    ap.add_argument("--batch-steps", type=int, default=10, help="timed batches of the batched c4 leg")
    ap.add_argument("--study", choices=["precision", "scaling"], default=None,
                    help="precision: the estimator study (section 4.2) over every eigenvector of a 16 x 16 Haar "
                         "unitary for n = --study-n-min .. --study-n-max; scaling: time and device memory "
                         "against N_total (section 4.1) on the analytic test problem, N_total = 6 .. "
                         "--study-total-max; each prints one JSON line and exits")
    ap.add_argument("--study-total-max", type=int, default=28)
    ap.add_argument("--study-n-min", type=int, default=4)
    ap.add_argument("--study-n-max", type=int, default=24)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (calibrates the HBM byte "
                         "counters of a profiler pass) and exit")
    return ap.parse_args()


def copy_probe(mib: int) -> int:
    """A plain copy kernel of known size: reads and writes mib MiB, 3 times."""
    import torch
    n = mib * (1 << 20)
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": n, "launches": 3}), flush=True)
    return 0


def precision_study_main(a) -> int:
    """Estimator errors against the exact eigenphases, per n and form."""
    import torch
    from paper_2507_17175_amd import qpe, study
    from workloads import eigenbasis_problems

    qpe.load_library()
    probs = eigenbasis_problems(a.study_n_min, n_mat=4, seed=12)
    U = torch.from_numpy(probs[0].U).cuda()
    psis = [torch.from_numpy(p.psi).cuda() for p in probs]
    ns = list(range(a.study_n_min, a.study_n_max + 1))
    out = {"study": "phase-estimator precision vs N_meas (section 4.2)",
           "workload": "every eigenvector of one seeded 16 x 16 Haar unitary (uniform eigenphases), 16 instances "
                       "per n, batched",
           "estimators": {"argmax": "max-norm: argmax_m P(m) / N", "weighted": "sum_m P(m) m / N (plain |error|)",
                          "circular": "arg(sum_m P(m) exp(2 pi i m / N)) / 2 pi (circular error)"}}
    for form in ("mixed", "fp64"):
        t0 = time.perf_counter()
        rows = study.precision_study(U, psis, probs[0].phis, ns, form=form)
        torch.cuda.synchronize()
        out[form] = {"rows": rows, "seconds": round(time.perf_counter() - t0, 3),
                     "log2_slope_argmax": round(study.halving_slope(rows, "argmax_mean"), 3),
                     "log2_slope_circular": round(study.halving_slope(rows, "circular_mean"), 3)}
    print(json.dumps(out), flush=True)
    return 0


def end_to_end(qpe, torch, p, form="mixed", reps=3):
    """One circuit from host inputs to host probabilities, split the way the
    paper's profile splits it (allocation, host-to-device copies, the
    application of the circuit, device-to-host copy). The device workspace
    is allocated fresh each time (the caching allocator emptied first); U and
    psi come from pinned host memory. Median over reps."""
    U_h = torch.from_numpy(p.U).pin_memory()
    psi_h = torch.from_numpy(p.psi).pin_memory()
    shapes = [(p.n_meas, p.n_mat)]
    need = qpe.workspace_bytes(shapes, form)
    rows = []
    for _ in range(reps):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        U_d = U_h.to("cuda", non_blocking=True)
        psi_d = psi_h.to("cuda", non_blocking=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        P_d = qpe.run_batch([(U_d, psi_d, p.n_meas)], form=form, workspace=ws)[0]
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        P_h = P_d.cpu()
        t4 = time.perf_counter()
        rows.append((t1 - t0, t2 - t1, t3 - t2, t4 - t3, t4 - t0))
        del ws, U_d, psi_d, P_d, P_h
    med = np.median(np.array(rows), axis=0) * 1e3
    return {"alloc_ms": round(float(med[0]), 3), "h2d_ms": round(float(med[1]), 3), "run_ms": round(float(med[2]), 3),
            "d2h_ms": round(float(med[3]), 3), "total_ms": round(float(med[4]), 3),
            "circuits_per_s_incl_transfers": round(1e3 / float(med[4]), 3),
            "h2d_bytes": int(p.U.nbytes + p.psi.nbytes), "d2h_bytes": int(8 << p.n_meas),
            "workspace_bytes": int(need), "reps": reps}


def scaling_study_main(a) -> int:
    """Section 4.1 sweeps on the analytic test problem (known eigenphases
    j / 2^N_mat; U = P Lambda P^-1 is not unitary, so the powers skip the
    Newton-Schulz step): N_mat = min(N_total // 2, 12), N_meas = the rest,
    input the eigenvector of j = d / 3, whose phase is exact in N_meas >=
    N_mat bits, so all probability must sit at m = j 2^(N_meas - N_mat)."""
    import torch
    from paper_2507_17175_amd import qpe, study
    from workloads import analytic_problem

    qpe.load_library()
    cases = []
    for total in range(6, a.study_total_max + 1):
        t = min(total // 2, 12)
        n = total - t
        j = (1 << t) // 3
        p = analytic_problem(n, t, j)
        cases.append({"U": torch.from_numpy(p.U).cuda(), "psi": torch.from_numpy(p.psi).cuda(), "n": n,
                      "peak": j << (n - t)})
    t0 = time.perf_counter()
    rows = []
    for c in cases:
        rows += study.scaling_sweep([c], flags=qpe.NO_POLAR)
        print(json.dumps({"progress": rows[-1]}), file=sys.stderr, flush=True)
        del c["U"], c["psi"]
    out = {"study": "time and device memory vs N_total (section 4.1), analytic test problem (section 3)",
           "rows": rows, "seconds": round(time.perf_counter() - t0, 2)}
    print(json.dumps(out), flush=True)
    return 0


def batch_of_copies(qpe, torch, prob, copies, steps, P_single):
    """`copies` copies of one instance as one batched run, captured in a HIP
    graph and replayed `steps` times; every copy's P must equal the single
    run's bit for bit."""
    run = qpe.Runner([(prob["U"], prob["psi"], prob["n"])] * copies, form="mixed")
    run()
    torch.cuda.synchronize()
    graph = qpe.CapturedRun(run)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    same = all(np.array_equal(P.cpu().numpy(), P_single) for P in run.probs[:: max(1, copies // 64)])
    return {"instances": copies, "circuits_per_s": round(copies * steps / el, 1),
            "ms_per_batch": round(1e3 * el / steps, 3), "copies_equal_single_run": bool(same)}


def time_form(qpe, torch, prob, form, steps, warmup, flags=0):
    """Times `steps` circuits with HIP events around the controlled-product
    launches only (the roofline figure); the per-stage breakdown comes from
    two more circuits with every stage timed, after the timed region."""
    run = qpe.Runner([(prob["U"], prob["psi"], prob["n"])], form=form, flags=flags)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    run.ctx.enable_timing(80 * steps + 64)
    run.ctx.set_timing_mask(["ctrl_gemm"])
    run.ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = run.ctx.read_timing()
    run.ctx.set_timing_mask(None)
    run.ctx.reset_timing()
    for _ in range(2):
        run()
    stages = run.ctx.read_timing()
    timing.update({k: (v[0] * steps // 2, v[1] * steps / 2) for k, v in stages.items() if k != "ctrl_gemm"})
    rep = run.reports()[0]
    P = run.probs[0].cpu().numpy()
    return (t1 - t0), timing, rep, P


def main():
    a = parse()
    if a.steps is None:
        a.steps = 1 if a.config == "c5" else 20
    if a.warmup is None:
        a.warmup = 0 if a.config == "c5" else 3
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {a.gpus}); "
              "the multi-GPU sharding is a design, not an implementation", file=sys.stderr)
        return 2
    if a.copy_probe_mib:
        return copy_probe(a.copy_probe_mib)
    if a.study == "precision":
        return precision_study_main(a)
    if a.study == "scaling":
        return scaling_study_main(a)
    import torch
    from paper_2507_17175_amd import qpe
    from workloads import config_problems

    qpe.load_library()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if a.config == "c4":
        return bench_batch(a, qpe, torch, config_problems)
    if a.config == "c5":
        return bench_c5(a, qpe, torch)
    p = config_problems(a.config)[0]
    n, t = p.n_meas, p.n_mat
    N, d = 1 << n, 1 << t
    prob = {"U": torch.from_numpy(p.U).cuda(), "psi": torch.from_numpy(p.psi).cuda(), "n": n}

    tuned = {}
    if not a.no_autotune:
        # the autotuner picks the tile variants of this operator size (a few
        # circuits per variant, before and outside the timed region)
        ctx = qpe.context(torch.cuda.current_device())
        tuned["mixed"] = ctx.autotune(prob["U"], prob["psi"], n, form="mixed", reps=2)
        if not a.no_fp64:
            tuned["fp64"] = ctx.autotune(prob["U"], prob["psi"], n, form="fp64", reps=1)

    el, timing, rep, P_mixed = time_form(qpe, torch, prob, "mixed", a.steps, a.warmup)
    ms_per = 1e3 * el / a.steps
    value = a.steps / el

    flops_per_launch = 8.0 * (N // 2) * d * d  # algorithmic, complex MACs x 8
    g_cnt, g_ms = timing["ctrl_gemm"]
    avg_s = (g_ms / g_cnt) / 1e3 if g_cnt else float("nan")
    achieved = flops_per_launch / avg_s / 1e12
    ctx = qpe.context(torch.cuda.current_device())
    ctrl_variant = ctx.get_variant("ctrl_mixed", t) if t >= 5 else None
    if t >= 5:
        roofline = {
            "kernel": (f"{CTRL_KERNELS.get(ctrl_variant, CTRL_DEFAULT)} (controlled product, split-FP16 x3 on MFMA; "
                       f"variant {ctrl_variant}"
                       + (", the built-in kernel at this size" if ctrl_variant in TRAFFIC_VARIANTS else "") + ")"),
            "bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_F16_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_F16_TFLOPS, 4),
            "executed_frac": round(EXECUTED["split_fp16x3"] * achieved / PEAK_F16_TFLOPS, 4),
        }
    else:
        # d <= 16: one thread per row on the vector ALUs in FP32 (no split);
        # a launch this small is decided by its latency, not by the ALUs
        roofline = {
            "kernel": "k_ctrl_small (controlled product on the vector ALUs, FP32)",
            "bound": "alu", "achieved": round(achieved, 6), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 8), "executed_frac": round(achieved / PEAK_FP32_TFLOPS, 8),
        }
    roofline.update({"flops_per_launch": flops_per_launch, "avg_launch_ms": round(avg_s * 1e3, 4), "launches": g_cnt})
    # traffic: HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE), or null
    # valid for the kernel the counters were taken on: the built-in choice at
    # this size (variant 0) or the same kernel picked explicitly
    tr = traffic_for_current_kernel() if (a.config == "c2" and ctrl_variant in TRAFFIC_VARIANTS) else None
    roofline["traffic"] = tr["bytes_per_launch"] if tr else None
    roofline["traffic_detail"] = tr
    breakdown = {k: {"launches": c, "ms_per_circuit": round(ms / a.steps, 4)} for k, (c, ms) in timing.items()}

    out = {
        "metric": "QPE circuits/s (mixed form, max|dP| <= 1e-6 vs FP64 oracle)",
        "value": round(value, 3),
        "unit": "circuits/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16", "dtype_detail": DTYPE_DETAIL,
        "data": "synthetic (seeded Haar unitary, eigenvector input)",
        "config": {"workload": CONFIGS[a.config], "n_meas": n, "n_mat": t, "amplitudes": N * d,
                   "state": "complex64", "U": "complex128", "form": "mixed"},
        "roofline": roofline,
        "autotune": tuned or None,
        "breakdown_mixed": breakdown,
        "report_mixed": {"prob_sum": float(rep["prob_sum"]), "unitarity_defect": float(rep["unitarity_defect"]),
                         "input_peak": float(rep["input_peak"]), "flags": int(rep["flags"])},
        "hbm_state_gbs": round((n * N * d * 8 + 3 * N * d * 8) / (ms_per / 1e3) / 1e9, 1),
    }

    # Prefix-doubling form of the controlled stage (same probabilities, bit
    # for bit): rows [2^k, 2^(k+1)) = rows [0, 2^k) V_k^T, 2^n - 1 row
    # products instead of n 2^(n-1).
    el_d, timing_d, rep_d, P_dbl = time_form(qpe, torch, prob, "mixed", a.steps, 1, flags=qpe.PREFIX_DOUBLING)
    dc, dms = timing_d["ctrl_gemm"]
    out["prefix_doubling_form"] = {
        "circuits_per_s": round(a.steps / el_d, 3), "ms_per_circuit": round(1e3 * el_d / a.steps, 3),
        "ctrl_algorithmic_flops_per_circuit": 8.0 * (N - 1) * d * d,
        "ctrl_ms_per_circuit": round(dms / a.steps, 4),
        "bitwise_equal_to_gate_route": bool(np.array_equal(P_dbl, P_mixed)),
        "breakdown": {k: {"launches": c, "ms_per_circuit": round(ms / a.steps, 4)} for k, (c, ms) in timing_d.items()},
    }

    # The six-product split-BF16 scheme (QPE_SPLIT_BF16) on the same
    # workload, for comparison with the default split-FP16 one.
    el_b, timing_b, rep_b, P_bf16 = time_form(qpe, torch, prob, "mixed", max(3, a.steps // 2), 1,
                                               flags=qpe.SPLIT_BF16)
    bc, bms = timing_b["ctrl_gemm"]
    bavg = (bms / bc) / 1e3 if bc else float("nan")
    out["split_bf16_form"] = {
        "circuits_per_s": round(max(3, a.steps // 2) / el_b, 3),
        "ctrl_gemm": {"achieved": round(flops_per_launch / bavg / 1e12, 2), "avg_launch_ms": round(bavg * 1e3, 4),
                      "frac": round(flops_per_launch / bavg / 1e12 / PEAK_F16_TFLOPS, 4),
                      "executed_frac": round(EXECUTED["split_bf16x6"] * flops_per_launch / bavg / 1e12
                                             / PEAK_F16_TFLOPS, 4)},
    }

    out["end_to_end_mixed"] = end_to_end(qpe, torch, p, "mixed")

    if a.config == "c1":
        # A 2^10-amplitude circuit is launch-bound on its own: also time it as
        # a batch of identical instances (one grouped run, replayed graph).
        out["batch_of_copies"] = batch_of_copies(qpe, torch, prob, 4096, a.steps, P_mixed)

    if not a.no_fp64:
        fsteps = a.fp64_steps or max(3, a.steps // 2)
        el64, timing64, rep64, P_fp64 = time_form(qpe, torch, prob, "fp64", fsteps, 1)
        c64, ms64 = timing64["ctrl_gemm"]
        avg64 = (ms64 / c64) / 1e3 if c64 else float("nan")
        ach64 = flops_per_launch / avg64 / 1e12
        out["fp64_form"] = {
            "circuits_per_s": round(fsteps / el64, 3), "ms_per_circuit": round(1e3 * el64 / fsteps, 3),
            "steps": fsteps,
            # The kernel forms each complex product from three real ones
            # (Gauss): 6 executed flop per complex multiply-add. `achieved`
            # and `frac` count those against the FP64 peak (a true fraction,
            # <= 1); `algorithmic_tflops` counts 8 flop per multiply-add,
            # the figure the mixed form's roofline uses, and can exceed the
            # FP64 peak for that reason.
            "ctrl_gemm": {"achieved": round(0.75 * ach64, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                          "frac": round(0.75 * ach64 / PEAK_FP64_TFLOPS, 4),
                          "algorithmic_tflops": round(ach64, 2),
                          "avg_launch_ms": round(avg64 * 1e3, 4)},
            "breakdown": {k: {"launches": c, "ms_per_circuit": round(ms / fsteps, 4)}
                          for k, (c, ms) in timing64.items()},
        }
        out["mixed_over_fp64"] = round(value / (fsteps / el64), 3)

    if not a.no_batch and a.config == "c2":
        # The batched pattern: the 512 uneven instances of the batched
        # workload in one graph-replayed run, mixed against FP64.
        out["batched_c4"] = measure_batch(qpe, torch, config_problems("c4"), a.batch_steps, 2,
                                          autotune=not a.no_autotune)
        out["batched_c4"]["workload"] = CONFIGS["c4"]

    if not a.no_cpu_baseline:
        # CPU baseline leg: the oracle, untouched, on one full circuit of the
        # same workload, using the host's cores through numpy/scipy.
        import oracle.qpe_oracle as O
        cores = os.cpu_count() or 1
        t0 = time.perf_counter()
        P_ref = O.qpe_probs(p.U, p.psi, n)
        t1 = time.perf_counter()
        out["cpu_baseline"] = {"value": round(1.0 / (t1 - t0), 5), "unit": "circuits/s", "cores": cores,
                               "kind": "oracle", "sample": f"1 full circuit of {CONFIGS[a.config]}",
                               "seconds": round(t1 - t0, 2)}
        out["max_abs_err_mixed"] = float(np.abs(P_mixed - P_ref).max())
        out["split_bf16_form"]["max_abs_err"] = float(np.abs(P_bf16 - P_ref).max())
        if not a.no_fp64:
            out["fp64_form"]["max_abs_err"] = float(np.abs(P_fp64 - P_ref).max())
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
