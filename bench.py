"""Benchmark of the ILE marginalized-likelihood step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched]

A step is one pass of the whole hot path over one batch: on-device sampling
of the extrinsic parameters, ln L_t for every sample (geometry, harmonics,
coefficients, the time-shifted contraction, interpolation and the window
log-sum-exp), ln w, and the FP64 reduction to ln L_marg with n_eff, n_ESS and
n_var (one call of rift_ile_marginalize).  Inputs (Q, U) are resident in HBM
before the timed region.  The default workload is the batched one (512
heterogeneous intrinsic points, 1.98e8 evaluations per step).  The steps are
timed twice, with direct launches (the evaluation kernels timed with HIP
events for the roofline) and with each evaluation run replayed from a
captured hipGraph; the replayed rate is the headline value.  Beside it the
default run measures the single-point workload (the utilization target) and
the gradient workload (timing and per-component error of the FP32 adjoint).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma_tflops": 157.3, "fp64_tflops": 78.6, "hbm_gbs": 8000.0}

# HBM bytes per step of the evaluation kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (KiB per dispatch, summed over a step's dispatches, scaled
# by 2.0 and 1.0: what the same counters read for a plain device copy of known
# size on the same box), keyed by workload, with the SHA-256 of the kernel
# source they were taken with.  Reported only while that source is unchanged.
MEASURED_TRAFFIC = {
    # profiles/mfma_kernel_batched_512pts.md: 19,761,493 KiB x 2.0 + 6,617,605 KiB x 1.0 over the 8 class dispatches
    "batched": {"sha256": "c3e061b9d552391d41c590262f4b80b34a8e358ac83bd7d2a4343f7db9ddf69d", "bytes_per_step": 47247965568.0},
    # profiles/mfma_kernel_single_1e6.md: 167,358 KiB x 2.0 + 33,832 KiB x 1.0
    "single": {"sha256": "c3e061b9d552391d41c590262f4b80b34a8e358ac83bd7d2a4343f7db9ddf69d", "bytes_per_step": 377393120.0},
}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2210_07912_amd", "csrc", "k_mfma.hip")


def flops_per_eval(K, M, n_t):
    """Algorithmic FLOPs of one time-marginalized evaluation: the contraction
    of the K (n_t + 3) needed rows (4 flops per complex mode product, real
    part), the 4-tap interpolation (8 flops per window sample and detector),
    the log-sum-exp (4 per window sample), the quadratic term (4 K M^2) and
    the per-sample coefficients (6 K M + 200)."""
    return K * (n_t + 3) * 4 * M + 8 * K * n_t + 4 * n_t + 4 * K * M * M + 6 * K * M + 200


def flops_per_grad(K, M, n_t):
    """Forward evaluation plus the adjoint: the transposed contraction
    G_k = sum_r c_k[r] Q_k[r] (K (n_t + 3) 4 M), the transposed interpolation
    c_k (8 K (n_t + 3)), the derivative interpolation (8 K n_t), the softmax
    weights (2 n_t), U a and V a for the chain rule (8 K M^2) and the chain
    rule itself (40 K M)."""
    return (flops_per_eval(K, M, n_t) + K * (n_t + 3) * 4 * M + 8 * K * (n_t + 3) + 8 * K * n_t + 2 * n_t
            + 8 * K * M * M + 40 * K * M)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _shape(p):
    return p["det_pos"].shape[0], len(p["ell"]), p["n_t"]


def _consistent(g, th, f_s):
    """Gradient [7, N] in consistent units: d/d(angle), D d/dD, (1/f_s) d/dtau."""
    u = g.copy()
    u[5] = u[5] * th[5]
    u[6] = u[6] / f_s
    return u


def measure_forward(name, steps, warmup, graph=True, n_override=0):
    """Time the forward step of a workload (direct launches with the
    evaluation kernels timed by events, then hipGraph replays)."""
    import torch

    import synth
    from paper_2210_07912_amd import ile

    w = synth.workload(name)
    pts = [synth.make_point(s) for s in w.points]
    counts = [n_override] * len(pts) if n_override else list(w.n_samples)
    h = ile.RiftILE(pts, precision=w.precision, tau_width=w.tau_width)
    seed = synth.BASE_SEED + synth.WORKLOADS.index(name)
    rounds = w.rounds if w.adaptive else 1
    mask = 0x3F if w.adaptive else 0

    def step(i):
        return h.marginalize(seed + i, counts, n_rounds=rounds, adapt_mask=mask, floor_eps=0.1)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    h.profile(True)
    t0 = time.perf_counter()
    res = None
    for i in range(steps):
        res = step(100 + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = h.profile(False)
    evals = sum(counts) * rounds
    dt = (t1 - t0) / steps
    fp32 = w.precision == "fp32"
    # roofline of the dominant kernels (the evaluation kernels of every (T, K)
    # class, one persistent launch each, fanned out over side streams): the
    # timed steps' algorithmic FLOP spread over the timed evaluation runs,
    # over their average duration between the events around each run
    fl = rounds * sum(c * flops_per_eval(*_shape(p)) for c, p in zip(counts, pts))
    fl_per_launch = fl * steps / max(k_launches, 1)
    k_avg_ms = k_ms / max(k_launches, 1)
    achieved = fl_per_launch / (k_avg_ms * 1e-3) / 1e12 if k_launches else None
    peak = PEAK["fp32_mfma_tflops"] if fp32 else PEAK["fp64_tflops"]
    classes = sorted({((len(p["ell"]) + 1) // 2, p["det_pos"].shape[0]) for p in pts})
    roof = {"bound": "mfma" if fp32 else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": (achieved / peak) if achieved else None, "traffic": None,
            "kernel": ("mfma_kernel<T,K>" if fp32 else "plain_kernel<double>"),
            "classes": [f"T{t}K{k}" for t, k in classes] if fp32 else None,
            "kernel_ms": k_avg_ms, "launches_per_step": k_launches / steps,
            "flops_per_eval": fl / max(evals, 1), "flops_per_launch": fl_per_launch}
    if fp32:
        # matrix-core FLOP the kernels execute per evaluation: 16-row blocks
        # 0..ceil(n_t/16) of every detector times 2 M_p elements
        ex = [2 * p["det_pos"].shape[0] * 16 * ((p["n_t"] + 15) // 16 + 1) * 2 * ((len(p["ell"]) + 1) // 2 * 2)
              for p in pts]
        roof["mfma_executed_per_eval"] = sum(c * e for c, e in zip(counts, ex)) / max(sum(counts), 1)
    tr = MEASURED_TRAFFIC.get(name)
    if tr and not n_override and tr["sha256"] == _sha(KERNEL_SOURCE) and k_launches:
        roof["traffic"] = tr["bytes_per_step"] * steps / k_launches
        roof["hbm_gbs"] = roof["traffic"] / (k_avg_ms * 1e-3) / 1e9
        roof["hbm_frac"] = roof["hbm_gbs"] / PEAK["hbm_gbs"]
    out = {"value": evals / dt, "ms_per_step": dt * 1e3, "evals_per_step": evals, "points": len(pts),
           "rounds": rounds, "roofline": roof, "seed": seed,
           "lnL_marg": [r["lnL_marg"] for r in res][:4], "n_eff": [r["n_eff"] for r in res][:4],
           "launch": "direct"}
    if fp32:
        out["autotune"] = {f"T{t}K{k}": m for (t, k), m in sorted(h.autotune_table().items())}
    if graph and fp32:
        h.set_graph(True)
        for i in range(max(warmup, 1)):
            step(i)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for i in range(steps):
            step(100 + i)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        cap, rep = h.graph_stats()
        h.set_graph(False)
        gdt = (t3 - t2) / steps
        out["direct"] = {"value": evals / dt, "ms_per_step": dt * 1e3}
        out["value"] = evals / gdt
        out["ms_per_step"] = gdt * 1e3
        out["graph"] = {"captures": cap, "replays": rep}
        out["launch"] = "hipGraph replay of each evaluation run"
    return out, h, pts, counts, seed


def measure_grad(steps, warmup, with_errors=True):
    """The gradient workload: a step draws 1e5 samples on the device and
    computes ln L_t and its gradient in the seven parameters (one adjoint
    call, with the FP64 refinement of the samples whose mass lies in a few
    window blocks), then the FP64 reduction.  The errors: every sample's FP32
    gradient against the FP64 adjoint on the same FP32-rounded inputs, per
    component, in consistent units (angles, ln D, tau in window samples)."""
    import numpy as np
    import torch

    import synth
    from paper_2210_07912_amd import ile

    w = synth.workload("grad")
    d = synth.make_point(w.points[0])
    n = w.n_samples[0]
    h = ile.RiftILE([d], precision="fp32", tau_width=w.tau_width)
    seed = synth.BASE_SEED + synth.WORKLOADS.index("grad")

    def step(i):
        th, _, _ = h.sample(0, seed + i, 0, n)
        g, lt = h.backward(th, want_lnL=True)
        return [h.reduce(lt)]

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    h.profile(True)
    t0 = time.perf_counter()
    for i in range(steps):
        step(100 + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = h.profile(False)
    dt = (t1 - t0) / steps
    K, M, n_t = _shape(d)
    fl = n * flops_per_grad(K, M, n_t)
    k_avg = k_ms / max(k_launches, 1)
    achieved = fl * steps / max(k_launches, 1) / (k_avg * 1e-3) / 1e12 if k_launches else None
    out = {"value": n / dt, "unit": "gradient evals/s", "ms_per_step": dt * 1e3, "samples": n,
           "roofline": {"bound": "mfma", "kernel": "mfma_bwd_kernel<11,3>", "achieved": achieved,
                        "peak": PEAK["fp32_mfma_tflops"], "unit": "TFLOP/s",
                        "frac": achieved / PEAK["fp32_mfma_tflops"] if achieved else None, "kernel_ms": k_avg,
                        "flops_per_eval": flops_per_grad(K, M, n_t)}}
    if with_errors:
        th, _, _ = h.sample(0, seed + 999, 0, n)
        g32, l32 = h.backward(th, want_lnL=True)
        h.set_grad_refine(False)
        g0, _ = h.backward(th, want_lnL=True)
        h.set_grad_refine(True)
        dr = dict(d)
        for key in ("Q", "U"):
            dr[key] = np.asarray(d[key]).astype(np.complex64).astype(np.complex128)
        h64 = ile.RiftILE([dr], precision="fp64", tau_width=w.tau_width)
        g64, l64 = h64.backward(th.double(), want_lnL=True)
        thn = th.cpu().numpy().astype(np.float64)
        f_s = d["f_s"]
        ur = _consistent(g64.cpu().numpy(), thn, f_s)
        scale = np.abs(ur).max(axis=0)
        names = ["alpha", "delta", "psi", "iota", "phi", "lnD", "tau"]

        def errs(gx):
            ux = _consistent(gx.cpu().numpy().astype(np.float64), thn, f_s)
            return np.abs(ux - ur) / scale

        e32, e0 = errs(g32), errs(g0)
        l64n = l64.cpu().numpy()
        top = l64n >= l64n.max() - 20.0
        own = np.abs(_consistent(g32.cpu().numpy().astype(np.float64), thn, f_s) - ur) / np.maximum(np.abs(ur), 1e-300)
        big = np.abs(ur) >= 1e-3 * scale
        out["error"] = {
            "reference": "FP64 adjoint on the same FP32-rounded inputs, all samples",
            "measure": "max over samples of |g32_c - g64_c| / max_c' |g64_c'|, consistent units "
                       "(angles rad, ln D, tau in window samples)",
            "per_component": {k: float(e32[i].max()) for i, k in enumerate(names)},
            "per_component_p99_9": {k: float(np.percentile(e32[i], 99.9)) for i, k in enumerate(names)},
            "per_component_fp32_only": {k: float(e0[i].max()) for i, k in enumerate(names)},
            "refined_fraction": float(np.mean(np.any(g32.cpu().numpy() != g0.cpu().numpy(), axis=0))),
            "weight_carrying_samples": int(top.sum()),
            "weight_carrying_max_own_relative": float(np.where(big & top[None, :], own, 0.0).max()),
        }
        h64.close()
    h.close()
    return out


def cpu_baseline(pts, counts, precision, seconds, runs, tau_width=0.0):
    """The oracle (FP64 CPU reference) built for this host (-O3 -march=native,
    OpenMP over samples) on a bounded sample of the workload: up to 32 of its
    points (evenly spaced), a fixed number of prior samples each, timing
    ln L_t of every sample plus the FP64 reduction per point; the median of
    `runs` runs."""
    import numpy as np

    import synth
    from oracle import oracle

    tmp = tempfile.mkdtemp(prefix="rift_oracle_")
    oracle.use_native_build(tmp)
    step = max(1, len(pts) // 32)
    sel = list(range(0, len(pts), step))[:32]
    ops = [oracle.Point.from_dict(pts[i], complex64=(precision == "fp32")) for i in sel]

    def run(S):
        ths = [synth.prior_samples(synth.BASE_SEED + 77 + j, min(S, counts[i]), tau_width)
               .astype(np.float32).astype(np.float64) for j, i in enumerate(sel)]
        t_a = time.perf_counter()
        for op, th in zip(ops, ths):
            oracle.reduce(oracle.lnL_t(op, th))
        t_b = time.perf_counter()
        return sum(th.shape[1] for th in ths), t_b - t_a

    n_probe, t_probe = run(64)
    S = int(max(64, min(min(counts[i] for i in sel), 64 * (seconds / runs) / max(t_probe, 1e-6))))
    rates, n_run = [], 0
    for _ in range(runs):
        n_run, t = run(S)
        rates.append(n_run / t)
    return {"value": statistics.median(rates), "unit": "evals/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{len(sel)} of {len(pts)} points (indices 0, {step}, {2 * step}, ...), {S} prior samples each "
                      f"({n_run} evaluations per run): ln L_t of every sample plus the FP64 reduction per point; "
                      f"median of {runs} runs; oracle built -O3 -march=native with OpenMP",
            "runs": rates, "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched",
                    help="batched (default: 512 points, 1.98e8 samples) | single | plain | grad | adaptive")
    ap.add_argument("--n", type=int, default=0, help="samples per point per step (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="oracle time over all baseline runs")
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the measurements beside the timed steps (other workloads, FP64 replays, ...)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (points would shard across GPUs "
              "with one 40-byte FP64 exchange per point)",
              file=sys.stderr)
        sys.exit(2)

    import math

    import numpy as np
    import torch

    import synth
    from paper_2210_07912_amd import ile

    name = args.workload
    if name == "grad":
        g = measure_grad(args.steps, args.warmup, with_errors=not args.no_extras)
        w = synth.workload("grad")
        pts = [synth.make_point(s) for s in w.points]
        out = {"metric": "extrinsic lnL evals/sec (time-marginalized) at |dln L_marg|<=1e-3 vs FP64",
               "value": g["value"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": g["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f32", "data": "synthetic",
               "config": {"workload": "grad", "points": 1, "samples_per_step": g["samples"],
                          "note": "ln L_t and its gradient in 7 parameters per evaluation"},
               "roofline": g["roofline"], "grad": g}
        if not args.no_extras:
            h = ile.RiftILE(pts, precision="fp32", tau_width=w.tau_width)
            counts = list(w.n_samples)
            seed = synth.BASE_SEED + synth.WORKLOADS.index("grad")
            ref = {}
            for nm, gflag in (("histogram", False), ("gradient_refined", True)):
                h.marginalize(seed, counts[0], n_rounds=2, adapt_mask=0x3F, floor_eps=0.1, gradient=gflag)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                r = h.marginalize(seed + 7, counts[0], n_rounds=w.rounds, adapt_mask=0x3F, floor_eps=0.1,
                                  gradient=gflag, n_ascent=64, ascent_steps=12, ascent_mix=0.3)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                ref[nm] = {"evals_per_s": counts[0] * w.rounds / (t3 - t2), "s": t3 - t2,
                           "lnL_marg": r[0]["lnL_marg"], "sigma_lnL": r[0]["sigma_lnL"], "n_eff": r[0]["n_eff"]}
            out["refinement"] = {"rounds": w.rounds, "samples_per_round": counts[0],
                                 "adapt": "alpha, delta, psi, iota, phi, D histograms", **ref}
            h.close()
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(pts, list(w.n_samples), "fp32", args.cpu_seconds, args.cpu_runs,
                                               w.tau_width)
        print(json.dumps(out), flush=True)
        return

    m, h, pts, counts, seed = measure_forward(name, args.steps, args.warmup, graph=not args.no_graph,
                                              n_override=args.n)
    w = synth.workload(name)
    fp32 = w.precision == "fp32"
    out = {
        "metric": "extrinsic lnL evals/sec (time-marginalized) at |dln L_marg|<=1e-3 vs FP64",
        "value": m["value"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64", "data": "synthetic",
        "config": {"workload": name, "points": len(pts),
                   "samples_per_point": counts[0] if len(set(counts)) == 1 else "varied",
                   "samples_per_step": m["evals_per_step"], "rounds": m["rounds"],
                   "K": sorted({p["det_pos"].shape[0] for p in pts}), "M": sorted({len(p["ell"]) for p in pts}),
                   "n_t": [min(p["n_t"] for p in pts), max(p["n_t"] for p in pts)], "seed": seed,
                   "launch": m["launch"]},
        "roofline": m["roofline"],
    }
    for k in ("direct", "graph", "autotune", "lnL_marg", "n_eff"):
        if k in m:
            out[k] = m[k]

    # the utilization target's workload (1 point, K = 3, M = 21, n_t = 820, 1e6
    # samples) and the gradient workload, beside the headline
    if name == "batched" and not args.no_extras:
        s, hs, _, _, _ = measure_forward("single", 20, 3, graph=not args.no_graph)
        hs.close()
        out["single_point"] = {k: s[k] for k in ("value", "ms_per_step", "roofline", "launch", "lnL_marg")}
        out["grad"] = measure_grad(10, 2, with_errors=not args.no_fp64)

    # distance marginalization on the same step (ln L_tD in place of ln L_t:
    # each sample evaluated at D_ref, its largest data term, then 24 nodes in
    # D): its rate against the step's, measured on the same handle
    if fp32 and not args.n and not args.no_extras and name in ("batched", "single"):
        h.set_distance_marginalization(True)
        h.set_graph(not args.no_graph)
        rounds = m["rounds"]
        nd = max(1, min(args.steps, 5))
        for i in range(max(1, min(args.warmup, 2))):
            h.marginalize(seed + i, counts, n_rounds=rounds, adapt_mask=0, floor_eps=0.1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for i in range(nd):
            r = h.marginalize(seed + 100 + i, counts, n_rounds=rounds, adapt_mask=0, floor_eps=0.1)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        h.set_distance_marginalization(False)
        h.set_graph(False)
        ddt = (t3 - t2) / nd
        out["distance_marginalization"] = {"evals_per_s": m["evals_per_step"] / ddt, "ms_per_step": ddt * 1e3,
                                           "steps": nd, "cost_vs_time_only": ddt * 1e3 / m["ms_per_step"],
                                           "lnL_marg": [x["lnL_marg"] for x in r][:4]}

    # the Q/U/V precompute at the single-point shape: 3 detectors, 21 modes,
    # 8 s at 4096 Hz (N = 32768), the 999 stored rows; host arrays in and out
    if name == "single" and not args.n and not args.no_extras:
        N, df = 32768, 0.125
        data, psd, modes, _ = synth.fd_inputs(synth.BASE_SEED + 50, n_det=3, n_modes=21, N=N, df=df, f_low=20.0)
        L = pts[0]["n_t"] + 2 * pts[0]["pad"] + 3
        ile.precompute(data, psd, modes, df, 20.0, 0, L)  # warm-up (FFT plan, code objects)
        t2 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            ile.precompute(data, psd, modes, df, 20.0, 0, L)
        t3 = time.perf_counter()
        out["precompute"] = {"K": 3, "M": 21, "N": N, "rows": L, "ms": (t3 - t2) / reps * 1e3,
                             "note": "host arrays in and out, device buffers allocated per call"}

    # sampling coordinates: the sky in each point's detector-network frame and
    # the polarization and phase in phase-rotated coordinates against the
    # equatorial, unrotated ones, with histograms in the six angles and
    # distance over 10 rounds: on the first 8 points of this workload (1e5
    # samples per round) and on the (2, +-2) workload of 4 face-on/off and 4
    # edge-on points at SNR 25 (1e6 per round, three seeds: per-point median
    # n_eff).  Then the Gaussian-mixture proposal against the histograms on
    # the first 8 points.
    if w.adaptive and not args.n and not args.no_extras:
        cfgs = (("equatorial", False, False), ("network_frame", True, False), ("phase_rotation", False, True),
                ("network_frame_phase_rotation", True, True))
        wq = synth.workload("quadrupole")
        coords = {}
        for sname, spts, n_r, seeds in (("first8", pts[:8], 100_000, (seed + 11,)),
                                        ("quadrupole", [synth.make_point(sp) for sp in wq.points], 1_000_000,
                                         (seed + 21, seed + 22, seed + 23))):
            hs = ile.RiftILE(spts, precision=w.precision, tau_width=w.tau_width)
            cc = {"samples_per_round": n_r, "seeds": len(seeds),
                  "cos_iota": [round(math.cos(p["theta_inj"][3]), 3) for p in spts]}
            for nm, net, ph in cfgs:
                hs.set_network_frame(net)
                hs.set_phase_rotation(ph)
                rs = [hs.marginalize(sd, n_r, n_rounds=10, adapt_mask=0x3F, floor_eps=0.1) for sd in seeds]
                ne = np.array([[x["n_eff"] for x in r] for r in rs])
                lm = np.array([[x["lnL_marg"] for x in r] for r in rs])
                cc[nm] = {"n_eff_median": np.median(ne, axis=0).tolist(),
                          "n_eff_geomean": float(np.exp(np.log(np.median(ne, axis=0)).mean())),
                          "lnL_marg_median": np.median(lm, axis=0).tolist(),
                          "lnL_marg_spread": np.ptp(lm, axis=0).tolist()}
            hs.close()
            coords[sname] = cc
        out["coordinates"] = {"rounds": 10, "floor_eps": 0.1, **coords}
        # distance marginalization in the adaptive runs: all six angles and
        # the distance adapted (no marginalization) against the distance
        # integrated per sample with the five angles adapted, and with the
        # sky alone adapted (the production setting of Sec. III), on the
        # first 8 points and the 8 loudest; 10 rounds of 1e5 samples
        loud = sorted(range(len(w.points)), key=lambda i: -w.points[i].snr)[:8]
        dm = {}
        for sname, idx in (("first8", list(range(8))), ("loudest8", loud)):
            hs = ile.RiftILE([pts[i] for i in idx], precision=w.precision, tau_width=w.tau_width)
            cc = {"points": idx, "snr": [round(w.points[i].snr, 2) for i in idx]}
            for nm, dmarg, amask in (("sampled_D_adapt_all", False, 0x3F), ("dmarg_adapt_angles", True, 0x1F),
                                     ("dmarg_adapt_sky", True, 0x03)):
                hs.set_distance_marginalization(dmarg)
                hs.marginalize(seed + 30, 100_000, n_rounds=1, adapt_mask=amask, floor_eps=0.1)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                r = hs.marginalize(seed + 31, 100_000, n_rounds=10, adapt_mask=amask, floor_eps=0.1)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                ne = np.array([x["n_eff"] for x in r])
                cc[nm] = {"ms": (t3 - t2) * 1e3, "n_eff": ne.tolist(), "n_eff_geomean": float(np.exp(np.log(ne).mean())),
                          "sigma_lnL": [x["sigma_lnL"] for x in r], "lnL_marg": [x["lnL_marg"] for x in r]}
            hs.close()
            dm[sname] = cc
        out["distance_marginalization_adaptive"] = {"rounds": 10, "samples_per_round": 100_000, "floor_eps": 0.1,
                                                    **dm}
        sub = pts[:8]
        hs = ile.RiftILE(sub, precision=w.precision, tau_width=w.tau_width)
        gm = {}
        # correlated pairs (psi, phi) and (iota, D): the pairs the polarization-phase and
        # inclination-distance degeneracies tie together
        for nm, kk, pr in (("histogram", 0, ()), ("gmm_k3", 3, ()), ("gmm_k3_pairs", 3, ((2, 4), (3, 5)))):
            hs.marginalize(seed + 12, 100_000, n_rounds=2, adapt_mask=0x3F, floor_eps=0.1, gmm_components=kk,
                           gmm_pairs=pr)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            r = hs.marginalize(seed + 13, 100_000, n_rounds=10, adapt_mask=0x3F, floor_eps=0.1, gmm_components=kk,
                               gmm_pairs=pr)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            gm[nm] = {"ms": (t3 - t2) * 1e3, "n_eff": [x["n_eff"] for x in r],
                      "sigma_lnL": [x["sigma_lnL"] for x in r], "lnL_marg": [x["lnL_marg"] for x in r]}
        hs.close()
        out["gmm"] = {"points": len(sub), "rounds": 10, "samples_per_round": 100_000, "floor_eps": 0.1, **gm}

    # FP32 vs FP64 on the same samples (same GPU): |d ln L_marg| and the FP64 rate
    if not args.no_fp64 and fp32 and len(pts) == 1:
        nn = min(counts[0], 200_000)
        h64 = ile.RiftILE(pts, precision="fp64", tau_width=w.tau_width)
        th64, _, _ = h64.sample(0, seed, 0, nn)
        th32 = th64.float()
        l32 = h.lnL(th32)
        l64a = h64.lnL(th32.double())
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        l64 = h64.lnL(th32.double())
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        r32, r64 = h.reduce(l32), h64.reduce(l64)
        out["fp64_plain"] = {"evals_per_s": nn / (t3 - t2), "samples": nn,
                             "lnL_marg_fp32": r32["lnL_marg"], "lnL_marg_fp64": r64["lnL_marg"],
                             "abs_delta_lnL_marg": abs(r32["lnL_marg"] - r64["lnL_marg"]),
                             "max_abs_delta_lnL_t": float((l32.double() - l64a).abs().max())}
        h64.close()

    # the estimate against the FP64 plain form on the very same samples (their
    # samples and proposal ratios replayed): for the adaptive workload the
    # first 4 points and the 15 loudest (SNR >= 50) over all rounds, for the
    # batched workload 32 of its points
    if not args.no_fp64 and (w.adaptive or name == "batched") and not args.n:
        if w.adaptive:
            idx = list(range(4)) + [i for i, s in enumerate(w.points) if s.snr >= 50.0]
        else:
            idx = list(range(0, len(pts), max(1, len(pts) // 32)))[:32]
        sub = [pts[i] for i in idx]
        cs = [counts[i] for i in idx]
        hs = ile.RiftILE(sub, precision="fp32", tau_width=w.tau_width)
        h64 = ile.RiftILE(sub, precision="fp64", tau_width=w.tau_width)
        ns = len(sub)
        per_round = sum(cs)
        rounds = m["rounds"]
        mask = 0x3F if w.adaptive else 0

        def replay(kw):
            res32, th, lw = hs.marginalize(seed + 13, cs, n_rounds=rounds, adapt_mask=mask, floor_eps=0.1,
                                           return_samples=True, **kw)
            deltas = []
            for i in range(ns):
                cols = torch.cat([torch.arange(r * per_round + sum(cs[:i]), r * per_round + sum(cs[:i + 1]),
                                               device=th.device) for r in range(rounds)])
                t_i = th[:, cols]
                l32 = hs.lnL(t_i, [(i, 0, t_i.shape[1])])
                l64 = h64.lnL(t_i.double(), [(i, 0, t_i.shape[1])])
                r64 = h64.reduce(l64 + (lw[cols].double() - l32.double()))
                deltas.append(abs(res32[i]["lnL_marg"] - r64["lnL_marg"]))
            return {"points": idx, "snr": [round(w.points[i].snr, 2) for i in idx], "samples": per_round * rounds,
                    "max_abs_delta_lnL_marg": max(deltas), "abs_delta_lnL_marg": deltas,
                    "n_eff": [r["n_eff"] for r in res32]}

        out["fp64_replay"] = replay({})
        if w.adaptive and not args.no_extras:
            # the same with the Gaussian-mixture proposal and the pairs (psi, phi), (iota, D)
            out["fp64_replay_gmm"] = replay(dict(gmm_components=3, gmm_pairs=((2, 4), (3, 5))))
        hs.close()
        h64.close()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pts, counts, w.precision, args.cpu_seconds, args.cpu_runs, w.tau_width)
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
