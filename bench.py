"""Benchmark of the ILE marginalized-likelihood step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload single]

A step is one pass of the whole hot path over one batch: on-device sampling
of the extrinsic parameters, ln L_t for every sample (geometry, harmonics,
coefficients, the time-shifted contraction, interpolation and the window
log-sum-exp), ln w, and the FP64 reduction to ln L_marg with n_eff, n_ESS and
n_var (one call of rift_ile_marginalize).  Inputs (Q, U) are resident in HBM
before the timed region.  The steps are timed twice, with direct launches (the
evaluation kernel timed with HIP events for the roofline) and with each
evaluation run replayed from a captured hipGraph; for FP32 workloads other
than the gradient the replayed rate is the headline value.  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma_tflops": 157.3, "fp64_tflops": 78.6, "hbm_gbs": 8000.0}

# HBM bytes per launch of the evaluation kernel for the default workload, from
# rocprofv3 FETCH_SIZE (x 2.0) and WRITE_SIZE (x 1.0) passes, the factors read
# off a plain device copy (profiles/mfma_kernel_single_1e6.md).  It describes
# the kernel as it was measured and is reported for that workload only.
MEASURED_TRAFFIC = {"single": 377580268.0}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single",
                    help="plain | single | batched | grad | adaptive (default: single, 1e6 samples)")
    ap.add_argument("--n", type=int, default=0, help="samples per step (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the measurements beside the timed steps (precompute, network frame, refinement)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (points would shard across GPUs "
              "with one 40-byte FP64 exchange per point)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2210_07912_amd import ile

    w = synth.workload(args.workload)
    pts = [synth.make_point(s) for s in w.points]
    n = args.n or w.n_samples[0]
    counts = [n] * len(pts) if args.n else list(w.n_samples)
    h = ile.RiftILE(pts, precision=w.precision, tau_width=w.tau_width)
    seed = synth.BASE_SEED + synth.WORKLOADS.index(args.workload)
    rounds = w.rounds if w.adaptive else 1
    mask = 0x3F if w.adaptive else 0
    grad = args.workload == "grad"
    if grad:
        # a step: draw the samples on the device, then ln L_t and its gradient
        # in the seven parameters (one adjoint launch)
        def step(i):
            th, _, _ = h.sample(0, seed + i, 0, counts[0])
            g, lt = h.backward(th, want_lnL=True)
            return [h.reduce(lt)]
    else:
        def step(i):
            return h.marginalize(seed + i, counts, n_rounds=rounds, adapt_mask=mask, floor_eps=0.1)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    h.profile(True)
    t0 = time.perf_counter()
    res = None
    for i in range(args.steps):
        res = step(100 + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = h.profile(False)
    evals_per_step = sum(counts) * rounds
    dt = (t1 - t0) / args.steps
    value = evals_per_step / dt

    # roofline of the dominant kernel (the evaluation kernel): algorithmic
    # FLOP of the timed steps spread over its launches (a step makes one
    # launch per round and class of points), over its average duration
    per = flops_per_grad if grad else flops_per_eval
    fl = rounds * sum(c * per(p["det_pos"].shape[0], len(p["ell"]), p["n_t"]) for c, p in zip(counts, pts))
    fl_per_launch = fl * args.steps / max(k_launches, 1)
    k_avg_ms = k_ms / max(k_launches, 1)
    achieved = fl_per_launch / (k_avg_ms * 1e-3) / 1e12 if k_launches else None
    dtype = "f32" if w.precision == "fp32" else "f64"
    mfma = w.precision == "fp32"
    # the plain kernel (FP64 handles) is FP64 vector-ALU bound (78.6)
    peak = PEAK["fp32_mfma_tflops"] if mfma else PEAK["fp64_tflops"]
    roof = {"bound": "mfma" if mfma else "alu", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": (achieved / peak) if achieved else None,
            "traffic": MEASURED_TRAFFIC.get(args.workload) if not args.n else None,
            "kernel": ("mfma_bwd_kernel" if grad else "mfma_kernel") if mfma else "plain_kernel",
            "kernel_ms": k_avg_ms, "launches_per_step": k_launches / args.steps,
            "flops_per_eval": fl / max(rounds * sum(counts), 1)}
    if mfma:
        # matrix-core FLOP the forward kernel executes per evaluation: 16-row
        # blocks 0..ceil(n_t/16) of every detector times 2 M_p elements
        # (excluding the padding slots of partly filled tiles)
        ex = [2 * p["det_pos"].shape[0] * 16 * ((p["n_t"] + 15) // 16 + 1) * 2 * ((len(p["ell"]) + 1) // 2 * 2)
              for p in pts]
        # (the adjoint: z and the transposed product G_k, one sweep)
        roof["mfma_executed_per_eval"] = sum(c * e for c, e in zip(counts, ex)) / max(sum(counts), 1) * (2 if grad else 1)
    if roof["traffic"] and k_avg_ms:
        roof["hbm_gbs"] = roof["traffic"] / (k_avg_ms * 1e-3) / 1e9
        roof["hbm_frac"] = roof["hbm_gbs"] / PEAK["hbm_gbs"]

    out = {
        "metric": "extrinsic lnL evals/sec (time-marginalized) at |dln L_marg|<=1e-3 vs FP64",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "points": len(pts),
                   "samples_per_point": counts[0] if len(set(counts)) == 1 else "varied", "samples_per_step": evals_per_step,
                   "rounds": rounds, "K": [p["det_pos"].shape[0] for p in pts][:1], "M": [len(p["ell"]) for p in pts][:1],
                   "n_t": [p["n_t"] for p in pts][:1], "seed": seed},
        "roofline": roof,
        # matrix-core feed measured per (T, K) class by the handle (staged | direct)
        "autotune": ({f"T{t}K{k}": m for (t, k), m in sorted(h.autotune_table().items())}
                     if mfma and not grad else None),
        "lnL_marg": [r["lnL_marg"] for r in res][:4], "n_eff": [r["n_eff"] for r in res][:4],
    }

    # the same steps with the evaluation runs replayed from captured hipGraphs
    # (FP32 handles; host-timed, the kernel timing hook stays off)
    if not args.no_graph and w.precision == "fp32" and not grad:
        h.set_graph(True)
        for i in range(max(args.warmup, 1)):
            step(i)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for i in range(args.steps):
            step(100 + i)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        cap, rep = h.graph_stats()
        h.set_graph(False)
        gdt = (t3 - t2) / args.steps
        # the headline is the replayed form (same work per step: sampling,
        # evaluation and reduction); the direct launches stay beside it
        out["direct"] = {"value": value, "ms_per_step": dt * 1e3}
        out["value"] = evals_per_step / gdt
        out["ms_per_step"] = gdt * 1e3
        out["graph"] = {"captures": cap, "replays": rep}
        out["config"]["launch"] = "hipGraph replay of each evaluation run"
    else:
        out["config"]["launch"] = "direct"

    # the gradient configuration's second part: 20 rounds of 1e5 samples of
    # adaptive importance sampling, histogram proposal alone and refined by the
    # gradient (the top samples climb ln L_t along the adjoint between rounds)
    if grad and not args.n and not args.no_extras:
        ref = {}
        for name, gflag in (("histogram", False), ("gradient_refined", True)):
            h.marginalize(seed, counts[0], n_rounds=2, adapt_mask=0x3F, floor_eps=0.1, gradient=gflag)  # warm-up
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            r = h.marginalize(seed + 7, counts[0], n_rounds=w.rounds, adapt_mask=0x3F, floor_eps=0.1, gradient=gflag,
                              n_ascent=64, ascent_steps=12, ascent_mix=0.3)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            ref[name] = {"evals_per_s": counts[0] * w.rounds / (t3 - t2), "s": t3 - t2,
                         "lnL_marg": r[0]["lnL_marg"], "sigma_lnL": r[0]["sigma_lnL"], "n_eff": r[0]["n_eff"]}
        out["refinement"] = {"rounds": w.rounds, "samples_per_round": counts[0], "adapt": "alpha, delta, psi, iota, "
                             "phi, D histograms", **ref}

    # the Q/U/V precompute at the single-point shape: 3 detectors, 21 modes,
    # 8 s at 4096 Hz (N = 32768), the 999 stored rows; host arrays in and out
    if args.workload == "single" and not args.n and not args.no_extras:
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

    # adaptive sampling with the sky in each point's detector-network frame
    # against the equatorial frame: n_eff and sigma of ln L_marg on the first
    # points of the workload (10 rounds of 1e5 samples)
    if w.adaptive and not args.n and not args.no_extras:
        sub = pts[:8]
        hs = ile.RiftILE(sub, precision=w.precision, tau_width=w.tau_width)
        nf = {}
        for name, net in (("equatorial", False), ("network_frame", True)):
            hs.set_network_frame(net)
            r = hs.marginalize(seed + 11, 100_000, n_rounds=10, adapt_mask=0x3F, floor_eps=0.1)
            nf[name] = {"n_eff": [x["n_eff"] for x in r], "sigma_lnL": [x["sigma_lnL"] for x in r],
                        "lnL_marg": [x["lnL_marg"] for x in r]}
        out["network_frame"] = {"points": len(sub), "rounds": 10, "samples_per_round": 100_000, **nf}
        # the Gaussian-mixture proposal (3 components per parameter, 10 EM
        # iterations per round) against the histograms, equatorial frame
        hs.set_network_frame(False)
        gm = {}
        # correlated pairs (psi, phi) and (iota, D): the pairs the polarization-phase and
        # inclination-distance degeneracies tie together
        for name, kk, pr in (("histogram", 0, ()), ("gmm_k3", 3, ()), ("gmm_k3_pairs", 3, ((2, 4), (3, 5)))):
            hs.marginalize(seed + 12, 100_000, n_rounds=2, adapt_mask=0x3F, floor_eps=0.1, gmm_components=kk,
                           gmm_pairs=pr)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            r = hs.marginalize(seed + 13, 100_000, n_rounds=10, adapt_mask=0x3F, floor_eps=0.1, gmm_components=kk,
                               gmm_pairs=pr)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            gm[name] = {"ms": (t3 - t2) * 1e3, "n_eff": [x["n_eff"] for x in r], "discarded": [x["n_nonfinite"] for x in r],
                        "sigma_lnL": [x["sigma_lnL"] for x in r], "lnL_marg": [x["lnL_marg"] for x in r]}
        hs.close()
        out["gmm"] = {"points": len(sub), "rounds": 10, "samples_per_round": 100_000, "floor_eps": 0.1, **gm}

    # FP32 vs FP64 on the same samples (same GPU): |d ln L_marg| and the FP64 rate
    if not args.no_fp64 and w.precision == "fp32" and len(pts) == 1 and not grad:
        nn = min(counts[0], 200_000)
        h64 = ile.RiftILE(pts, precision="fp64", tau_width=w.tau_width)
        th64, _, _ = h64.sample(0, seed, 0, nn)
        th32 = th64.float()
        l32 = h.lnL(th32)
        l64a = h64.lnL(th32.double())
        torch.cuda.synchronize()
        h64.profile(True)
        t2 = time.perf_counter()
        l64 = h64.lnL(th32.double())
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        h64.profile(False)
        r32, r64 = h.reduce(l32), h64.reduce(l64)
        out["fp64_plain"] = {"evals_per_s": nn / (t3 - t2), "samples": nn,
                             "lnL_marg_fp32": r32["lnL_marg"], "lnL_marg_fp64": r64["lnL_marg"],
                             "abs_delta_lnL_marg": abs(r32["lnL_marg"] - r64["lnL_marg"]),
                             "max_abs_delta_lnL_t": float((l32.double() - l64a).abs().max())}
        h64.close()

    # the estimate against the FP64 plain form on the very same samples (their
    # samples and proposal ratios replayed): 4 points of the adaptive workload
    # over all rounds, 32 points of the batched workload
    if not args.no_fp64 and (w.adaptive or args.workload == "batched") and not args.n and not args.no_extras:
        sub = pts[:4] if w.adaptive else pts[:32]
        hs = ile.RiftILE(sub, precision="fp32", tau_width=w.tau_width)
        h64 = ile.RiftILE(sub, precision="fp64", tau_width=w.tau_width)
        ns = len(sub)
        per_round = sum(counts[:ns])

        def replay(kw):
            res32, th, lw = hs.marginalize(seed + 13, counts[:ns], n_rounds=rounds, adapt_mask=mask, floor_eps=0.1,
                                           return_samples=True, **kw)
            deltas = []
            for i in range(len(sub)):
                cols = torch.cat([torch.arange(r * per_round + sum(counts[:i]), r * per_round + sum(counts[:i + 1]),
                                               device=th.device) for r in range(rounds)])
                t_i = th[:, cols]
                l32 = hs.lnL(t_i, [(i, 0, t_i.shape[1])])
                l64 = h64.lnL(t_i.double(), [(i, 0, t_i.shape[1])])
                r64 = h64.reduce(l64 + (lw[cols].double() - l32.double()))
                deltas.append(abs(res32[i]["lnL_marg"] - r64["lnL_marg"]))
            return {"points": ns, "samples": per_round * rounds, "max_abs_delta_lnL_marg": max(deltas),
                    "abs_delta_lnL_marg": deltas, "n_eff": [r["n_eff"] for r in res32]}

        out["fp64_replay"] = replay({})
        if w.adaptive:
            # the same with the Gaussian-mixture proposal and the pairs (psi, phi), (iota, D)
            out["fp64_replay_gmm"] = replay(dict(gmm_components=3, gmm_pairs=((2, 4), (3, 5))))
        hs.close()
        h64.close()

    if not args.no_cpu_baseline:
        from oracle import oracle
        p = pts[0]
        op = oracle.Point.from_dict(p, complex64=(w.precision == "fp32"))
        th = synth.prior_samples(seed, 4096, w.tau_width)
        fn = oracle.grad if grad else oracle.lnL_t
        t_a = time.perf_counter()
        fn(op, th[:, :256])
        t_b = time.perf_counter()
        rate = 256 / (t_b - t_a)
        ns = int(min(4096, max(256, rate * args.cpu_seconds)))
        if ns > 256:
            t_a = time.perf_counter()
            fn(op, th[:, :ns])
            t_b = time.perf_counter()
            rate = ns / (t_b - t_a)
        out["cpu_baseline"] = {"value": rate, "unit": "evals/s", "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"{ns} prior samples of point 0 ({args.workload}), "
                               + ("ln L_t and gradient" if grad else "ln L_t only") + ", FP64",
                               "cpu_model": _cpu_model()}
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
