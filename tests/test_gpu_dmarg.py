"""GPU parity of distance marginalization (Sec. III.B, distance
marginalization): ln L_tD from the library (FP64 plain kernel, FP32 matrix
cores, FP32 plain kernel) against the oracle's composite quadrature on the
same seeded samples, with the distance row of theta not read; an adaptive
run over the six other parameters following the oracle's run; the refusals
(adapted distance, adjoint, gradient refinement, checkpoint of another
setting).

Tolerances.  FP64: the library's rule (3 x 24 Gauss-Legendre nodes in ln x
on the envelope's interval, T = 50) is within 1e-10 of the integral, so
1e-8 (1 + |ln L_tD|).  FP32: the window values carry the FP32 rounding of
the forward path, scaled by the node x_i, so the bound of the forward tests
applies with B taken at the integrand's peak, B(x*) = x*^2 B_1 with
x* = A_max / 2 B_1 clamped to the prior's range, plus 2e-5 for the 24-node
rule (T = 30: below 1e-5 on the oracle's cases)."""
import math

import numpy as np
import pytest
import torch

import synth
from test_gpu_parity import _fp32_tol, _handle, _say

pytestmark = pytest.mark.gpu

D_MIN, D_MAX = 10.0, 1000.0


@pytest.fixture(scope="module")
def ile():
    from paper_2210_07912_amd import ile as m
    m.lib()
    return m


def _peak_B(orc, op, d, th):
    """B at the integrand's peak x* = clamp(A_max / 2 B_1) for every sample."""
    out = np.zeros(th.shape[1])
    xlo, xhi = d["d_ref"] / D_MAX, d["d_ref"] / D_MIN
    for i in range(th.shape[1]):
        t = th[:, i].copy()
        t[5] = d["d_ref"]
        B1 = orc.coeffs(op, t)[1]
        A = orc.ell(op, t).max() + B1
        x = min(max(A / (2 * B1), xlo), xhi) if B1 > 0 else xhi
        out[i] = x * x * B1
    return out


def _samples(d, seed, n, nan_frac=0.5):
    th = synth.mixed_samples(d, seed, n)
    th[5, : int(n * nan_frac)] = np.nan  # the distance row is not read
    return th


def _cases():
    w = synth.workload("tiny_batched")
    specs = [synth.workload("tiny").points[0]] + list(w.points)
    return [synth.make_point(s) for s in specs]


def test_dmarg_fp64_matches_oracle(ile, orc):
    pts = _cases()
    ths, refs, items, off = [], [], [], 0
    for i, d in enumerate(pts):
        th = _samples(d, 500 + i, 160)
        ths.append(th)
        refs.append(orc.lnL_tD(orc.Point.from_dict(d), th))
        items.append((i, off, th.shape[1]))
        off += th.shape[1]
    h = _handle(ile, pts, "fp64")
    h.set_distance_marginalization(True)
    _say(f"dmarg fp64: {len(pts)} points, {off} samples")
    out = h.lnL(torch.tensor(np.concatenate(ths, axis=1)), items).cpu().numpy()
    for i, (_, o, n) in enumerate(items):
        err = np.abs(out[o:o + n] - refs[i])
        _say(f"  point {i}: max|d| {err.max():.2e}")
        assert np.all(err <= 1e-8 * (1 + np.abs(refs[i]))), (i, np.flatnonzero(err > 1e-8 * (1 + np.abs(refs[i])))[:5])
    h.close()


@pytest.mark.parametrize("plain", [False, True])
def test_dmarg_fp32_matches_oracle(ile, orc, plain):
    pts = _cases()
    ths, refs, ops, items, off = [], [], [], [], 0
    for i, d in enumerate(pts):
        th = _samples(d, 600 + i, 200).astype(np.float32).astype(np.float64)
        ths.append(th)
        ops.append(orc.Point.from_dict(d, complex64=True))
        refs.append(orc.lnL_tD(ops[-1], th))
        items.append((i, off, th.shape[1]))
        off += th.shape[1]
    h = _handle(ile, pts, "fp32", plain=plain)
    h.set_distance_marginalization(True)
    _say(f"dmarg fp32 plain={plain}: {len(pts)} points, {off} samples")
    out = h.lnL(torch.tensor(np.concatenate(ths, axis=1), dtype=torch.float32), items).cpu().numpy()
    for i, (_, o, n) in enumerate(items):
        got = out[o:o + n].astype(np.float64)
        Bp = _peak_B(orc, ops[i], pts[i], ths[i])
        tol = _fp32_tol(refs[i], Bp, ops[i].K, ops[i].M) + 2e-5
        err = np.abs(got - refs[i])
        _say(f"  point {i}: max|d| {err.max():.2e}, max |d|/tol {np.max(err / tol):.3f}")
        assert np.all(err <= tol), (i, np.flatnonzero(~(err <= tol))[:5], got[~(err <= tol)][:3], refs[i][~(err <= tol)][:3])
    h.close()


@pytest.mark.parametrize("which", ["single", "loud"])
def test_dmarg_full_size_sampled(ile, orc, which):
    """The single-point workload's shape at 2e5 samples, and the loudest
    adaptive point (SNR near 60): 256 sampled columns against the oracle."""
    if which == "single":
        spec = synth.workload("single").points[0]
    else:
        w = synth.workload("adaptive")
        spec = w.points[max(range(len(w.points)), key=lambda i: w.points[i].snr)]
    d = synth.make_point(spec)
    n = 200_000
    th = _samples(d, 700, n, nan_frac=0.25).astype(np.float32).astype(np.float64)
    h = _handle(ile, [d], "fp32")
    h.set_distance_marginalization(True)
    _say(f"dmarg {which} n={n}")
    out = h.lnL(torch.tensor(th, dtype=torch.float32)).cpu().numpy().astype(np.float64)
    assert np.isfinite(out).all()
    cols = np.random.default_rng(3).choice(n, 256, replace=False)
    cols[:16] = np.arange(n // 2, n // 2 + 16)  # some near the injection (second half: mixed draws near it)
    op = orc.Point.from_dict(d, complex64=True)
    ref = orc.lnL_tD(op, th[:, cols])
    Bp = _peak_B(orc, op, d, th[:, cols])
    tol = _fp32_tol(ref, Bp, op.K, op.M) + 2e-5
    err = np.abs(out[cols] - ref)
    _say(f"  max|d| {err.max():.2e}, max |d|/tol {np.max(err / tol):.3f}, lnL_tD range {ref.min():.1f}..{ref.max():.1f}")
    assert np.all(err <= tol)
    h.close()


def _oracle_marginalize_dm(orc, pts, seed, counts, rounds, mask, eps):
    """The oracle's adaptive run with distance marginalization: draws of the
    other six parameters (histograms over mask), ln w = ln L_tD + ln ratio,
    adaptation, pooled over rounds."""
    cdf = [None] * len(pts)
    masks = [0] * len(pts)
    lnw_all = [[] for _ in pts]
    for r in range(rounds):
        for i, (p, n) in enumerate(zip(pts, counts)):
            th, lr, bins, _ = orc.draw(seed, i, r, n, cdf=cdf[i], adapt_mask=masks[i])
            lnw = orc.lnL_tD(p, th) + lr
            lnw_all[i].append(lnw)
            if r + 1 < rounds:
                cdf[i] = orc.adapt(bins, lnw, floor_eps=eps, adapt_mask=mask)
                masks[i] = mask
    return [orc.reduce(np.concatenate(x)) for x in lnw_all]


def test_dmarg_marginalize_follows_oracle(ile, orc):
    w = synth.workload("tiny_batched")
    pts = [synth.make_point(s) for s in w.points[:2]]
    counts = [1500, 1200]
    seed, rounds, mask, eps = 2210079132, 3, 0x1F, 0.1
    ref = _oracle_marginalize_dm(orc, [orc.Point.from_dict(d) for d in pts], seed, counts, rounds, mask, eps)
    h = _handle(ile, pts, "fp64")
    h.set_distance_marginalization(True)
    _say("dmarg adaptive marginalize fp64")
    res = h.marginalize(seed, counts, n_rounds=rounds, adapt_mask=mask, floor_eps=eps)
    for r, o in zip(res, ref):
        _say(f"  gpu {r['lnL_marg']:.9f} oracle {o['lnL_marg']:.9f} n_eff {r['n_eff']:.1f}/{o['n_eff']:.1f}")
        assert r["n"] == o["n"]
        assert abs(r["lnL_marg"] - o["lnL_marg"]) < 1e-6
    # refusals: an adapted distance, the adjoint, the gradient refinement, a
    # checkpoint taken with another setting
    for kw in (dict(adapt_mask=0x3F), dict(adapt_mask=0x1F, gradient=True)):
        with pytest.raises(ile.RiftError) as e:
            h.marginalize(seed, counts, n_rounds=1, floor_eps=eps, **kw)
        assert e.value.status == -1
    with pytest.raises(ile.RiftError) as e:
        h.backward(torch.zeros((7, 4), dtype=torch.float64, device="cuda"))
    assert e.value.status == -1
    ck = h.save_checkpoint()
    h2 = _handle(ile, pts, "fp64")
    with pytest.raises(ile.RiftError) as e:
        h2.load_checkpoint(ck)
    assert "distance marginalization 1" in str(e.value)
    h2.set_distance_marginalization(True)
    h2.load_checkpoint(ck)
    h2.close()
    h.close()


def test_dmarg_fp32_marginalize_against_fp64_replay(ile, orc):
    """FP32 adaptive run with distance marginalization (sky, polarization,
    inclination, phase adapted) against the FP64 handle re-evaluating the
    very same samples and ratios: |d ln L_marg| <= 1e-3."""
    w = synth.workload("tiny_batched")
    pts = [synth.make_point(s) for s in w.points[:4]]
    counts = [4000, 3000, 3500, 2000]
    h = _handle(ile, pts, "fp32")
    h.set_distance_marginalization(True)
    h64 = _handle(ile, pts, "fp64")
    h64.set_distance_marginalization(True)
    rounds = 3
    res, th, lw = h.marginalize(2210079133, counts, n_rounds=rounds, adapt_mask=0x1F, floor_eps=0.1,
                                return_samples=True)
    per_round = sum(counts)
    offs = np.concatenate([[0], np.cumsum(counts)])
    items = [(i, int(offs[i]), counts[i]) for i in range(len(pts))]
    for i in range(len(pts)):
        cols = torch.tensor(np.concatenate([np.arange(r * per_round + offs[i], r * per_round + offs[i] + counts[i])
                                            for r in range(rounds)]), device=th.device)
        t = th[:, cols]
        l32 = h.lnL(t, [(i, 0, t.shape[1])])
        l64 = h64.lnL(t.double(), [(i, 0, t.shape[1])])
        r64 = h64.reduce(l64 + (lw[cols].double() - l32.double()))
        _say(f"  point {i}: fp32 {res[i]['lnL_marg']:.9f} fp64 replay {r64['lnL_marg']:.9f} n_eff {res[i]['n_eff']:.1f}")
        assert abs(res[i]["lnL_marg"] - r64["lnL_marg"]) < 1e-3
    del items
    h.close()
    h64.close()


def test_dmarg_edge_cases(ile, orc):
    """Degenerate integrands: no quadratic term (U = 0, every row of Q the
    same, so ell_j = A D_ref / D: the envelope has no interior maximum for
    A < 0 and one at x = 3 / A for A > 0), against the oracle's integral
    (itself pinned by the exponential-integral closed form); and a prior
    range narrowed to 2e-6 of its width, where ln L_tD must equal ln L_t at
    that distance (the time-only evaluation of the same handle type)."""
    spec = synth.workload("tiny").points[0]
    d = synth.make_point(spec)
    flat = dict(d)
    q = np.zeros_like(d["Q"])
    q[:] = d["Q"][:, d["Q"].shape[1] // 2: d["Q"].shape[1] // 2 + 1, :]
    flat["Q"], flat["U"] = q, np.zeros_like(d["U"])
    th = synth.prior_samples(31, 300)
    for prec in ("fp64", "fp32"):
        h = _handle(ile, [flat], prec)
        h.set_distance_marginalization(True)
        t = th.astype(np.float32).astype(np.float64) if prec == "fp32" else th
        got = h.lnL(torch.tensor(t, dtype=torch.float32 if prec == "fp32" else torch.float64)).cpu().numpy()
        ref = orc.lnL_tD(orc.Point.from_dict(flat, complex64=(prec == "fp32")), t)
        err = np.abs(got - ref)
        tol = (1e-8 if prec == "fp64" else 2e-5) * (1 + np.abs(ref))
        _say(f"dmarg U = 0 {prec}: max|d| {err.max():.2e}, ln L_tD {ref.min():.2f}..{ref.max():.2f}")
        assert np.all(err <= tol)
        h.close()
    D0 = 321.0
    th2 = synth.mixed_samples(d, 32, 200)
    th2[5] = D0
    for prec in ("fp64", "fp32"):
        h = _handle(ile, [d], prec, d_min=D0 * (1 - 1e-6), d_max=D0 * (1 + 1e-6))
        dt = torch.float32 if prec == "fp32" else torch.float64
        lt = h.lnL(torch.tensor(th2, dtype=dt)).cpu().numpy().astype(np.float64)
        h.set_distance_marginalization(True)
        ld = h.lnL(torch.tensor(th2, dtype=dt)).cpu().numpy().astype(np.float64)
        err = np.abs(ld - lt)
        _say(f"dmarg narrow prior {prec}: max|d| {err.max():.2e}")
        assert np.all(err <= (1e-7 if prec == "fp64" else 5e-4) * (1 + np.abs(lt)))
        h.close()
