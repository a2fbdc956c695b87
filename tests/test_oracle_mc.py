"""Oracle pins for the Monte Carlo layer: Philox known-answer vectors, prior
transforms (Kolmogorov-Smirnov), histogram proposals, the sample-size
measures of App. B (closed forms and the App. B reweighting toy), and the
Monte Carlo estimate of a 2-parameter marginal likelihood against brute-force
quadrature."""
import math

import numpy as np
import pytest
from scipy import stats

import synth


def test_philox_known_answers(orc):
    # Random123 known-answer vectors for Philox4x32-10 (Salmon et al., SC'11)
    assert orc.philox([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert orc.philox([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert orc.philox([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == [
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_u01(orc):
    assert orc.u01(0) == 0.5 / 2 ** 24
    assert orc.u01(0xFFFFFFFF) == 1 - 0.5 / 2 ** 24
    assert np.float32(orc.u01(0x12345678)) == orc.u01(0x12345678)  # exact in FP32


def test_prior_draws_follow_the_priors(orc):
    n = 20000
    th, lr, bins, raw = orc.draw(2210079120, 3, 1, n, tau_width=1 / 4096)
    assert np.all(lr == 0.0)
    a3, b3 = 10.0 ** 3, 1000.0 ** 3
    cdfs = [
        lambda x: x / (2 * math.pi),
        lambda x: 0.5 * (np.sin(x) + 1),
        lambda x: x / math.pi,
        lambda x: 0.5 * (1 - np.cos(x)),
        lambda x: x / (2 * math.pi),
        lambda x: (x ** 3 - a3) / (b3 - a3),
        lambda x: x * 4096 + 0.5,
    ]
    for d in range(7):
        assert stats.kstest(th[d], cdfs[d]).pvalue > 1e-3, d
    # bins of prior dimensions: floor(u * nb) of the raw uniform
    u = ((raw[:7] >> 8).astype(np.float64) + 0.5) / 2 ** 24
    assert np.array_equal(bins, np.floor(u * 100).astype(np.uint8))
    # a different round or point gives an independent stream
    th2, _, _, _ = orc.draw(2210079120, 3, 2, n)
    assert abs(np.corrcoef(th[0], th2[0])[0, 1]) < 0.05


def _hl_positions():
    return np.array([synth.DETECTORS["H1"]["vertex"], synth.DETECTORS["L1"]["vertex"]])


def test_network_frame_axes(orc):
    """The network sky frame (Sec. II.A, rotated detector-network-frame sky
    coordinates): orthonormal, right-handed, north pole along the H1 -> L1
    baseline; for a baseline along the Earth's axis the fallback axis is used."""
    pos = _hl_positions()
    ax = orc.network_frame(pos)
    assert np.abs(ax @ ax.T - np.eye(3)).max() < 1e-14
    assert abs(np.linalg.det(ax) - 1.0) < 1e-14
    b = pos[1] - pos[0]
    assert np.abs(ax[2] - b / np.linalg.norm(b)).max() < 1e-15
    polar = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 5.0]])
    ax2 = orc.network_frame(polar)
    assert np.abs(ax2 @ ax2.T - np.eye(3)).max() < 1e-14 and np.allclose(ax2[2], [0, 0, 1])


def test_network_frame_draws(orc):
    """Sky drawn in the network frame: (i) still the isotropic prior (alpha
    uniform, sin(delta) uniform: Kolmogorov-Smirnov), with ln p - ln p_s = 0;
    (ii) the H1 - L1 arrival-time difference is a function of the frame's
    polar coordinate alone, dt = -|b| cos(theta') / c with cos(theta') =
    2 u - 1 of the sample's raw uniform; (iii) frame_u inverts the draw; the
    other five parameters and the bins equal those of the equatorial draw."""
    pos = _hl_positions()
    gmst = 1.234
    n = 20000
    th, lr, bins, raw = orc.draw(2210079120, 3, 1, n, tau_width=1 / 4096, frame=(pos, gmst))
    assert np.all(lr == 0.0)
    assert stats.kstest(th[0], lambda x: x / (2 * math.pi)).pvalue > 1e-3
    assert stats.kstest(th[1], lambda x: 0.5 * (np.sin(x) + 1)).pvalue > 1e-3
    u = ((raw[:2] >> 8).astype(np.float64) + 0.5) / 2 ** 24
    h = th[0] - gmst
    nhat = np.array([np.cos(th[1]) * np.cos(h), np.cos(th[1]) * np.sin(h), np.sin(th[1])])
    b = pos[1] - pos[0]
    c = 299792458.0
    dt = -(b @ nhat) / c
    assert np.abs(dt - (-np.linalg.norm(b) * (2 * u[1] - 1) / c)).max() < 1e-15
    for i in range(0, n, 997):
        u0, u1 = orc.frame_u(pos, gmst, th[0, i], th[1, i])
        assert abs(u1 - u[1, i]) < 1e-12
        assert min(abs(u0 - u[0, i]), 1 - abs(u0 - u[0, i])) < 1e-12
    th_e, lr_e, bins_e, raw_e = orc.draw(2210079120, 3, 1, n, tau_width=1 / 4096)
    assert np.array_equal(th[2:], th_e[2:]) and np.array_equal(bins, bins_e) and np.array_equal(raw, raw_e)


def _modes(d, keep):
    """The point restricted to the modes listed in keep."""
    e, idx = dict(d), np.asarray(keep)
    e["Q"] = d["Q"][:, :, idx]
    e["U"] = d["U"][:, idx][:, :, idx]
    if d.get("V") is not None:
        e["V"] = d["V"][:, idx][:, :, idx]
    e["ell"], e["em"] = np.asarray(d["ell"])[idx], np.asarray(d["em"])[idx]
    return e


def test_phase_rotation_map(orc):
    """(u_s, u_d) -> (psi, phi): into [0, pi) x [0, 2 pi), exactly four
    preimages in the unit square for every image point (u_s - u_d fixed mod
    1/2, u_s + u_d mod 1), constant Jacobian 8 pi^2 = 4 x the torus area, so
    the uniform measure goes to the uniform measure."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        psi, phi = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
        pre = []
        for a in range(-2, 3):
            for b in range(-2, 3):
                x, y = psi / (2 * math.pi) + a / 2, phi / (2 * math.pi) + b
                us, ud = (x + y) / 2, (y - x) / 2
                if 0 <= us < 1 and 0 <= ud < 1:
                    pre.append((us, ud))
        assert len(pre) == 4
        for us, ud in pre:
            p2, f2 = orc.phase_rot(us, ud)
            assert abs(p2 - psi) < 1e-12 or abs(abs(p2 - psi) - math.pi) < 1e-12
            assert abs(f2 - phi) < 1e-12 or abs(abs(f2 - phi) - 2 * math.pi) < 1e-12
    h = 1e-7
    for us, ud in rng.uniform(0.05, 0.95, size=(50, 2)):
        p0, f0 = orc.phase_rot(us, ud)
        p1, f1 = orc.phase_rot(us + h, ud)
        p2, f2 = orc.phase_rot(us, ud + h)
        J = np.array([[p1 - p0, p2 - p0], [f1 - f0, f2 - f0]]) / h
        if np.abs(J).max() < 100:  # not across a wrap
            assert abs(abs(np.linalg.det(J)) - 8 * math.pi ** 2) < 1e-5
    for us, ud in rng.uniform(0, 1, size=(1000, 2)):
        p0, f0 = orc.phase_rot(us, ud)
        assert 0 <= p0 < math.pi and 0 <= f0 < 2 * math.pi


def test_phase_rotated_draws(orc):
    """Draws in phase-rotated coordinates: (psi, phi) jointly uniform on the
    torus (Kolmogorov-Smirnov per axis, chi^2 on an 8 x 8 grid), ln p - ln p_s
    = 0 for the prior, theta[psi, phi] the map of the raw uniforms of those
    two dimensions, everything else as in the plain draw (bins, raw words,
    the other five parameters; with the network frame too)."""
    n = 20000
    th, lr, bins, raw = orc.draw(2210079120, 3, 1, n, tau_width=1 / 4096, phase=True)
    assert np.all(lr == 0.0)
    assert stats.kstest(th[2], lambda x: x / math.pi).pvalue > 1e-3
    assert stats.kstest(th[4], lambda x: x / (2 * math.pi)).pvalue > 1e-3
    cnt, _, _ = np.histogram2d(th[2], th[4], bins=8, range=[[0, math.pi], [0, 2 * math.pi]])
    chi2 = ((cnt - n / 64) ** 2 / (n / 64)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-3
    u = ((raw[:7] >> 8).astype(np.float64) + 0.5) / 2 ** 24
    for i in range(0, n, 211):
        assert (th[2, i], th[4, i]) == orc.phase_rot(u[2, i], u[4, i])
    th_e, lr_e, bins_e, raw_e = orc.draw(2210079120, 3, 1, n, tau_width=1 / 4096)
    keep = [0, 1, 3, 5, 6]
    assert np.array_equal(th[keep], th_e[keep]) and np.array_equal(bins, bins_e) and np.array_equal(raw, raw_e)
    pos = _hl_positions()
    th_f, _, _, _ = orc.draw(2210079120, 3, 1, 500, tau_width=1 / 4096, frame=(pos, 0.4), phase=True)
    th_g, _, _, _ = orc.draw(2210079120, 3, 1, 500, tau_width=1 / 4096, frame=(pos, 0.4))
    assert np.array_equal(th_f[[0, 1, 3, 5, 6]], th_g[[0, 1, 3, 5, 6]])
    assert np.array_equal(th_f[[2, 4]], th[[2, 4], :500])


def test_phase_rotated_coordinates_separate_the_modes(orc):
    """The point of the coordinates: with only the (2, 2) mode, ln L_t does
    not depend on u_s (the likelihood is flat along phi + psi); with only the
    (2, -2) mode it does not depend on u_d; with both it depends on both."""
    d = synth.make_point(synth.PIN_SPECS[5])
    ell, em = list(d["ell"]), list(d["em"])
    i22 = [i for i in range(len(ell)) if ell[i] == 2 and em[i] == 2]
    i2m = [i for i in range(len(ell)) if ell[i] == 2 and em[i] == -2]
    assert i22 and i2m
    th = np.tile(d["theta_inj"][:, None], (1, 16)).astype(np.float64)
    th[3] = 1.2  # inclined, so that both modes carry weight
    rng = np.random.default_rng(5)

    def spread(p, fixed):
        out = []
        for _ in range(4):
            c = rng.uniform()
            v = rng.uniform(size=16)
            us, ud = (v, np.full(16, c)) if fixed == "ud" else (np.full(16, c), v)
            t = th.copy()
            for j in range(16):
                t[2, j], t[4, j] = orc.phase_rot(us[j], ud[j])
            out.append(np.ptp(orc.lnL_t(p, t)))
        return max(out)

    p22 = orc.Point.from_dict(_modes(d, i22))
    p2m = orc.Point.from_dict(_modes(d, i2m))
    pall = orc.Point.from_dict(d)
    assert spread(p22, "ud") < 1e-9 and spread(p22, "us") > 1e-2
    assert spread(p2m, "us") < 1e-9 and spread(p2m, "ud") > 1e-2
    assert spread(pall, "ud") > 1e-2 and spread(pall, "us") > 1e-2


def test_phase_rotated_mc_matches_quadrature(orc):
    """Marginalize over (psi, phi) with the other parameters at the
    injection: histogram proposals adapted in (u_s, u_d) over three rounds,
    pooled, against the periodic trapezoid rule on the torus (spectrally
    accurate for this smooth periodic integrand)."""
    spec = synth.PIN_SPECS[5]
    d = synth.make_point(spec)
    p = orc.Point.from_dict(d)
    t0 = d["theta_inj"]

    def lnL_pp(psi, phi):
        th = np.tile(t0[:, None], (1, psi.size))
        th[2], th[4] = psi, phi
        return orc.lnL_t(p, th)

    def quad(n):
        ps = np.arange(n) * math.pi / n
        fs = np.arange(2 * n) * math.pi / n
        P, F = np.meshgrid(ps, fs, indexing="ij")
        lnl = lnL_pp(P.ravel(), F.ravel())
        m = lnl.max()
        return m + math.log(np.exp(lnl - m).mean())

    q1, q2 = quad(96), quad(128)
    assert abs(q1 - q2) < 1e-9
    cdf, mask, lnw_all = None, 0, []
    for r in range(3):
        th, lr, bins, _ = orc.draw(91, 0, r, 20000, cdf=cdf, adapt_mask=mask, phase=True)
        lnw = lnL_pp(th[2], th[4]) + lr
        lnw_all.append(lnw)
        cdf = orc.adapt(bins, lnw, floor_eps=0.1, adapt_mask=0b10100)
        mask = 0b10100
    r = orc.reduce(np.concatenate(lnw_all))
    assert r["n_var"] > 1000
    assert abs(r["lnL_marg"] - q2) < 4 * r["sigma_lnL"], (r, q2)


def test_histogram_proposal(orc):
    rng = np.random.default_rng(8)
    nb = 100
    cdf = np.zeros((7, nb + 1))
    masses = rng.dirichlet(np.ones(nb) * 0.7, size=7)
    cdf[:, 1:] = np.cumsum(masses, axis=1)
    cdf[:, -1] = 1.0
    mask = 0b0111011
    n = 40000
    th, lr, bins, raw = orc.draw(99, 0, 4, n, cdf=cdf, adapt_mask=mask)
    expect_lr = np.zeros(n)
    for d in range(7):
        if (mask >> d) & 1:
            mass = cdf[d, 1:] - cdf[d, :-1]
            expect_lr -= np.log(nb * mass[bins[d]])
            counts = np.bincount(bins[d], minlength=nb)
            ok = mass * n > 20
            chi2 = ((counts[ok] - n * mass[ok]) ** 2 / (n * mass[ok])).sum()
            assert stats.chi2.sf(chi2, ok.sum() - 1) > 1e-3
        else:
            # a prior dimension: the bin is floor(100 u) of a uniform, so the
            # counts are uniform over the 100 bins
            counts = np.bincount(bins[d], minlength=nb)
            chi2 = ((counts - n / nb) ** 2 / (n / nb)).sum()
            assert stats.chi2.sf(chi2, nb - 1) > 1e-3, (d, chi2)
    assert np.allclose(lr, expect_lr, atol=1e-12)
    # the prior-CDF coordinate of each sample lies inside its bin (tau is
    # fixed at 0 here, so it has no coordinate)
    for d in range(6):
        u = np.array([_ucoord(orc, d, th[:, i]) for i in range(0, n, 97)])
        b = bins[d, ::97]
        assert np.all(u >= b / nb - 1e-9) and np.all(u <= (b + 1) / nb + 1e-9)


def _ucoord(orc, d, th):
    a3, b3 = 1e3, 1e9
    t = th[d]
    return [t / (2 * math.pi), 0.5 * (math.sin(t) + 1), t / math.pi, 0.5 * (1 + math.cos(t)),
            t / (2 * math.pi), (t ** 3 - a3) / (b3 - a3), 0.5][d]


def test_reduce_closed_forms(orc):
    n = 1000
    r = orc.reduce(np.full(n, -3.5))
    assert r["lnL_marg"] == pytest.approx(-3.5, abs=1e-14)
    assert r["n_eff"] == pytest.approx(n) and r["n_ess"] == pytest.approx(n)
    lnw = np.full(n, -np.inf); lnw[17] = 2.0
    r = orc.reduce(lnw)
    assert r["n_eff"] == 1.0 and r["n_ess"] == 1.0
    assert r["lnL_marg"] == pytest.approx(2.0 - math.log(n), abs=1e-14)
    lnw = np.array([0.0, math.log(3.0), np.nan, np.inf])
    r = orc.reduce(lnw)
    assert r["n_nonfinite"] == 2 and r["n"] == 2
    assert r["lnL_marg"] == pytest.approx(math.log(2.0), abs=1e-14)
    assert r["n_ess"] == pytest.approx(16 / 10)
    # unbiased variance: w = (1, 3): mean 2, s^2 = 2, n_var = 2 * 4 / 2
    assert r["n_var"] == pytest.approx(4.0)
    # huge log weights do not overflow (App. D.2 log-space sums)
    r = orc.reduce(np.array([1000.0, 1000.0 + math.log(3)]))
    assert r["lnL_marg"] == pytest.approx(1000 + math.log(2), abs=1e-12)


def test_appendix_b_toy(orc):
    """App. B toy: L = 1, p = 1, p_s = alpha x^(alpha-1) on [0, 1].  E[w] = 1;
    Var(w) = (1-alpha)^2 / (alpha (2-alpha)) for alpha < 2; for alpha > 1 the
    median n_eff ~ N alpha (N / ln 2)^(-(alpha-1)/alpha)."""
    rng = np.random.default_rng(12)
    N = 200000
    alpha = 1.2
    x = rng.random(N) ** (1 / alpha)
    lnw = -np.log(alpha) - (alpha - 1) * np.log(x)
    r = orc.reduce(lnw)
    assert abs(r["lnL_marg"]) < 4 * r["sigma_lnL"]
    V = (1 - alpha) ** 2 / (alpha * (2 - alpha))
    assert r["n_var"] == pytest.approx(N / V, rel=0.05)
    alpha, N = 3.0, 10000
    neffs = []
    for _ in range(201):
        x = rng.random(N) ** (1 / alpha)
        neffs.append(orc.reduce(-np.log(alpha) - (alpha - 1) * np.log(x))["n_eff"])
    pred = N * alpha * (N / math.log(2)) ** (-(alpha - 1) / alpha)
    assert np.median(neffs) == pytest.approx(pred, rel=0.12)


def test_mc_matches_quadrature(orc):
    """Marginalize over (cos iota, D) with the other extrinsic parameters at
    the injection: Eq. (lnL:MonteCarlo) with prior samples vs a composite
    Gauss-Legendre rule."""
    spec = synth.PIN_SPECS[5]
    d = synth.make_point(spec)
    p = orc.Point.from_dict(d)
    t0 = d["theta_inj"]

    def lnL_grid(ci, D):
        th = np.tile(t0[:, None], (1, ci.size))
        th[3] = np.arccos(ci)
        th[5] = D
        return orc.lnL_t(p, th)

    def quad(n_c, n_sub, n_per):
        xc, wc = np.polynomial.legendre.leggauss(n_c)
        xs, ws = np.polynomial.legendre.leggauss(n_per)
        edges = np.linspace(10.0, 1000.0, n_sub + 1)
        Ds = np.concatenate([0.5 * (b - a) * xs + 0.5 * (a + b) for a, b in zip(edges[:-1], edges[1:])])
        wD = np.concatenate([0.5 * (b - a) * ws for a, b in zip(edges[:-1], edges[1:])])
        pD = 3 * Ds ** 2 / (1000.0 ** 3 - 10.0 ** 3)
        CI, DD = np.meshgrid(xc, Ds, indexing="ij")
        lnl = lnL_grid(CI.ravel(), DD.ravel()).reshape(CI.shape)
        wts = (wc[:, None] * 0.5) * (wD * pD)[None, :]
        m = lnl.max()
        return m + math.log((wts * np.exp(lnl - m)).sum())

    q1 = quad(120, 30, 16)
    q2 = quad(160, 40, 20)
    assert abs(q1 - q2) < 1e-6
    th, lr, _, _ = orc.draw(77, 0, 0, 100000)
    lnl = lnL_grid(np.cos(th[3]), th[5])
    r = orc.reduce(lnl + lr)
    assert r["n_var"] > 100
    assert abs(r["lnL_marg"] - q2) < 4 * r["sigma_lnL"], (r, q2)


def test_adapt_closed_forms(orc):
    nb, eps = 100, 0.1
    n = 500
    bins = np.zeros((7, n), np.uint8)
    bins[:] = 42
    lnw = np.zeros(n)
    cdf = orc.adapt(bins, lnw, nb=nb, floor_eps=eps, adapt_mask=0b1)
    mass = cdf[0, 1:] - cdf[0, :-1]
    assert mass[42] == pytest.approx((1 - eps) + eps / nb, abs=1e-15)
    assert mass[0] == pytest.approx(eps / nb, abs=1e-15)
    assert np.allclose(cdf[1], np.linspace(0, 1, nb + 1), atol=1e-15)  # not adapted: uniform
    # weights enter proportionally and are max-shifted
    rng = np.random.default_rng(1)
    bins = rng.integers(0, nb, (7, n)).astype(np.uint8)
    lnw = rng.normal(size=n) * 3 + 500.0
    lnw[5] = np.nan
    cdf = orc.adapt(bins, lnw, nb=nb, floor_eps=eps, adapt_mask=0x7F)
    for dd in range(7):
        w = np.where(np.isfinite(lnw), np.exp(lnw - np.nanmax(lnw)), 0.0)
        m = np.bincount(bins[dd], weights=w, minlength=nb)
        h = (1 - eps) * nb * m / m.sum() + eps
        assert np.allclose(cdf[dd, 1:] - cdf[dd, :-1], h / nb, atol=1e-14)
    assert np.all(cdf[:, -1] == 1.0)
