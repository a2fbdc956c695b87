"""Oracle pins for distance marginalization (Sec. III.B, distance
marginalization): ln L_tD = ln int p(D) (1/n_t) sum_j exp(ell_j(D)) dD with
p(D) = 3 D^2 / (d_max^3 - d_min^3).  Pinned by the linear-quadratic form of
ell_j in x = D_ref / D, closed forms for a vanishing data term (incomplete
gamma) and a vanishing quadratic term (exponential integral), scipy's
adaptive quadrature over the oracle's own ell_j(D), the Monte Carlo average
over prior distances, the narrow-prior limit and convergence in the panel
count."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import synth

D_MIN, D_MAX = 10.0, 1000.0


def _point(orc, spec, Q=None, U=None):
    d = synth.make_point(spec)
    if Q is not None:
        d["Q"] = Q(d["Q"])
    if U is not None:
        d["U"] = U(d["U"])
    return d, orc.Point.from_dict(d)


def _prior(D):
    return 3.0 * D * D / (D_MAX ** 3 - D_MIN ** 3)


def test_window_values_are_linear_quadratic_in_inverse_distance(orc):
    """ell_j(D) = x A_j - x^2 B_1 with x = D_ref / D: a_km scales as 1/D and
    B as 1/D^2 (App. D Eq. (def:lnL:Decomposed))."""
    d, p = _point(orc, synth.workload("tiny").points[0])
    th = synth.mixed_samples(d, 3, 8)
    for i in range(th.shape[1]):
        t = th[:, i].copy()
        t[5] = d["d_ref"]
        A = orc.ell(p, t)
        B1 = orc.coeffs(p, t)[1]
        A = A + B1
        for D in (13.0, 100.0, 377.0, 999.0):
            t[5] = D
            x = d["d_ref"] / D
            got = orc.ell(p, t)
            want = x * A - x * x * B1
            assert np.abs(got - want).max() <= 1e-12 * (np.abs(x * A).max() + x * x * B1)


def _gamma_upper(s, x):
    """Upper incomplete gamma for s = 1/2 - n by the recurrence
    Gamma(s + 1, x) = s Gamma(s, x) + x^s e^-x from Gamma(1/2, x)."""
    g, a = math.sqrt(math.pi) * special.erfc(math.sqrt(x)), 0.5
    while a > s + 0.25:
        g = (g - x ** (a - 1) * math.exp(-x)) / (a - 1)
        a -= 1
    return g


def test_no_data_term_closed_form(orc):
    """Q = 0: ln L_tD = ln int p(D) exp(-B_1 D_ref^2 / D^2) dD, which is
    (3/2) c^{3/2} [Gamma(-3/2, c/d_max^2) - Gamma(-3/2, c/d_min^2)] /
    (d_max^3 - d_min^3) with c = B_1 D_ref^2."""
    d, p = _point(orc, synth.workload("tiny").points[0], Q=lambda q: np.zeros_like(q))
    th = synth.prior_samples(11, 6)
    for i in range(th.shape[1]):
        B1 = orc.coeffs(p, np.r_[th[:5, i], d["d_ref"], th[6, i]])[1]
        c = B1 * d["d_ref"] ** 2
        want = 1.5 * c ** 1.5 * (_gamma_upper(-1.5, c / D_MAX ** 2) - _gamma_upper(-1.5, c / D_MIN ** 2))
        want = math.log(want / (D_MAX ** 3 - D_MIN ** 3))
        got = orc.lnL_tD(p, th[:, i])
        assert abs(got - want) < 1e-11 * max(1.0, abs(want)), (got, want, B1)


def test_no_quadratic_term_closed_form(orc):
    """U = 0 and every row of Q equal: A_j = A for every window sample and
    B_1 = 0, so L_tD = int p(D) exp(A D_ref / D) dD.  With s = 1/D and
    z = -A D_ref > 0 this is 3 / (d_max^3 - d_min^3) times the integral of
    s^-4 e^{-z s} over [1/d_max, 1/d_min], i.e. s^-3 E_4(z s) at 1/d_max
    minus the same at 1/d_min."""
    def constant_rows(q):
        r = np.zeros_like(q)
        r[:] = q[:, q.shape[1] // 2: q.shape[1] // 2 + 1, :]
        return r
    d, p = _point(orc, synth.workload("tiny").points[0], Q=constant_rows, U=lambda u: np.zeros_like(u))
    th = synth.prior_samples(12, 40)
    checked = 0
    for i in range(th.shape[1]):
        t = np.r_[th[:5, i], d["d_ref"], th[6, i]]
        A = orc.ell(p, t)
        assert np.ptp(A) <= 1e-12 * max(1.0, np.abs(A).max())
        A = A[0]
        if A >= -1e-3:
            continue
        z = -A * d["d_ref"]
        s1, s2 = 1.0 / D_MAX, 1.0 / D_MIN
        want = 3.0 / (D_MAX ** 3 - D_MIN ** 3) * (s1 ** -3 * special.expn(4, z * s1) - s2 ** -3 * special.expn(4, z * s2))
        got = orc.lnL_tD(p, th[:, i])
        assert abs(got - math.log(want)) < 1e-11 * max(1.0, abs(math.log(want))), (got, math.log(want), A)
        checked += 1
    assert checked >= 10


@pytest.mark.parametrize("which", ["tiny", "single"])
def test_matches_adaptive_quadrature_of_ell(orc, which):
    """scipy's adaptive Gauss-Kronrod over D of p(D) mean_j exp(ell_j(D)),
    with ell_j(D) from the oracle's own window values at each D (no use of
    the linear-quadratic form), against the composite rule."""
    d, p = _point(orc, synth.workload(which).points[0])
    th = synth.mixed_samples(d, 5, 6)
    for i in range(th.shape[1]):
        t = th[:, i].copy()
        got = orc.lnL_tD(p, t)
        # the integrand's peak: largest mean_j exp(ell_j(D)) p(D) on a coarse grid
        Ds = np.geomspace(D_MIN, D_MAX, 400)
        vals = []
        for D in Ds:
            t[5] = D
            e = orc.ell(p, t)
            m = e.max()
            vals.append(m + math.log(np.exp(e - m).mean()) + math.log(_prior(D)))
        vals = np.array(vals)
        shift = vals.max()
        Dp = Ds[int(vals.argmax())]

        def f(D):
            t[5] = D
            e = orc.ell(p, t)
            return np.exp(e - shift).mean() * _prior(D)

        pts = sorted({Dp, Dp * 0.97, Dp * 1.03})
        val, err = integrate.quad(f, D_MIN, D_MAX, points=pts, limit=500, epsabs=0.0, epsrel=1e-11)
        want = shift + math.log(val)
        assert abs(got - want) < 1e-8 * max(1.0, abs(want)), (got, want, err / val)


def test_monte_carlo_over_prior_distances(orc):
    """The marginal over D equals the average of L_t over distances drawn from
    the prior (Eq. (lnL:MonteCarlo) in one dimension): within 4 sigma."""
    d, p = _point(orc, synth.PIN_SPECS[2])
    t = d["theta_inj"].copy()
    n = 40000
    u = np.random.default_rng(9).random(n)
    D = np.cbrt(D_MIN ** 3 + u * (D_MAX ** 3 - D_MIN ** 3))
    th = np.tile(t[:, None], (1, n))
    th[5] = D
    r = orc.reduce(orc.lnL_t(p, th))
    assert r["n_eff"] > 200
    got = orc.lnL_tD(p, t)
    assert abs(got - r["lnL_marg"]) < 4 * r["sigma_lnL"], (got, r)


def test_narrow_prior_limit(orc):
    """d_min -> d_max: L_tD -> L_t at that distance."""
    d, p = _point(orc, synth.workload("tiny").points[0])
    th = synth.mixed_samples(d, 7, 4)
    for i in range(th.shape[1]):
        t = th[:, i].copy()
        t[5] = 321.0
        want = orc.lnL_t(p, t)
        got = orc.lnL_tD(p, t, d_min=321.0 * (1 - 1e-9), d_max=321.0 * (1 + 1e-9), panels=4)
        assert abs(got - want) < 1e-7 * max(1.0, abs(want))


def test_panel_convergence_on_loud_points(orc):
    """The composite rule has converged at its automatic panel count on the
    loudest adaptive points (SNR near 60): prior samples (mass against d_max
    behind a steep exp(-x^2 B_1)) and samples near the injection."""
    w = synth.workload("adaptive")
    loud = sorted(range(len(w.points)), key=lambda i: -w.points[i].snr)[:2]
    for i in loud:
        d, p = _point(orc, w.points[i])
        th = synth.mixed_samples(d, 8, 6)
        a = orc.lnL_tD(p, th)
        b = orc.lnL_tD(p, th, panels=400000)
        assert np.abs(a - b).max() < 1e-10 * max(1.0, np.abs(a).max()), np.abs(a - b)
