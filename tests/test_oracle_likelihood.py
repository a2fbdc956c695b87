"""Oracle pins for the decomposed likelihood and its time marginalization.

* noise-free injection, quadratic overlap kernel (reproduced exactly by the
  Catmull-Rom interpolant): ell at the injected time and parameters equals
  rho^2/2 (App. D: rho^2/2 is the noise-free maximum of ln L_full);
* Cauchy-Schwarz: without noise, ell <= rho^2/2 everywhere;
* psi -> psi + pi leaves ln L_t unchanged; for the (2,+-2) modes so does
  (psi, phi) -> (psi + pi/2, phi + pi/2);
* distance enters as ell_j(D) = x A_j - x^2 B with x = D_ref / D;
* noise statistics at the truth: E[ell] = rho^2/2, Var[ell] =
  sum_k a_k^dag U_k a_k / 2 * sum_q w_q(mu_k)^2 (i.i.d. rows);
* time marginalization: n_t = 1 reduces to ell_0; small amplitudes agree with
  the naive log-mean-exp;
* the analytic gradient agrees with central finite differences.
"""
import math

import numpy as np
import pytest

import synth


def _pt(orc, spec, **kw):
    d = synth.make_point(spec, **kw)
    return d, orc.Point.from_dict(d)


def test_peak_is_rho2_over_2(orc):
    for spec in synth.PIN_SPECS[:2]:
        d, p = _pt(orc, spec)
        ell = orc.ell(p, d["theta_inj"])
        assert ell[d["j_inj"]] == pytest.approx(spec.snr ** 2 / 2, rel=1e-10)
        assert ell.max() == pytest.approx(spec.snr ** 2 / 2, rel=1e-10)


def test_cauchy_schwarz_bound(orc):
    for spec in synth.PIN_SPECS[:3]:
        d, p = _pt(orc, spec)
        th, _, _, _ = orc.draw(7, 0, 0, 300)
        th[5] = np.exp(np.random.default_rng(0).uniform(np.log(50), np.log(800), 300))
        bound = spec.snr ** 2 / 2
        for i in range(th.shape[1]):
            assert orc.ell(p, th[:, i]).max() <= bound * (1 + 1e-6)


def test_invariances(orc):
    spec = synth.workload("tiny").points[0]
    d, p = _pt(orc, spec)
    th, _, _, _ = orc.draw(11, 0, 0, 50)
    for i in range(50):
        t = th[:, i].copy()
        a = orc.lnL_t(p, t)
        t2 = t.copy(); t2[2] += math.pi
        assert orc.lnL_t(p, t2) == pytest.approx(a, abs=1e-9 * max(1, abs(a)))
    spec22 = synth.workload("plain").points[0]
    d, p = _pt(orc, spec22)
    for i in range(50):
        t = th[:, i].copy()
        a = orc.lnL_t(p, t)
        t2 = t.copy(); t2[2] += math.pi / 2; t2[4] += math.pi / 2
        assert orc.lnL_t(p, t2) == pytest.approx(a, abs=1e-9 * max(1, abs(a)))


def test_distance_dependence(orc):
    spec = synth.workload("tiny").points[0]
    d, p = _pt(orc, spec)
    t = d["theta_inj"].copy()
    xs = []
    ells = []
    for D in (80.0, 200.0, 550.0):
        t[5] = D
        xs.append(spec.d_ref / D)
        ells.append(orc.ell(p, t))
    # solve for A_j, B from the first two distances, predict the third
    x1, x2, x3 = xs
    Mx = np.array([[x1, -x1 * x1], [x2, -x2 * x2]])
    AB = np.linalg.solve(Mx, np.vstack([ells[0], ells[1]]))
    pred = x3 * AB[0] - x3 * x3 * AB[1]
    assert np.allclose(pred, ells[2], rtol=0, atol=1e-10 * np.abs(ells[2]).max())
    assert np.ptp(AB[1]) < 1e-9 * abs(AB[1].mean())  # B does not depend on time


def test_noise_statistics(orc):
    spec = synth.PIN_SPECS[4]
    d = synth.make_point(spec)
    th = d["theta_inj"].copy()
    th[6] = 0.37 / spec.f_s  # fractional row offset: variance shrinks by sum w^2
    p0 = orc.Point.from_dict(d)
    a, B = orc.coeffs(p0, th)
    K, L, M = d["Q"].shape
    # expected mean/variance
    var = 0.0
    for k in range(K):
        s = (th[6] + orc.delay(d["det_pos"][k], th[0], th[1], d["gmst"])) * spec.f_s
        w, _ = orc.catmull_rom(s - math.floor(s))
        var += 0.5 * np.real(a[k].conj() @ d["U"][k] @ a[k]) * (w ** 2).sum()
    j = d["j_inj"]
    ell0 = orc.ell(p0, th)[j]
    rng = np.random.default_rng(9)
    vals = []
    chol = [np.linalg.cholesky(d["U"][k]) for k in range(K)]
    for _ in range(400):
        Q = d["Q"].copy()
        for k in range(K):
            xi = (rng.standard_normal((L, M)) + 1j * rng.standard_normal((L, M))) / math.sqrt(2)
            Q[k] += xi @ chol[k].T
        dd = dict(d); dd["Q"] = Q
        vals.append(orc.ell(orc.Point.from_dict(dd), th)[j])
    vals = np.array(vals)
    n = len(vals)
    assert abs(vals.mean() - ell0) < 4 * math.sqrt(var / n)
    # variance within 4 sigma of its sampling error (Gaussian: sd(var_hat) = var sqrt(2/(n-1)))
    assert abs(vals.var(ddof=1) - var) < 4 * var * math.sqrt(2 / (n - 1))


def test_time_marginalization_reductions(orc):
    spec = synth.PointSpec(seed=synth.BASE_SEED + 31, dets=("H1", "L1"), n_modes=2, n_t=1, snr=8.0)
    d = synth.make_point(spec, injection=dict(a=np.ones((2, 2), complex), dt=np.zeros(2), rho2=1.0))
    p = orc.Point.from_dict(d)
    th, _, _, _ = orc.draw(3, 0, 0, 20)
    for i in range(20):
        assert orc.lnL_t(p, th[:, i]) == pytest.approx(orc.ell(p, th[:, i])[0], abs=1e-12)
    # small amplitude: the max-shifted LSE equals the naive mean of exp
    spec = synth.PointSpec(seed=synth.BASE_SEED + 32, dets=("H1", "L1", "V1"), n_modes=5, n_t=50, snr=1.0)
    d = synth.make_point(spec, injection=dict(a=0.01 * np.ones((3, 5), complex), dt=np.zeros(3), rho2=1.0))
    p = orc.Point.from_dict(d)
    for i in range(20):
        e = orc.ell(p, th[:, i])
        assert np.abs(e).max() < 30
        assert orc.lnL_t(p, th[:, i]) == pytest.approx(math.log(np.mean(np.exp(e))), abs=1e-12)


def test_gradient_matches_finite_differences(orc):
    spec = synth.workload("tiny").points[0]
    d, p = _pt(orc, spec)
    th, _, _, _ = orc.draw(5, 0, 0, 6, tau_width=1.0 / spec.f_s)
    # include samples near the injection where the likelihood varies fastest
    near = d["theta_inj"][:, None] + np.array([0.01, -0.01, 0.02, 0.03, -0.02, 5.0, 0.1 / spec.f_s])[:, None] * np.array([[1, -1]])
    th = np.hstack([th, near])
    lt, g = orc.grad(p, th)
    steps = np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-4, 1e-9])
    for i in range(th.shape[1]):
        for k in range(7):
            tp = th[:, i].copy(); tm = tp.copy()
            tp[k] += steps[k]; tm[k] -= steps[k]
            fd = (orc.lnL_t(p, tp) - orc.lnL_t(p, tm)) / (2 * steps[k])
            scale = max(abs(fd), 1e-3 * np.abs(g[:, i] * np.array([1, 1, 1, 1, 1, 100, 1e-4])).max(), 1e-6)
            assert abs(g[k, i] - fd) <= 2e-5 * scale + 1e-7, (i, k, g[k, i], fd)
        assert lt[i] == pytest.approx(orc.lnL_t(p, th[:, i]), abs=1e-12)
