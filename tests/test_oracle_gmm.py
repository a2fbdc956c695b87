"""Oracle pins for the Gaussian-mixture proposal (Sec. III.B, App. A): the
truncated-normal sampler against scipy's truncnorm, normalization of the
proposal (E[p / p_s] = 1 and a Kolmogorov-Smirnov test of the draws), EM
against closed forms (one component: the weighted moments; integer weights:
replicated samples), EM recovering a known mixture and never lowering the
weighted log-likelihood, and the online update against pooled moments."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import gmm


def test_truncated_normal_ppf_matches_scipy():
    v = np.linspace(0.0, 1.0, 257)[:-1] + 0.5 / 256
    for mu, sd in [(0.5, 0.1), (0.02, 0.05), (0.97, 0.3), (0.3, 2.0), (0.999, 1e-3)]:
        ref = stats.truncnorm.ppf(v, -mu / sd, (1 - mu) / sd, loc=mu, scale=sd)
        assert np.max(np.abs(gmm.tn_ppf(v, mu, sd) - ref)) < 1e-12


def test_proposal_density_integrates_to_one():
    w, mu, sd = np.array([0.5, 0.3, 0.2]), np.array([0.1, 0.5, 0.95]), np.array([0.05, 0.2, 0.01])
    for eps in (0.0, 0.1):
        tot = integrate.quad(lambda x: float(gmm.density(np.array([x]), w, mu, sd, eps)[0]), 0, 1,
                             points=[0.1, 0.5, 0.95], limit=200, epsabs=1e-13)[0]
        assert abs(tot - 1.0) < 1e-10


def _model():
    g = gmm.Gmm(3, 0b0010101, 0.1)
    g.w[0], g.mu[0], g.sd[0] = [0.6, 0.3, 0.1], [0.2, 0.7, 0.9], [0.05, 0.1, 0.02]
    g.w[2], g.mu[2], g.sd[2] = [0.2, 0.5, 0.3], [0.05, 0.5, 0.99], [0.03, 0.3, 0.05]
    g.w[4], g.mu[4], g.sd[4] = [1.0, 0.0, 0.0], [0.4, 0.5, 0.6], [0.2, 0.1, 0.1]
    g.n_trained = 1000.0
    return g


def test_mixture_draws_are_normalized_and_follow_the_mixture():
    g = _model()
    n = 6000
    th, lr, u = gmm.draw(2210079124, 2, 3, n, g)
    # E_{p_s}[p / p_s] = 1 (the prior is uniform in u)
    r = np.exp(lr)
    assert abs(r.mean() - 1.0) < 5 * r.std() / math.sqrt(n)
    for d in (0, 2, 4):
        def cdf(x, d=d):
            c = g.eps * x
            for k in range(3):
                if g.w[d, k] > 0:
                    mu, sd = g.mu[d, k], g.sd[d, k]
                    c = c + (1 - g.eps) * g.w[d, k] * stats.truncnorm.cdf(x, -mu / sd, (1 - mu) / sd, loc=mu, scale=sd)
            return c
        assert stats.kstest(u[d], cdf).pvalue > 1e-3
    # parameters outside the mask stay on the prior
    for d in (1, 3, 5, 6):
        assert stats.kstest(u[d], "uniform").pvalue > 1e-3
    # theta through the prior inverse CDFs
    assert np.allclose(th[0], 2 * np.pi * u[0]) and np.allclose(th[3], np.arccos(2 * u[3] - 1))


def test_em_one_component_gives_weighted_moments():
    rng = np.random.default_rng(5)
    u = rng.beta(2, 5, 4000)
    wt = rng.exponential(size=4000)
    w, mu, sd = gmm.em_fit(u, wt, [1.0], [0.5], [0.5], 1)
    m = np.sum(wt * u) / wt.sum()
    s = math.sqrt(np.sum(wt * (u - m) ** 2) / wt.sum())
    assert w[0] == 1.0 and abs(mu[0] - m) < 1e-14 and abs(sd[0] - s) < 1e-14


def test_em_integer_weights_equal_replicated_samples():
    rng = np.random.default_rng(6)
    u = rng.uniform(size=500)
    k = rng.integers(1, 4, size=500)
    a = gmm.em_fit(u, k.astype(float), [0.3, 0.3, 0.4], [0.2, 0.5, 0.8], [0.1, 0.1, 0.1], 5)
    b = gmm.em_fit(np.repeat(u, k), np.ones(int(k.sum())), [0.3, 0.3, 0.4], [0.2, 0.5, 0.8], [0.1, 0.1, 0.1], 5)
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) < 1e-12


def test_em_recovers_a_known_mixture_and_never_lowers_the_likelihood():
    rng = np.random.default_rng(7)
    n = 20000
    comp = rng.uniform(size=n) < 0.35
    u = np.where(comp, rng.normal(0.25, 0.04, n), rng.normal(0.7, 0.08, n))
    u = u[(u > 0) & (u < 1)]
    wt = np.ones(u.size)
    par = ([0.5, 0.5], [0.4, 0.6], [0.2, 0.2])
    ll = []
    for _ in range(60):
        w, mu, sd = par
        dens = sum(w[k] * stats.norm.pdf(u, mu[k], sd[k]) for k in range(2))
        ll.append(np.sum(wt * np.log(dens)))
        par = gmm.em_fit(u, wt, *par, 1)
    assert np.all(np.diff(ll) > -1e-9 * abs(ll[0]))
    w, mu, sd = par
    o = np.argsort(mu)
    assert np.allclose(w[o], [0.35, 0.65], atol=0.02)
    assert np.allclose(mu[o], [0.25, 0.7], atol=0.005)
    assert np.allclose(sd[o], [0.04, 0.08], rtol=0.05)


def test_online_update_pools_moments():
    rng = np.random.default_rng(8)
    x, y = rng.normal(0.3, 0.05, 3000), rng.normal(0.35, 0.08, 1000)
    old = gmm.Gmm(1, 1, 0.1, w=[[1.0]] * 7, mu=[[x.mean()]] * 7, sd=[[x.std()]] * 7, n_trained=x.size)
    w, mu, sd = gmm.merge(old, [1.0], [y.mean()], [y.std()], 0, y.size)
    z = np.concatenate([x, y])
    assert abs(mu[0] - z.mean()) < 1e-14 and abs(sd[0] - z.std()) < 1e-14 and w[0] == 1.0
    # merging a model with itself keeps it; shuffled components are matched back
    g = _model()
    p = [2, 0, 1]
    w, mu, sd = gmm.merge(g, g.w[0][p], g.mu[0][p], g.sd[0][p], 0, 500)
    assert np.allclose(w, g.w[0]) and np.allclose(mu, g.mu[0]) and np.allclose(sd, g.sd[0])


def test_weights_and_counts():
    wt, M = gmm.weights([0.0, -1.0, np.nan, -np.inf, np.inf, 2.0])
    assert M == 4
    assert np.allclose(wt, [math.exp(-2), math.exp(-3), 0, 0, 0, 1])


def test_adapt_round_from_the_prior():
    # first update: EM from the initial model, no merge (nothing trained yet)
    g0 = None
    th, lr, u = gmm.draw(11, 0, 0, 3000, g0)
    lnw = -0.5 * ((u[0] - 0.3) / 0.05) ** 2
    g1 = gmm.adapt(g0, u, lnw, K=2, mask=1, eps=0.05, n_iter=30)
    assert g1.n_trained == 3000 and g1.mask == 1
    top = np.argmax(g1.w[0])
    assert abs(g1.mu[0, top] - 0.3) < 0.01 and abs(g1.sd[0, top] - 0.05) < 0.01
    # the next round's draws concentrate there and stay unbiased
    th, lr, u2 = gmm.draw(11, 0, 1, 3000, g1)
    assert np.mean(np.abs(u2[0] - 0.3) < 0.15) > 0.8
    assert abs(np.exp(lr).mean() - 1) < 5 * np.exp(lr).std() / math.sqrt(3000)


def test_frame_sky_matches_the_c_oracle(orc):
    """The numpy network-frame map equals the C oracle's on its own draws
    (prior draws: the sky uniforms are the raw Philox words)."""
    import synth
    d = synth.make_point(synth.workload("tiny").points[0])
    th, _, _, raw = orc.draw(5, 0, 0, 200, frame=(d["det_pos"], d["gmst"]))
    v = ((raw.astype(np.float64) // 256) + 0.5) / 16777216.0
    a, dl = gmm.frame_sky(d["det_pos"], d["gmst"], v[0], v[1])
    assert np.abs(a - th[0]).max() < 1e-12 and np.abs(dl - th[1]).max() < 1e-12


def test_phase_rotation_matches_the_c_oracle(orc):
    """The numpy phase-rotated map equals the C oracle's on its own draws."""
    th, _, _, _ = orc.draw(5, 0, 0, 300, phase=True)
    th2, _, u = gmm.draw(5, 0, 0, 300, None, phase=True)
    assert np.array_equal(th[[2, 4]], th2[[2, 4]])
    assert np.abs(th - th2).max() < 1e-12


# --- correlated pairs ---------------------------------------------------------

def _pair_model():
    g = gmm.Gmm(2, 0b0011100, 0.1, pairs=[(2, 4)])
    g.pw[0] = np.array([0.7, 0.3])
    g.pmu[0] = np.array([[0.3, 0.6], [0.8, 0.1]])
    g.pcov[0] = np.array([[0.01, 0.008, 0.01], [0.04, -0.01, 0.01]])
    g.n_trained = 2000.0
    return g


def test_box_mass_against_quadrature():
    from scipy.stats import multivariate_normal
    for mu, cov in [([0.3, 0.6], [0.01, 0.008, 0.01]), ([0.95, 0.02], [0.09, -0.05, 0.04]), ([0.5, 0.5], [4.0, 0.0, 1e-4])]:
        C = np.array([[cov[0], cov[1]], [cov[1], cov[2]]])
        ref = integrate.dblquad(lambda y, x: multivariate_normal.pdf([x, y], mu, C), 0, 1, 0, 1,
                                epsabs=1e-12, epsrel=1e-12)[0]
        assert abs(gmm.box_mass(mu, cov) - ref) < 1e-9


def test_pair_em_one_component_gives_weighted_moments():
    rng = np.random.default_rng(9)
    x, y = rng.beta(2, 5, 3000), rng.beta(3, 3, 3000)
    y = 0.5 * y + 0.5 * x
    wt = rng.exponential(size=3000)
    w, mu, cov = gmm.em_fit_pair(x, y, wt, [1.0], [[0.5, 0.5]], [[0.1, 0.0, 0.1]], 1)
    W = wt.sum()
    mx, my = np.sum(wt * x) / W, np.sum(wt * y) / W
    ref = [np.sum(wt * (x - mx) ** 2) / W, np.sum(wt * (x - mx) * (y - my)) / W, np.sum(wt * (y - my) ** 2) / W]
    assert np.allclose(mu[0], [mx, my], atol=1e-14) and np.allclose(cov[0], ref, atol=1e-14)


def test_pair_online_update_pools_moments():
    rng = np.random.default_rng(10)
    A = rng.multivariate_normal([0.3, 0.4], [[0.01, 0.004], [0.004, 0.02]], 3000)
    B = rng.multivariate_normal([0.35, 0.45], [[0.02, -0.003], [-0.003, 0.01]], 1000)
    mom = lambda Z: (Z.mean(axis=0), np.array([np.var(Z[:, 0]), np.cov(Z.T, bias=True)[0, 1], np.var(Z[:, 1])]))
    ma, ca = mom(A)
    mb, cb = mom(B)
    old = gmm.Gmm(1, 0b11, 0.1, n_trained=A.shape[0], pairs=[(0, 1)])
    old.pw[0], old.pmu[0], old.pcov[0] = np.array([1.0]), ma[None], ca[None]
    w, mu, cov = gmm.merge_pair(old, 0, np.array([1.0]), mb[None], cb[None], B.shape[0])
    mz, cz = mom(np.concatenate([A, B]))
    assert np.allclose(mu[0], mz, atol=1e-14) and np.allclose(cov[0], cz, atol=1e-14) and w[0] == 1.0


def test_pair_draws_follow_the_truncated_mixture():
    from scipy.stats import multivariate_normal, chisquare
    g = _pair_model()
    n = 8000
    th, lr, u = gmm.draw(2210079128, 1, 2, n, g)
    assert np.all(np.isfinite(lr))
    r = np.exp(lr)
    assert abs(r.mean() - 1.0) < 5 * r.std() / math.sqrt(n)
    # cell probabilities of the pair proposal on a 5 x 5 grid, by the bivariate CDF
    e = np.linspace(0, 1, 6)
    zm = sum(g.pw[0][k] * gmm.box_mass(g.pmu[0][k], g.pcov[0][k]) for k in range(2))
    P = np.zeros((5, 5))
    for k in range(2):
        C = np.array([[g.pcov[0][k][0], g.pcov[0][k][1]], [g.pcov[0][k][1], g.pcov[0][k][2]]])
        F = lambda x, y: multivariate_normal.cdf([x, y], mean=g.pmu[0][k], cov=C, abseps=1e-12, releps=1e-12)
        for i in range(5):
            for j in range(5):
                P[i, j] += g.pw[0][k] * (F(e[i + 1], e[j + 1]) - F(e[i], e[j + 1]) - F(e[i + 1], e[j]) + F(e[i], e[j]))
    P = g.eps / 25 + (1 - g.eps) * P / zm
    obs = np.histogram2d(u[2], u[4], bins=[e, e])[0]
    assert abs(P.sum() - 1) < 1e-9
    assert chisquare(obs.ravel(), n * P.ravel()).pvalue > 1e-3
    # the 1-D parameter of the mask (3) keeps its own (initial) mixture; others the prior
    assert stats.kstest(u[0], "uniform").pvalue > 1e-3


def test_pair_draws_with_a_low_box_mass_average_to_one():
    """A pair whose mixture lies mostly outside the unit square: one
    component at the corner (0, 0), sd 0.05 per axis, correlation -0.99.
    Its box mass is the positive-quadrant probability 1/4 + asin(rho)/(2 pi)
    (about 0.0225), so the 64-try rejection gives up on a fraction
    (1 - eps)(1 - Z)^64 (about 0.21) of the draws, which carry zero weight,
    and the kept ones follow q = eps + (1 - eps)(1 - (1 - Z)^64) T.  Checked:
    q integrates to the kept fraction, the given-up fraction, the cells of the
    kept draws against q, their weights, and E[p/q] = 1 over all draws."""
    from scipy.stats import chisquare, multivariate_normal
    rho, sd = -0.99, 0.05
    g = gmm.Gmm(1, 0b0010100, 0.1, pairs=[(2, 4)])
    g.pw[0] = np.array([1.0])
    g.pmu[0] = np.array([[0.0, 0.0]])
    g.pcov[0] = np.array([[sd * sd, rho * sd * sd, sd * sd]])
    Z = gmm.box_mass(g.pmu[0][0], g.pcov[0][0])
    assert abs(Z - (0.25 + math.asin(rho) / (2.0 * math.pi))) < 1e-10
    keep = 1.0 - (1.0 - Z) ** 64
    # q over the square, eps = 0: (1 - eps) keep, T integrating to 1; by a
    # product Gauss-Legendre rule on [0, 0.4]^2 (beyond 0.4 the component's
    # mass is below 1e-15), split at 0.1 where the ridge x = -y/rho lies
    x, wq = np.polynomial.legendre.leggauss(400)
    xs = np.concatenate([0.05 * (x + 1.0), 0.1 + 0.15 * (x + 1.0)])
    ws = np.concatenate([0.05 * wq, 0.15 * wq])
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    qv = gmm.pair_draw_density(X.ravel(), Y.ravel(), g.pw[0], g.pmu[0], g.pcov[0], 0.0).reshape(X.shape)
    assert abs(np.einsum("i,j,ij->", ws, ws, qv) - keep) < 1e-8
    n = 4000
    th, lr, u = gmm.draw(2210079131, 0, 1, n, g)
    assert not np.isnan(lr).any()
    gave_up = np.isneginf(lr)
    frac = (1.0 - g.eps) * (1.0 - keep)
    assert abs(gave_up.mean() - frac) < 5.0 * math.sqrt(frac * (1 - frac) / n), (gave_up.mean(), frac)
    # kept draws in 4 x 4 cells of [0, 1)^2 against q / P(kept)
    e = np.array([0.0, 0.03, 0.06, 0.12, 1.0])
    C = np.array([[sd * sd, rho * sd * sd], [rho * sd * sd, sd * sd]])
    F = lambda a, b: multivariate_normal.cdf([a, b], mean=[0.0, 0.0], cov=C, abseps=1e-12, releps=1e-12)
    P = np.zeros((4, 4))
    for i in range(4):
        for j in range(4):
            cell = F(e[i + 1], e[j + 1]) - F(e[i], e[j + 1]) - F(e[i + 1], e[j]) + F(e[i], e[j])
            P[i, j] = g.eps * (e[i + 1] - e[i]) * (e[j + 1] - e[j]) + (1 - g.eps) * keep * cell / Z
    P /= P.sum()
    kept = ~gave_up
    obs = np.histogram2d(u[2][kept], u[4][kept], bins=[e, e])[0]
    ok = kept.sum() * P.ravel() > 5
    assert chisquare(obs.ravel()[ok], kept.sum() * P.ravel()[ok] * obs.ravel()[ok].sum()
                     / (kept.sum() * P.ravel()[ok]).sum()).pvalue > 1e-3
    # the kept draws carry the weight of that density (the pair is the only
    # adapted part of the mask here: parameters 2 and 4)
    q = gmm.pair_draw_density(u[2][kept], u[4][kept], g.pw[0], g.pmu[0], g.pcov[0], g.eps)
    assert np.allclose(lr[kept], -np.log(q), rtol=0, atol=1e-12)
    r = np.exp(lr)
    assert abs(r.mean() - 1.0) < 5 * r.std() / math.sqrt(n)
