"""FP64 reference for the Gaussian-mixture proposal (Sec. III.B, adaptive
sampling with Gaussian mixture models; App. A, EM for GMMs, online update,
finite domains).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product package never does.

The mixture lives in each adapted parameter's prior-CDF coordinate u in
[0, 1) (the prior is uniform there, so ln p - ln p_s = -ln p_s(u)), one
independent mixture per adapted parameter (the separable default form).
Readings where the text is silent or garbled:
  * weights: the printed responsibility carries w_n in both numerator and
    normalizer, where it cancels; the weights are taken to enter the M-step
    sums (weighted EM): mu_k = sum w r x / sum w r, and so on;
  * finite domain: every component is a normal truncated to [0, 1]
    (normalized by Phi(b) - Phi(a)), while EM fits untruncated normals to
    the samples, as the appendix describes;
  * a uniform floor eps is mixed in, p_s = eps + (1 - eps) sum_k pi_k N_t,
    as for the histogram proposal (defensive importance sampling);
  * each round's new model starts from the current one (warm start) and
    runs a fixed number of EM iterations; the online update then matches
    components by the smallest summed symmetric Mahalanobis distance over
    all permutations and combines them with the sample counts N (all
    earlier rounds) and M (this round);
  * the mixture weight of the combined component is (N pi_j + M pi_i) /
    (N + M) (the text's pi_k there is read as pi_i).
Random numbers: the uniform v of a parameter is the same Philox word as for
the histogram proposal; the component choice uses a second Philox block with
counter word 2 = 2^31 | (2 round + half).

Correlated pairs (the paper's correlated sampling in subsets of dimensions):
up to three disjoint pairs (a, b) of adapted parameters get bivariate
components in (u_a, u_b).  As the appendix describes, draws come from the
untruncated mixture and are rejected outside the unit square; an accepted
draw follows T(u) = sum_k pi_k N_k(u) / Z with Z = sum_k pi_k Z_k, Z_k the
component's mass in the square.  Tries use Philox counter word 2 =
3 * 2^30 | round << 10 | pair << 8 | try.  The rejection gives up after 64
tries, which happens with probability f = (1 - Z)^64, so among all draws the
pair's coordinates have the sub-density q(u) = eps + (1 - eps)(1 - f) T(u)
and the draws given up on carry zero weight (ln p - ln p_s = -inf; they stay
in the sample count, so that E[p/q] over all draws is 1).  EM fits bivariate normals (sd >=
1e-4 per axis, |correlation| <= 0.99); the online update uses the text's
symmetric Mahalanobis distances with each component's own covariance.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import ndtr, ndtri

from . import oracle

KMAX = 4
SD_MIN = 1e-4
ALPHA, DELTA, PSI, IOTA, PHI, DIST, TAU = range(7)


PAIR_TRIES = 64
RHO_MAX = 0.99


class Gmm:
    """Mixture state of one point: per parameter d, K components; per pair
    i (pairs[i] = (a, b)), K bivariate components pw [K], pmu [K, 2],
    pcov [K, 3] (xx, xy, yy)."""

    def __init__(self, K, mask, eps, w=None, mu=None, sd=None, n_trained=0.0, pairs=()):
        self.K, self.mask, self.eps, self.n_trained = int(K), int(mask), float(eps), float(n_trained)
        k = np.arange(K)
        self.w = np.tile(np.full(K, 1.0 / K), (7, 1)) if w is None else np.array(w, dtype=np.float64)
        self.mu = np.tile((k + 0.5) / K, (7, 1)) if mu is None else np.array(mu, dtype=np.float64)
        self.sd = np.tile(np.full(K, 0.5 / K), (7, 1)) if sd is None else np.array(sd, dtype=np.float64)
        self.pairs = [tuple(p) for p in pairs]
        self.pw = [np.full(K, 1.0 / K) for _ in self.pairs]
        self.pmu = [np.stack([(k + 0.5) / K, (k + 0.5) / K], axis=1) for _ in self.pairs]
        self.pcov = [np.tile([0.25 / K ** 2, 0.0, 0.25 / K ** 2], (K, 1)) for _ in self.pairs]

    def copy(self):
        g = Gmm(self.K, self.mask, self.eps, self.w, self.mu, self.sd, self.n_trained)
        g.pairs = list(self.pairs)
        g.pw = [x.copy() for x in self.pw]
        g.pmu = [x.copy() for x in self.pmu]
        g.pcov = [x.copy() for x in self.pcov]
        return g

    def paired(self):
        return {d for p in self.pairs for d in p}


def decode_pairs(code):
    """Pairs from the byte code: byte i = a | b << 4 with a < b (0: none)."""
    out = []
    for i in range(3):
        c = (code >> (8 * i)) & 0xFF
        if c:
            out.append((c & 15, c >> 4))
    return out


# --- bivariate components ------------------------------------------------------

def box_mass(mu, cov):
    """Mass of N(mu, cov) in [0, 1]^2 (scipy's bivariate normal CDF on the
    standardized rectangle, by inclusion-exclusion)."""
    from scipy.stats import multivariate_normal
    sx, sy = math.sqrt(cov[0]), math.sqrt(cov[2])
    rho = cov[1] / (sx * sy)
    R = np.array([[1.0, rho], [rho, 1.0]])
    F = lambda x, y: multivariate_normal.cdf([(x - mu[0]) / sx, (y - mu[1]) / sy], mean=[0.0, 0.0], cov=R,
                                             abseps=1e-15, releps=1e-15)
    return F(1, 1) - F(0, 1) - F(1, 0) + F(0, 0)


def pair_logpdf(x, y, mu, cov):
    """ln N((x, y); mu, cov)."""
    det = cov[0] * cov[2] - cov[1] * cov[1]
    dx, dy = x - mu[0], y - mu[1]
    q = (cov[2] * dx * dx - 2.0 * cov[1] * dx * dy + cov[0] * dy * dy) / det
    return -math.log(2.0 * math.pi) - 0.5 * math.log(det) - 0.5 * q


def pair_density(x, y, w, mu, cov, eps):
    """Pair proposal density in (u_a, u_b) on the unit square (rejection
    without a limit on the tries): eps + (1 - eps) T(u)."""
    zm = sum(w[k] * box_mass(mu[k], cov[k]) for k in range(len(w)) if w[k] > 0.0)
    s = np.zeros_like(np.asarray(x, dtype=np.float64))
    for k in range(len(w)):
        if w[k] > 0.0:
            s = s + w[k] * np.exp(pair_logpdf(x, y, mu[k], cov[k]))
    return eps + (1.0 - eps) * s / zm


def pair_draw_density(x, y, w, mu, cov, eps, tries=None):
    """Sub-density of the sampler's pair draws over all draws: the mixture
    branch keeps a draw with probability 1 - (1 - Z)^tries (Z the per-try
    acceptance sum_k pi_k Z_k), so q(u) = eps + (1 - eps)(1 - (1 - Z)^tries) T(u)."""
    tries = PAIR_TRIES if tries is None else tries
    zm = sum(w[k] * box_mass(mu[k], cov[k]) for k in range(len(w)) if w[k] > 0.0)
    keep = 1.0 - (1.0 - zm) ** tries
    s = np.zeros_like(np.asarray(x, dtype=np.float64))
    for k in range(len(w)):
        if w[k] > 0.0:
            s = s + w[k] * np.exp(pair_logpdf(x, y, mu[k], cov[k]))
    return eps + (1.0 - eps) * keep * s / zm


def chol(cov):
    l11 = math.sqrt(cov[0])
    l21 = cov[1] / l11
    return l11, l21, math.sqrt(max(cov[2] - l21 * l21, 0.0))


# --- truncated normal on [0, 1] ----------------------------------------------

def tn_norm(mu, sd):
    """(Phi(a), Z) with a = -mu / sd, b = (1 - mu) / sd, Z = Phi(b) - Phi(a)."""
    ca = ndtr(-mu / sd)
    return ca, ndtr((1.0 - mu) / sd) - ca


def tn_ppf(v, mu, sd):
    """Inverse CDF of N(mu, sd^2) truncated to [0, 1] at v in [0, 1)."""
    ca, z = tn_norm(mu, sd)
    return mu + sd * ndtri(ca + v * z)


def density(u, w, mu, sd, eps):
    """p_s(u) = eps + (1 - eps) sum_k w_k phi((u - mu_k) / sd_k) / (sd_k Z_k)."""
    u = np.asarray(u, dtype=np.float64)
    s = np.zeros_like(u)
    for k in range(len(w)):
        if w[k] > 0.0:
            _, z = tn_norm(mu[k], sd[k])
            t = (u - mu[k]) / sd[k]
            s = s + w[k] * np.exp(-0.5 * t * t) / (sd[k] * z * math.sqrt(2.0 * math.pi))
    return eps + (1.0 - eps) * s


# --- sampler -----------------------------------------------------------------

def prior_inv(d, u, d_min, d_max, tau_width):
    """Prior inverse CDFs u -> theta (the sampler's conventions)."""
    if d in (ALPHA, PHI):
        return 2.0 * math.pi * u
    if d == DELTA:
        return np.arcsin(2.0 * u - 1.0)
    if d == PSI:
        return math.pi * u
    if d == IOTA:
        return np.arccos(2.0 * u - 1.0)
    if d == DIST:
        a3, b3 = d_min ** 3, d_max ** 3
        return np.cbrt(a3 + u * (b3 - a3))
    return (u - 0.5) * tau_width


def frame_sky(det_pos, gmst, u0, u1):
    """Sky of the network frame of detectors 0 and 1 (the C oracle's axes):
    azimuth 2 pi u0 and polar cosine 2 u1 - 1 -> (alpha, delta)."""
    ax = oracle.network_frame(det_pos)
    ph, ct = 2.0 * math.pi * u0, 2.0 * u1 - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    n = np.outer(ax[0], st * np.cos(ph)) + np.outer(ax[1], st * np.sin(ph)) + np.outer(ax[2], ct)
    delta = np.arcsin(np.clip(n[2], -1.0, 1.0))
    alpha = np.mod(np.arctan2(n[1], n[0]) + gmst, 2.0 * math.pi)
    return alpha, delta


def phase_rot(us, ud):
    """Phase-rotated coordinates (the C oracle's map): psi = 2 pi (u_s - u_d)
    mod pi, phi = 2 pi (u_s + u_d) mod 2 pi."""
    x, y = 2.0 * math.pi * (us - ud), 2.0 * math.pi * (us + ud)
    return x - math.pi * np.floor(x / math.pi), y - 2.0 * math.pi * np.floor(y / (2.0 * math.pi))


def draw(seed, point, rnd, n, g: Gmm | None, *, d_min=10.0, d_max=1000.0, tau_width=0.0, start=0, frame=None,
         phase=False):
    """Samples start..start+n-1 of (point, round) from the mixture proposal
    (prior where g is None or a parameter is outside g.mask): theta [7, n],
    ln p - ln p_s [n], u [7, n].  frame = (det_pos, gmst): the sky drawn in
    the network frame of detectors 0 and 1.  phase: polarization and phase
    from the phase-rotated coordinates u[PSI] = u_s, u[PHI] = u_d."""
    _, _, _, raw = oracle.draw(seed, point, rnd, n, d_min=d_min, d_max=d_max, tau_width=tau_width, start=start)
    v = ((raw.astype(np.float64) // 256) + 0.5) / 16777216.0
    u = v.copy()
    lr = np.zeros(n)
    if g is not None and g.mask:
        key = (seed & 0xFFFFFFFF, seed >> 32)
        ex = np.zeros((8, n))
        for j in range(n):
            i = start + j
            for half in range(2):
                c = oracle.philox([i & 0xFFFFFFFF, i >> 32, 0x80000000 | (2 * rnd + half), point], key)
                for q in range(4):
                    ex[4 * half + q, j] = ((c[q] >> 8) + 0.5) / 16777216.0
        for d in range(7):
            if not (g.mask >> d) & 1 or d in g.paired():
                continue
            for j in range(n):
                cu = ex[d, j]
                if cu < g.eps:
                    uu = v[d, j]
                else:
                    c2 = (cu - g.eps) / (1.0 - g.eps)
                    k, acc = 0, g.w[d, 0]
                    while k < g.K - 1 and c2 >= acc:
                        k += 1
                        acc += g.w[d, k]
                    uu = float(tn_ppf(v[d, j], g.mu[d, k], g.sd[d, k]))
                    uu = min(max(uu, 0.0), 1.0 - 2.0 ** -53)
                u[d, j] = uu
            lr -= np.log(density(u[d], g.w[d], g.mu[d], g.sd[d], g.eps))
        for pi, (a, b) in enumerate(g.pairs):
            L = [chol(c) for c in g.pcov[pi]]
            for j in range(n):
                i = start + j
                if ex[a, j] < g.eps:
                    continue  # uniform: u_a, u_b stay the raw uniforms
                c0 = (ex[a, j] - g.eps) / (1.0 - g.eps)
                ok = False
                for t in range(PAIR_TRIES):
                    w4 = oracle.philox([i & 0xFFFFFFFF, i >> 32, 0xC0000000 | (rnd << 10) | (pi << 8) | t, point], key)
                    c = c0 if t == 0 else (w4[0] + 0.5) * 2.0 ** -32
                    k, acc = 0, g.pw[pi][0]
                    while k < g.K - 1 and c >= acc:
                        k += 1
                        acc += g.pw[pi][k]
                    u1 = (((w4[1] >> 6) << 27 | (w4[2] >> 5)) + 0.5) * 2.0 ** -53
                    u2 = (w4[3] + 0.5) * 2.0 ** -32
                    r = math.sqrt(-2.0 * math.log(u1))
                    z1, z2 = r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)
                    l11, l21, l22 = L[k]
                    x = g.pmu[pi][k][0] + l11 * z1
                    y = g.pmu[pi][k][1] + l21 * z1 + l22 * z2
                    if 0.0 <= x < 1.0 and 0.0 <= y < 1.0:
                        ok = True
                        break
                if ok:
                    u[a, j], u[b, j] = x, y
                else:
                    lr[j] = -np.inf  # given up on: zero weight (u_a, u_b stay the raw uniforms)
            dens = pair_draw_density(u[a], u[b], g.pw[pi], g.pmu[pi], g.pcov[pi], g.eps)
            lr -= np.log(dens)
    th = np.stack([prior_inv(d, u[d], d_min, d_max, tau_width) for d in range(7)])
    if frame is not None:
        th[ALPHA], th[DELTA] = frame_sky(frame[0], frame[1], u[ALPHA], u[DELTA])
    if phase:
        th[PSI], th[PHI] = phase_rot(u[PSI], u[PHI])
    return th, lr, u


# --- EM and the online update ------------------------------------------------

def weights(lnw):
    """w_n = exp(ln w_n - max ln w) over the finite ln w (others 0) and the
    sample count M (ln w neither NaN nor +inf)."""
    lnw = np.asarray(lnw, dtype=np.float64)
    fin = np.isfinite(lnw)
    M = int(np.sum(~np.isnan(lnw) & (lnw != np.inf)))
    if not fin.any():
        return np.zeros_like(lnw), M
    return np.where(fin, np.exp(np.where(fin, lnw, 0.0) - lnw[fin].max()), 0.0), M


def em_fit(u, wt, w, mu, sd, n_iter):
    """n_iter weighted EM iterations (App. A E-step and M-step, weights in
    the sums) for one parameter, from (w, mu, sd); untruncated normals."""
    w, mu, sd = np.array(w, dtype=np.float64), np.array(mu, dtype=np.float64), np.array(sd, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    for _ in range(n_iter):
        lp = np.full((u.size, w.size), -np.inf)
        for k in range(w.size):
            if w[k] > 0.0:
                t = (u - mu[k]) / sd[k]
                lp[:, k] = math.log(w[k]) - math.log(sd[k]) - 0.5 * t * t
        m = lp.max(axis=1, keepdims=True)
        r = np.exp(lp - m)
        r /= r.sum(axis=1, keepdims=True)
        S0 = (wt[:, None] * r).sum(axis=0)
        tot = S0.sum()
        if not tot > 0.0:
            break
        for k in range(w.size):
            if S0[k] > 0.0:
                dk = u - mu[k]
                m1 = np.sum(wt * r[:, k] * dk) / S0[k]
                m2 = np.sum(wt * r[:, k] * dk * dk) / S0[k]
                mu[k] = mu[k] + m1
                sd[k] = max(math.sqrt(max(m2 - m1 * m1, 0.0)), SD_MIN)
            w[k] = S0[k] / tot
    return w, mu, sd


def match(old_mu, old_sd, new_mu, new_sd):
    """Permutation p (new component i <-> old component p[i]) minimizing the
    summed symmetric Mahalanobis distance; the first minimum in
    lexicographic order of permutations."""
    K = len(old_mu)
    best, bp = None, None
    for p in itertools.permutations(range(K)):
        s = 0.0
        for i in range(K):
            j = p[i]
            dd = abs(new_mu[i] - old_mu[j])
            s += dd / new_sd[i] + dd / old_sd[j]
        if best is None or s < best:
            best, bp = s, p
    return bp


def merge(old: Gmm, new_w, new_mu, new_sd, d, M):
    """Online update of parameter d: combine the model trained on N =
    old.n_trained samples with the new fit on M samples (App. A)."""
    N = old.n_trained
    K = old.K
    if N <= 0.0:
        return np.array(new_w), np.array(new_mu), np.array(new_sd)
    p = match(old.mu[d], old.sd[d], new_mu, new_sd)
    w = np.zeros(K)
    mu = np.zeros(K)
    sd = np.zeros(K)
    for i in range(K):
        j = p[i]
        a, b = N * old.w[d, j], M * new_w[i]
        if not a + b > 0.0:
            w[j], mu[j], sd[j] = 0.0, old.mu[d, j], old.sd[d, j]
            continue
        mu[j] = (a * old.mu[d, j] + b * new_mu[i]) / (a + b)
        dm = old.mu[d, j] - new_mu[i]
        var = (a * old.sd[d, j] ** 2 + b * new_sd[i] ** 2) / (a + b) + a * b * dm * dm / ((a + b) * (a + b))
        sd[j] = max(math.sqrt(var), SD_MIN)
        w[j] = (a + b) / (N + M)
    return w, mu, sd


def regularize(cov):
    """sd >= SD_MIN per axis, |correlation| <= RHO_MAX."""
    sxx, syy = max(cov[0], SD_MIN * SD_MIN), max(cov[2], SD_MIN * SD_MIN)
    cmax = RHO_MAX * math.sqrt(sxx * syy)
    return np.array([sxx, min(max(cov[1], -cmax), cmax), syy])


def em_fit_pair(x, y, wt, w, mu, cov, n_iter):
    """n_iter weighted EM iterations for one pair's bivariate components."""
    w, mu, cov = np.array(w, dtype=np.float64), np.array(mu, dtype=np.float64), np.array(cov, dtype=np.float64)
    K = w.size
    for _ in range(n_iter):
        lp = np.full((x.size, K), -np.inf)
        for k in range(K):
            if w[k] > 0.0:
                lp[:, k] = math.log(w[k]) + pair_logpdf(x, y, mu[k], cov[k]) + math.log(2.0 * math.pi)
        m = lp.max(axis=1, keepdims=True)
        r = np.exp(lp - m)
        r /= r.sum(axis=1, keepdims=True)
        S0 = (wt[:, None] * r).sum(axis=0)
        tot = S0.sum()
        if not tot > 0.0:
            break
        for k in range(K):
            if S0[k] > 0.0:
                q = wt * r[:, k]
                dx, dy = x - mu[k, 0], y - mu[k, 1]
                mx, my = np.sum(q * dx) / S0[k], np.sum(q * dy) / S0[k]
                cxx = np.sum(q * dx * dx) / S0[k] - mx * mx
                cxy = np.sum(q * dx * dy) / S0[k] - mx * my
                cyy = np.sum(q * dy * dy) / S0[k] - my * my
                mu[k] = mu[k] + [mx, my]
                cov[k] = regularize([cxx, cxy, cyy])
            w[k] = S0[k] / tot
    return w, mu, cov


def _inv(c):
    det = c[0] * c[2] - c[1] * c[1]
    return np.array([c[2], -c[1], c[0]]) / det


def _maha(d, c):
    i = _inv(c)
    return math.sqrt(max(i[0] * d[0] * d[0] + 2.0 * i[1] * d[0] * d[1] + i[2] * d[1] * d[1], 0.0))


def merge_pair(old: Gmm, pi, nw, nm, nc, M):
    """Online update of pair pi (App. A): matching by the summed symmetric
    Mahalanobis distance, combination with the sample counts N and M."""
    N, K = old.n_trained, old.K
    if N <= 0.0:
        return np.array(nw), np.array(nm), np.array(nc)
    ow, om, oc = old.pw[pi], old.pmu[pi], old.pcov[pi]
    best, bp = None, None
    for p in itertools.permutations(range(K)):
        s = 0.0
        for i in range(K):
            d = om[p[i]] - nm[i]
            s += _maha(d, nc[i]) + _maha(d, oc[p[i]])
        if best is None or s < best:
            best, bp = s, p
    w, mu, cov = ow.copy(), om.copy(), oc.copy()
    for i in range(K):
        j = bp[i]
        a, b = N * ow[j], M * nw[i]
        if not a + b > 0.0:
            w[j] = 0.0
            continue
        d = om[j] - nm[i]
        mu[j] = (a * om[j] + b * nm[i]) / (a + b)
        f = a * b / ((a + b) * (a + b))
        cov[j] = regularize((a * oc[j] + b * nc[i]) / (a + b) + f * np.array([d[0] * d[0], d[0] * d[1], d[1] * d[1]]))
        w[j] = (a + b) / (N + M)
    return w, mu, cov


def adapt(g: Gmm | None, u, lnw, *, K, mask, eps, n_iter, pairs=()):
    """One round's update of a point's mixture from the round's u [7, n] and
    ln w [n]; g None (or a different K or pair list): start from the
    initial model."""
    pairs = [tuple(p) for p in pairs]
    cur = g.copy() if (g is not None and g.K == K and g.pairs == pairs) else Gmm(K, mask, eps, pairs=pairs)
    wt, M = weights(lnw)
    if not wt.sum() > 0.0:
        cur.mask, cur.eps = mask, eps
        return cur
    out = cur.copy()
    for d in range(7):
        if not (mask >> d) & 1 or d in cur.paired():
            continue
        nw, nm, ns = em_fit(u[d], wt, cur.w[d], cur.mu[d], cur.sd[d], n_iter)
        out.w[d], out.mu[d], out.sd[d] = merge(cur, nw, nm, ns, d, M)
    for pi, (a, b) in enumerate(pairs):
        nw, nm, nc = em_fit_pair(np.asarray(u[a], dtype=np.float64), np.asarray(u[b], dtype=np.float64), wt,
                                 cur.pw[pi], cur.pmu[pi], cur.pcov[pi], n_iter)
        out.pw[pi], out.pmu[pi], out.pcov[pi] = merge_pair(cur, pi, nw, nm, nc, M)
    out.n_trained = cur.n_trained + M
    out.mask, out.eps = mask, eps
    return out
