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


class Gmm:
    """Mixture state of one point: per parameter d, K components."""

    def __init__(self, K, mask, eps, w=None, mu=None, sd=None, n_trained=0.0):
        self.K, self.mask, self.eps, self.n_trained = int(K), int(mask), float(eps), float(n_trained)
        k = np.arange(K)
        self.w = np.tile(np.full(K, 1.0 / K), (7, 1)) if w is None else np.array(w, dtype=np.float64)
        self.mu = np.tile((k + 0.5) / K, (7, 1)) if mu is None else np.array(mu, dtype=np.float64)
        self.sd = np.tile(np.full(K, 0.5 / K), (7, 1)) if sd is None else np.array(sd, dtype=np.float64)

    def copy(self):
        return Gmm(self.K, self.mask, self.eps, self.w, self.mu, self.sd, self.n_trained)


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


def draw(seed, point, rnd, n, g: Gmm | None, *, d_min=10.0, d_max=1000.0, tau_width=0.0, start=0, frame=None):
    """Samples start..start+n-1 of (point, round) from the mixture proposal
    (prior where g is None or a parameter is outside g.mask): theta [7, n],
    ln p - ln p_s [n], u [7, n].  frame = (det_pos, gmst): the sky drawn in
    the network frame of detectors 0 and 1."""
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
            if not (g.mask >> d) & 1:
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
    th = np.stack([prior_inv(d, u[d], d_min, d_max, tau_width) for d in range(7)])
    if frame is not None:
        th[ALPHA], th[DELTA] = frame_sky(frame[0], frame[1], u[ALPHA], u[DELTA])
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


def adapt(g: Gmm | None, u, lnw, *, K, mask, eps, n_iter):
    """One round's update of a point's mixture from the round's u [7, n] and
    ln w [n]; g None (or a different K): start from the initial model."""
    cur = g.copy() if (g is not None and g.K == K) else Gmm(K, mask, eps)
    wt, M = weights(lnw)
    if not wt.sum() > 0.0:
        cur.mask, cur.eps = mask, eps
        return cur
    out = cur.copy()
    for d in range(7):
        if not (mask >> d) & 1:
            continue
        nw, nm, ns = em_fit(u[d], wt, cur.w[d], cur.mu[d], cur.sd[d], n_iter)
        out.w[d], out.mu[d], out.sd[d] = merge(cur, nw, nm, ns, d, M)
    out.n_trained = cur.n_trained + M
    out.mask, out.eps = mask, eps
    return out
