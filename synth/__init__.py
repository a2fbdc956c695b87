"""Seeded synthetic inputs for the ILE likelihood: detector geometry, mode
lists, mode-mode overlaps U and data-mode overlap series Q, and the five
workloads the tests and the benchmark run.

This module holds none of the likelihood's arithmetic (no antenna patterns,
no harmonics, no contraction, no time marginalization).  An injected signal
needs the injection's per-detector coefficients and arrival delays; those are
read from ``injections.npz``, which ``make_injections.py`` writes by calling
only the FP64 oracle.  Both the oracle and the HIP library consume what this
module returns; neither imports the other.

Recipe (standing in for lalsimulation waveforms and public strain data, which
the method's paper uses and which are not available here):

* detectors H1, L1, V1 at their published vertex positions with their arm
  unit vectors; response tensor D = (x x^T - y y^T) / 2;
* modes: 2 -> (2,+-2); 5 -> l=2; 9 -> l=2 plus (3,+-3), (3,+-2); 21 -> l=2..4;
* U_k = s_k G G^dagger / R with G in C^{M x R}, R = M + 2, i.i.d. CN(0, 1),
  per-detector sensitivity s_k ~ U[0.5, 1]; one common factor c scales every
  U_k so that the network SNR rho^2 = sum_k a_k^dagger U_k a_k / 2 at the
  injection hits the target;
* Q_k(t_r) = c U_k a_k K(t_r - t_inj - dt_k) / 2 + chol(c U_k) xi_r,
  xi_r ~ CN(0, I) i.i.d. per row, t_r = t_q0 + r / f_s, r = 0..L-1 with
  L = n_t + 2P + 3 and P = ceil(f_s max_k |r_k| / c_light + 1/2);
  K(tau) = exp(-tau^2 / 2 sigma^2) exp(-2 pi i f_c tau) with sigma = 3 ms,
  f_c = 100 Hz (the "gauss" kernel), or the truncated quadratic
  K(tau) = max(0, 1 - (tau / tau_0)^2) with tau_0 = 6 rows, reproduced exactly
  by a 4-tap cubic interpolant near its peak ("quad");
* the injection sits on window sample j = n_t // 2 at tau = 0.
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field

import numpy as np

C_SI = 299792458.0
BASE_SEED = 2210079120
HERE = os.path.dirname(os.path.abspath(__file__))
INJECTION_FILE = os.path.join(HERE, "injections.npz")

# Published site coordinates: Earth-fixed vertex positions (m) and arm unit
# vectors of the LIGO Hanford and Livingston sites (LIGO-T980044, Althouse,
# Jones & Lazzarini) and of Virgo (as tabulated by Anderson et al.,
# Phys. Rev. D 63, 042003 (2001)).
DETECTORS = {
    "H1": dict(
        vertex=(-2.16141492636e06, -3.83469517889e06, 4.60035022664e06),
        xarm=(-0.22389266154, 0.79983062746, 0.55690487831),
        yarm=(-0.91397818574, 0.02609403989, -0.40492342125),
    ),
    "L1": dict(
        vertex=(-7.42760447238e04, -5.49628371971e06, 3.22425701744e06),
        xarm=(-0.95457412153, -0.14158077340, -0.26218911324),
        yarm=(0.29774156894, -0.48791033647, -0.82054461286),
    ),
    "V1": dict(
        vertex=(4.54637409900e06, 8.42989697626e05, 4.37857696241e06),
        xarm=(-0.70045821479, 0.20848948619, 0.68256166277),
        yarm=(-0.05379255368, -0.96908180549, 0.24080451708),
    ),
}

MODE_SETS = {
    2: [(2, 2), (2, -2)],
    5: [(2, m) for m in (2, 1, 0, -1, -2)],
    9: [(2, m) for m in (2, 1, 0, -1, -2)] + [(3, 3), (3, -3), (3, 2), (3, -2)],
    21: [(l, m) for l in (2, 3, 4) for m in range(l, -l - 1, -1)],
}

PRIOR = dict(d_min=10.0, d_max=1000.0)


def detector_arrays(names):
    pos = np.array([DETECTORS[n]["vertex"] for n in names], dtype=np.float64)
    resp = []
    for n in names:
        x = np.array(DETECTORS[n]["xarm"])
        y = np.array(DETECTORS[n]["yarm"])
        resp.append(0.5 * (np.outer(x, x) - np.outer(y, y)))
    return pos, np.array(resp)


def pad_for(det_pos, f_s):
    tau_max = max(np.linalg.norm(r) for r in det_pos) / C_SI
    return int(math.ceil(f_s * tau_max + 0.5))


@dataclass
class PointSpec:
    """Everything that determines one synthetic intrinsic point."""
    seed: int
    dets: tuple = ("H1", "L1", "V1")
    n_modes: int = 21
    n_t: int = 820
    f_s: float = 4096.0
    snr: float = 25.0
    d_ref: float = 100.0
    kernel: str = "gauss"      # "gauss" | "quad" | "none"
    noise: bool = True
    sigma_t: float = 3e-3
    f_c: float = 100.0
    tau0_rows: float = 6.0     # quadratic kernel half-width in rows
    v_nonzero: bool = False    # add a random complex-symmetric V (tests only)

    def key(self):
        return f"{self.seed}:{','.join(self.dets)}:{self.n_modes}:{self.n_t}:{self.f_s}:{self.snr}"


def _rng(seed, *salt):
    return np.random.default_rng([int(seed) & 0xFFFFFFFFFFFF, *salt])


def draw_injection(spec: PointSpec):
    """Injected extrinsic parameters from the workload priors (tau = 0) and
    the sidereal angle gmst."""
    g = _rng(spec.seed, 1)
    u = g.random(7)
    th = np.array([
        2 * math.pi * u[0],
        math.asin(2 * u[1] - 1),
        math.pi * u[2],
        math.acos(2 * u[3] - 1),
        2 * math.pi * u[4],
        # keep injections loud enough to matter: D in [100, 600] Mpc
        100.0 + 500.0 * u[5],
        0.0,
    ])
    gmst = 2 * math.pi * g.random()
    return th, gmst


def make_U(spec: PointSpec):
    """Unscaled mode-mode overlaps [K, M, M] (Hermitian PSD) and optional V."""
    g = _rng(spec.seed, 2)
    K, M = len(spec.dets), spec.n_modes
    R = M + 2
    U = np.zeros((K, M, M), dtype=np.complex128)
    for k in range(K):
        G = (g.standard_normal((M, R)) + 1j * g.standard_normal((M, R))) / math.sqrt(2)
        s = 0.5 + 0.5 * g.random()
        U[k] = s * (G @ G.conj().T) / R
        U[k] = 0.5 * (U[k] + U[k].conj().T)
    V = None
    if spec.v_nonzero:
        V = np.zeros((K, M, M), dtype=np.complex128)
        for k in range(K):
            A = (g.standard_normal((M, M)) + 1j * g.standard_normal((M, M))) * 0.05
            V[k] = A + A.T
    return U, V


def geometry(spec: PointSpec):
    pos, resp = detector_arrays(spec.dets)
    P = pad_for(pos, spec.f_s)
    return pos, resp, P


def _fingerprint(th, U):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(th).tobytes())
    h.update(np.ascontiguousarray(U).tobytes())
    return h.hexdigest()[:16]


_INJ_CACHE = None


def load_injections(path=INJECTION_FILE):
    global _INJ_CACHE
    if _INJ_CACHE is None:
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} missing: run python synth/make_injections.py")
        with np.load(path, allow_pickle=False) as z:
            keys = [str(k) for k in z["keys"]]
            _INJ_CACHE = {k: dict(a=z[f"a_{i}"], dt=z[f"dt_{i}"], rho2=float(z["rho2"][i]),
                                  fp=str(z["fp"][i])) for i, k in enumerate(keys)}
    return _INJ_CACHE


def make_point(spec: PointSpec, injection=None):
    """Build one point.  ``injection`` = dict(a=[K, M] complex coefficients at
    the injected distance, dt=[K] arrival delays (s), rho2=network SNR^2 of
    the unscaled U); default: looked up in the fixture file."""
    th, gmst = draw_injection(spec)
    U0, V = make_U(spec)
    pos, resp, P = geometry(spec)
    K, M = len(spec.dets), spec.n_modes
    L = spec.n_t + 2 * P + 3
    ell = np.array([lm[0] for lm in MODE_SETS[M]], dtype=np.int32)
    em = np.array([lm[1] for lm in MODE_SETS[M]], dtype=np.int32)
    if injection is None and spec.kernel != "none":
        inj = load_injections().get(spec.key())
        if inj is None:
            raise KeyError(f"no injection for {spec.key()}: run python synth/make_injections.py")
        if inj["fp"] != _fingerprint(th, U0):
            raise ValueError(f"stale injection for {spec.key()}: run python synth/make_injections.py")
        injection = inj
    g = _rng(spec.seed, 3)
    t_q0 = 0.0
    j_inj = spec.n_t // 2
    t_inj = t_q0 + (P + 1 + j_inj) / spec.f_s
    t_r = t_q0 + np.arange(L) / spec.f_s
    if injection is not None and spec.kernel != "none":
        c = spec.snr ** 2 / injection["rho2"]
    else:
        c = 1.0
    U = c * U0
    Q = np.zeros((K, L, M), dtype=np.complex128)
    for k in range(K):
        if injection is not None and spec.kernel != "none":
            tau = t_r - t_inj - injection["dt"][k]
            if spec.kernel == "gauss":
                kern = np.exp(-tau ** 2 / (2 * spec.sigma_t ** 2)) * np.exp(-2j * math.pi * spec.f_c * tau)
            elif spec.kernel == "quad":
                t0 = spec.tau0_rows / spec.f_s
                kern = np.maximum(0.0, 1.0 - (tau / t0) ** 2).astype(np.complex128)
            else:
                raise ValueError(spec.kernel)
            sig = 0.5 * (U[k] @ injection["a"][k])
            Q[k] = kern[:, None] * sig[None, :]
        if spec.noise:
            Lc = np.linalg.cholesky(U[k] + 1e-12 * np.trace(U[k]).real / M * np.eye(M))
            xi = (g.standard_normal((L, M)) + 1j * g.standard_normal((L, M))) / math.sqrt(2)
            Q[k] += xi @ Lc.T
    return dict(Q=Q, U=U, V=V, det_pos=pos, det_resp=resp, ell=ell, em=em, n_t=spec.n_t, pad=P,
                f_s=spec.f_s, d_ref=spec.d_ref, gmst=gmst, theta_inj=th, j_inj=j_inj, t_q0=t_q0,
                snr=spec.snr, U_scale=c)


# --- workloads ---------------------------------------------------------------

@dataclass
class Workload:
    name: str
    precision: str                 # "fp64" | "fp32"
    points: list = field(default_factory=list)
    n_samples: list = field(default_factory=list)
    rounds: int = 1
    tau_width: float = 0.0
    adaptive: bool = False


def workload(name: str) -> Workload:
    """The five configurations of the method's benchmark plan, plus small
    parity cases ("tiny", "tiny_batched")."""
    if name == "plain":        # 1 point, FP64, H1+L1, (2,+-2), 410-sample window, SNR 15, 1e4
        s = PointSpec(seed=BASE_SEED + 0, dets=("H1", "L1"), n_modes=2, n_t=410, snr=15.0)
        return Workload(name, "fp64", [s], [10_000])
    if name == "single":       # 1 point, FP32, H1+L1+V1, 21 modes, 820-sample window, SNR 25, 1e6
        s = PointSpec(seed=BASE_SEED + 1, n_modes=21, n_t=820, snr=25.0)
        return Workload(name, "fp32", [s], [1_000_000])
    if name == "batched":      # 512 heterogeneous points
        g = _rng(BASE_SEED + 2, 0)
        pts, ns = [], []
        for i in range(512):
            M = int(g.choice([2, 5, 9, 21]))
            dets = ("H1", "L1") if g.random() < 0.5 else ("H1", "L1", "V1")
            n_t = int(g.integers(200, 801))
            n = int(round(10 ** g.uniform(5, 6)))
            snr = float(g.uniform(8, 40))
            pts.append(PointSpec(seed=BASE_SEED + 2 + 1000 * (i + 1), dets=dets, n_modes=M, n_t=n_t, snr=snr))
            ns.append(n)
        return Workload(name, "fp32", pts, ns)
    if name == "grad":         # gradient workload: 1e5 samples, tau drawn within one sample
        s = PointSpec(seed=BASE_SEED + 3, n_modes=21, n_t=820, snr=25.0)
        return Workload(name, "fp32", [s], [100_000], rounds=20, tau_width=1.0 / 4096.0)
    if name == "adaptive":     # 64 points x 10 rounds x 1e6, SNR 10..60
        g = _rng(BASE_SEED + 4, 0)
        pts = [PointSpec(seed=BASE_SEED + 4 + 1000 * (i + 1), n_modes=21, n_t=820,
                         snr=float(g.uniform(10, 60))) for i in range(64)]
        return Workload(name, "fp32", pts, [1_000_000] * 64, rounds=10, adaptive=True)
    if name == "quadrupole":   # 8 points, (2, +-2) only, SNR 25: 4 near face-on/off, 4 near edge-on
        pts, face, edge, i = [], 0, 0, 0
        while face < 4 or edge < 4:
            s = PointSpec(seed=BASE_SEED + 5 + 1000 * (i + 1), n_modes=2, n_t=410, snr=25.0)
            ci = abs(math.cos(draw_injection(s)[0][3]))
            if ci > 0.85 and face < 4:
                pts.append(s)
                face += 1
            elif ci < 0.3 and edge < 4:
                pts.append(s)
                edge += 1
            i += 1
        return Workload(name, "fp32", pts, [100_000] * 8, rounds=10, adaptive=True)
    if name == "tiny":
        s = PointSpec(seed=BASE_SEED + 10, dets=("H1", "L1", "V1"), n_modes=5, n_t=100, snr=12.0)
        return Workload(name, "fp32", [s], [4096])
    if name == "tiny_batched":
        g = _rng(BASE_SEED + 11, 0)
        pts, ns = [], []
        for i in range(6):
            M = [2, 5, 9, 21, 5, 2][i]
            dets = ("H1", "L1") if i % 2 else ("H1", "L1", "V1")
            pts.append(PointSpec(seed=BASE_SEED + 11 + 1000 * (i + 1), dets=dets, n_modes=M,
                                 n_t=int(g.integers(40, 200)), snr=float(g.uniform(8, 30))))
            ns.append(int(g.integers(100, 3000)))
        return Workload(name, "fp32", pts, ns)
    raise KeyError(name)


WORKLOADS = ("plain", "single", "batched", "grad", "adaptive", "quadrupole", "tiny", "tiny_batched")

# specs used only by the oracle's pin tests (quadratic kernel, no noise)
PIN_SPECS = [
    PointSpec(seed=BASE_SEED + 20, dets=("H1", "L1"), n_modes=2, n_t=64, snr=15.0, kernel="quad", noise=False),
    PointSpec(seed=BASE_SEED + 21, dets=("H1", "L1", "V1"), n_modes=21, n_t=64, snr=25.0, kernel="quad", noise=False),
    PointSpec(seed=BASE_SEED + 22, dets=("H1", "L1", "V1"), n_modes=5, n_t=64, snr=20.0, kernel="gauss", noise=False),
    PointSpec(seed=BASE_SEED + 23, dets=("H1", "L1", "V1"), n_modes=9, n_t=64, snr=20.0, kernel="gauss",
              noise=True, v_nonzero=True),
    PointSpec(seed=BASE_SEED + 30, dets=("H1", "L1", "V1"), n_modes=5, n_t=32, snr=10.0, kernel="quad",
              noise=False),
    PointSpec(seed=BASE_SEED + 33, dets=("H1", "L1"), n_modes=2, n_t=16, snr=8.0, kernel="gauss", noise=True),
]


def prior_samples(seed, n, tau_width=0.0, d_min=10.0, d_max=1000.0):
    """[7, n] FP64 draws from the workload priors (numpy PCG64)."""
    g = _rng(seed, 5)
    u = g.random((7, n))
    a3, b3 = d_min ** 3, d_max ** 3
    return np.stack([
        2 * math.pi * u[0], np.arcsin(2 * u[1] - 1), math.pi * u[2], np.arccos(2 * u[3] - 1),
        2 * math.pi * u[4], np.cbrt(a3 + u[5] * (b3 - a3)), (u[6] - 0.5) * tau_width,
    ])


def mixed_samples(point, seed, n, frac_near=0.5, tau_width=0.0):
    """Prior draws mixed with draws scattered around the injection, so that
    the high-likelihood region is exercised; FP32-representable values."""
    th = prior_samples(seed, n, tau_width)
    g = _rng(seed, 6)
    k = int(n * frac_near)
    if k and "theta_inj" in point:
        t0 = point["theta_inj"]
        sc = np.array([0.02, 0.02, 0.05, 0.1, 0.1, 0.1 * t0[5], 0.0])
        near = t0[:, None] + sc[:, None] * g.standard_normal((7, k))
        near[6] = (g.random(k) - 0.5) * tau_width
        near[5] = np.abs(near[5]) + 1.0
        th[:, :k] = near
    return th.astype(np.float32).astype(np.float64)


# points for Monte Carlo agreement tests: low SNR, so that a few 1e4 samples
# per round give n_eff in the tens to hundreds and the sigma estimates mean
# something
MC_SPECS = [
    PointSpec(seed=BASE_SEED + 40, dets=("H1", "L1", "V1"), n_modes=5, n_t=100, snr=3.0),
]


def all_specs():
    out = list(PIN_SPECS) + list(MC_SPECS)
    for w in WORKLOADS:
        out.extend(workload(w).points)
    return out


def fd_inputs(seed, n_det=2, n_modes=3, N=4096, df=0.5, f_low=20.0, f_high=None, noise=True):
    """Synthetic frequency-domain inputs for the Q/U/V precompute: a two-sided
    grid of N samples in FFT order (numpy.fft.fftfreq of N samples at
    f_s = N df), a coloured one-sided PSD per detector S_k(|f|) > 0, complex
    mode spectra h_m(f) ~ |f|^(-7/6) with a smooth random phase, independent on
    the two sides of the grid and zero outside [f_low, f_high], and data that
    is complex Gaussian noise (variance S_k / (4 df) per real part) or zero.
    Returns (data [K, N], psd [K, N], modes [M, N], f [N])."""
    g = _rng(seed, 21)
    f = np.fft.fftfreq(N, d=1.0 / (N * df))
    af = np.abs(f)
    f_high = f_high if f_high is not None else 0.4 * N * df
    fs = np.maximum(af, df)
    psd = np.empty((n_det, N))
    for k in range(n_det):
        psd[k] = g.uniform(0.5, 2.0) * (1.0 + (40.0 / fs) ** 4 + (fs / 300.0) ** 2)
    band = (af > f_low) & (af < f_high)
    modes = np.zeros((n_modes, N), dtype=np.complex128)
    for m in range(n_modes):
        c = g.normal(size=4)
        phase = c[0] + c[1] * fs / 100.0 + c[2] * np.sign(f) * (fs / 100.0) ** 2 + c[3] * (100.0 / fs)
        modes[m] = np.where(band, g.uniform(0.5, 2.0) * (fs / 100.0) ** (-7.0 / 6.0) * np.exp(1j * phase), 0.0)
    if noise:
        sig = np.sqrt(psd / (4.0 * df))
        data = sig * (g.normal(size=(n_det, N)) + 1j * g.normal(size=(n_det, N)))
    else:
        data = np.zeros((n_det, N), dtype=np.complex128)
    return data, psd, modes, f
