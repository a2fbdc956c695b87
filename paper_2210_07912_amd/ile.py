"""Python binding of the C ABI in ``include/rift_ile.h`` (ctypes).

Argument marshalling only: every step of the path runs in the HIP library
``librift_ile.so``.  PyTorch supplies device memory and the stream.  If the
library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librift_ile.so")

RIFT_FP32, RIFT_FP64 = 0, 1
NPAR = 7
NBINS = 100
STATUS = {0: "ok", -1: "invalid argument", -2: "shape", -3: "not Hermitian", -4: "window", -5: "non-finite",
          -6: "out of memory", -7: "device", -8: "state"}


class RiftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rift_ile status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class Point(C.Structure):
    _fields_ = [
        ("n_det", C.c_int), ("n_modes", C.c_int), ("n_t", C.c_int), ("pad", C.c_int),
        ("ell", C.POINTER(C.c_int)), ("em", C.POINTER(C.c_int)),
        ("f_s", C.c_double), ("d_ref", C.c_double), ("gmst", C.c_double),
        ("det_pos", C.POINTER(C.c_double)), ("det_resp", C.POINTER(C.c_double)),
        ("Q", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)), ("V", C.POINTER(C.c_double)),
    ]


class Desc(C.Structure):
    _fields_ = [("n_points", C.c_int), ("points", C.POINTER(Point)), ("precision", C.c_int),
                ("d_min", C.c_double), ("d_max", C.c_double), ("tau_width", C.c_double)]


class FdPoint(C.Structure):
    _fields_ = [("n_det", C.c_int), ("n_modes", C.c_int), ("n_f", C.c_int64), ("df", C.c_double),
                ("f_low", C.c_double), ("data", C.c_void_p), ("psd", C.c_void_p), ("modes", C.c_void_p)]


class Item(C.Structure):
    _fields_ = [("point", C.c_int), ("offset", C.c_int64), ("count", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("lnL_marg", C.c_double), ("sigma_lnL", C.c_double), ("n_eff", C.c_double),
                ("n_ess", C.c_double), ("n_var", C.c_double), ("max_lnw", C.c_double),
                ("n", C.c_int64), ("n_nonfinite", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MC(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_per_round", C.c_int64), ("n_per_point", C.POINTER(C.c_int64)),
                ("n_rounds", C.c_int), ("adapt_mask", C.c_uint), ("floor_eps", C.c_double),
                ("reset_proposal", C.c_int), ("flags", C.c_uint), ("n_ascent", C.c_int),
                ("ascent_steps", C.c_int), ("ascent_mix", C.c_double), ("gmm_components", C.c_int),
                ("gmm_iters", C.c_int), ("gmm_pairs", C.c_uint), ("first_round", C.c_int)]


RIFT_MC_GRADIENT = 1
GMM_MAX = 4  # mixture components per parameter


def encode_pairs(pairs):
    """[(a, b), ...] -> byte code (byte i = a | b << 4)."""
    code = 0
    for i, (a, b) in enumerate(pairs):
        code |= (int(a) | int(b) << 4) << (8 * i)
    return code


def decode_pairs(code):
    return [((code >> (8 * i)) & 15, (code >> (8 * i + 4)) & 15) for i in range(3) if (code >> (8 * i)) & 0xFF]


FUNCTIONS = {
    "rift_ile_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Desc), C.c_void_p]),
    "rift_ile_destroy": (None, [C.c_void_p]),
    "rift_ile_last_error": (C.c_char_p, [C.c_void_p]),
    "rift_ile_status_string": (C.c_char_p, [C.c_int]),
    "rift_ile_abi_version": (C.c_int, []),
    "rift_ile_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rift_ile_set_graph": (C.c_int, [C.c_void_p, C.c_int]),
    "rift_ile_graph_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "rift_ile_set_autotune": (C.c_int, [C.c_void_p, C.c_int]),
    "rift_ile_set_network_frame": (C.c_int, [C.c_void_p, C.c_int]),
    "rift_ile_set_phase_rotation": (C.c_int, [C.c_void_p, C.c_int]),
    "rift_ile_set_distance_marginalization": (C.c_int, [C.c_void_p, C.c_int]),
    "rift_ile_set_autotune_cache": (C.c_int, [C.c_void_p, C.c_char_p]),
    "rift_ile_set_grad_refine": (C.c_int, [C.c_void_p, C.c_int]),
    "rift_ile_precompute": (C.c_int, [C.POINTER(FdPoint), C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "rift_ile_autotune_table": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "rift_ile_profile": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "rift_ile_sample": (C.c_int, [C.c_void_p, C.c_int, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
    "rift_ile_lnL": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(Item), C.c_int64, C.c_void_p, C.c_void_p]),
    "rift_ile_reduce": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(Result)]),
    "rift_ile_reduce_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(Result)]),
    "rift_ile_adapt": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_uint, C.c_double]),
    "rift_ile_get_proposal": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_uint)]),
    "rift_ile_set_proposal": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_uint]),
    "rift_ile_get_gmm": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_uint),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rift_ile_set_gmm": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_uint, C.c_double, C.c_double,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rift_ile_adapt_gmm": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_uint, C.c_uint,
                                     C.c_double, C.c_int, C.c_int]),
    "rift_ile_set_gmm_pairs": (C.c_int, [C.c_void_p, C.c_int, C.c_uint, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rift_ile_get_gmm_pairs": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_uint), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rift_ile_marginalize": (C.c_int, [C.c_void_p, C.POINTER(MC), C.POINTER(Result), C.c_void_p, C.c_void_p]),
    "rift_ile_checkpoint_bytes": (C.c_int64, [C.c_void_p]),
    "rift_ile_save_checkpoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "rift_ile_load_checkpoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "rift_ile_backward": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(Item), C.c_int64, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
}

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_2210_07912_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in FUNCTIONS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def build_desc(points, precision=RIFT_FP32, d_min=10.0, d_max=1000.0, tau_width=0.0):
    """rift_ile_desc for a list of point dicts; returns (desc, arrays to keep
    alive for the duration of rift_ile_create)."""
    keep = []
    arr = (Point * len(points))()
    for i, p in enumerate(points):
        Q = np.ascontiguousarray(np.asarray(p["Q"]).astype(np.complex128)).view(np.float64)
        U = np.ascontiguousarray(np.asarray(p["U"]).astype(np.complex128)).view(np.float64)
        V = None if p.get("V") is None else np.ascontiguousarray(np.asarray(p["V"]).astype(np.complex128)).view(np.float64)
        pos = np.ascontiguousarray(p["det_pos"], dtype=np.float64)
        resp = np.ascontiguousarray(p["det_resp"], dtype=np.float64)
        ell = np.ascontiguousarray(p["ell"], dtype=np.int32)
        em = np.ascontiguousarray(p["em"], dtype=np.int32)
        keep += [Q, U, V, pos, resp, ell, em]
        arr[i] = Point(pos.shape[0], ell.shape[0], int(p["n_t"]), int(p["pad"]),
                       ell.ctypes.data_as(C.POINTER(C.c_int)), em.ctypes.data_as(C.POINTER(C.c_int)),
                       float(p["f_s"]), float(p["d_ref"]), float(p["gmst"]), _dptr(pos), _dptr(resp),
                       _dptr(Q), _dptr(U), _dptr(V))
    keep.append(arr)
    return Desc(len(points), arr, precision, d_min, d_max, tau_width), keep


class RiftILE:
    """A handle on one or more intrinsic points.

    points: list of dicts with Q [K, L, M] complex, U [K, M, M] complex,
    optional V, det_pos [K, 3], det_resp [K, 3, 3], ell, em, n_t, pad, f_s,
    d_ref, gmst (the layout of ``rift_ile_point``).
    """

    def __init__(self, points, precision="fp32", d_min=10.0, d_max=1000.0, tau_width=0.0, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("RiftILE needs a HIP device")
        self.device = torch.device(device or "cuda")
        self.precision = RIFT_FP32 if precision == "fp32" else RIFT_FP64
        self.dtype = torch.float32 if self.precision == RIFT_FP32 else torch.float64
        self.n_points = len(points)
        desc, keep = build_desc(points, self.precision, d_min, d_max, tau_width)
        self.meta = [dict(K=int(np.asarray(p["det_pos"]).shape[0]), M=len(p["ell"]), n_t=int(p["n_t"])) for p in points]
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            st = lib().rift_ile_create(C.byref(h), C.byref(desc), C.c_void_p(self.stream.cuda_stream))
        del keep
        if st != 0:
            raise RiftError(st, lib().rift_ile_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().rift_ile_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise RiftError(st, lib().rift_ile_last_error(self.h).decode())

    def _as_theta(self, theta):
        t = torch.as_tensor(theta, device=self.device, dtype=self.dtype)
        if t.dim() != 2 or t.shape[0] != NPAR:
            raise ValueError("theta must be [7, N]")
        return t.contiguous()

    def set_graph(self, enable=True):
        """Capture each FP32 evaluation run into a hipGraph once and replay it
        when a later run has the same shape and buffers."""
        self._check(lib().rift_ile_set_graph(self.h, int(enable)))

    def graph_stats(self):
        """(graphs captured, replays launched) since the handle was created."""
        c, r = C.c_int64(), C.c_int64()
        self._check(lib().rift_ile_graph_stats(self.h, C.byref(c), C.byref(r)))
        return c.value, r.value

    def set_network_frame(self, enable=True):
        """Draw the sky in each point's detector-network frame (pole along
        the baseline of its detectors 0 and 1); the histograms of dimensions
        0 and 1 then adapt in that frame's azimuth and polar cosine."""
        self._check(lib().rift_ile_set_network_frame(self.h, int(enable)))

    def set_phase_rotation(self, enable=True):
        """Draw polarization and orbital phase in the phase-rotated
        coordinates u_s = (phi + psi) / 4 pi, u_d = (phi - psi) / 4 pi; the
        histograms and mixtures of dimensions 2 and 4 then adapt in those."""
        self._check(lib().rift_ile_set_phase_rotation(self.h, int(enable)))

    def set_distance_marginalization(self, enable=True):
        """lnL and marginalize return ln L_tD, integrated over the distance
        prior p(D) ~ D^2 on [d_min, d_max]; theta's distance is not read."""
        self._check(lib().rift_ile_set_distance_marginalization(self.h, int(enable)))

    def set_grad_refine(self, enable=True):
        """FP64 re-evaluation of the FP32 adjoint over the window blocks that
        hold each sample's softmax mass (default on)."""
        self._check(lib().rift_ile_set_grad_refine(self.h, int(enable)))

    def set_autotune(self, mode=1):
        """Launch configuration of FP32 evaluations: 1 (default) measure the
        seven configurations (staged or direct feed, full or half residency,
        the direct feed with registers capped for three or four wavefronts per
        SIMD, the staged feed capped for three) of each (T, K) class and n_t
        bucket on its first evaluation and use the fastest; 0 always staged;
        2 always direct; 3, 4 always the capped direct forms; 5 always the
        capped staged form.  ``True``/``False`` mean 1/0."""
        self._check(lib().rift_ile_set_autotune(self.h, int(mode)))

    def autotune_table(self):
        """{(T, K): configuration} for the classes run so far: "staged",
        "direct", "staged/half", "direct/half" (half: half the resident
        workgroups per compute unit), "direct/3w", "direct/4w" or "staged/3w"
        (registers capped for three or four wavefronts per SIMD)."""
        arr = (C.c_int * 48)()
        self._check(lib().rift_ile_autotune_table(self.h, arr))
        names = {1: "staged", 2: "direct", 3: "staged/half", 4: "direct/half", 5: "direct/3w", 6: "direct/4w",
                 7: "staged/3w"}
        return {(i // 3 + 1, i % 3 + 1): names[v] for i, v in enumerate(arr) if v in names}

    def set_autotune_cache(self, path):
        """Read measured launch configurations from ``path`` (if it exists)
        and append new measurements to it; None: stop appending."""
        self._check(lib().rift_ile_set_autotune_cache(self.h, None if path is None else str(path).encode()))

    def profile(self, enable=True):
        """(ms, launches) of the dominant kernel since the last call; then
        switch event timing on or off."""
        ms, n = C.c_double(), C.c_int64()
        self._check(lib().rift_ile_profile(self.h, int(enable), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # --- entry points -------------------------------------------------------
    def sample(self, point, seed, rnd, n, first=0):
        th = torch.empty((NPAR, n), device=self.device, dtype=self.dtype)
        lr = torch.empty(n, device=self.device, dtype=self.dtype)
        bins = torch.empty((NPAR, n), device=self.device, dtype=torch.uint8)
        self._check(lib().rift_ile_sample(self.h, point, seed, rnd, first, n, _ptr(th), _ptr(lr), _ptr(bins)))
        return th, lr, bins

    def lnL(self, theta, items=None):
        """theta [7, N] -> ln L_t [N].  items: list of (point, offset, count);
        default: all columns against point 0."""
        th = self._as_theta(theta)
        n = th.shape[1]
        out = torch.empty(n, device=self.device, dtype=self.dtype)
        its = items if items is not None else [(0, 0, n)]
        arr = (Item * len(its))(*[Item(int(p), int(o), int(c)) for p, o, c in its])
        self._check(lib().rift_ile_lnL(self.h, len(its), arr, n, _ptr(th), _ptr(out)))
        return out

    def reduce(self, lnL, ln_ratio=None):
        lnL = torch.as_tensor(lnL, device=self.device, dtype=self.dtype).contiguous()
        lr = None if ln_ratio is None else torch.as_tensor(ln_ratio, device=self.device, dtype=self.dtype).contiguous()
        r = Result()
        self._check(lib().rift_ile_reduce(self.h, lnL.numel(), _ptr(lnL), _ptr(lr), C.byref(r)))
        return r.as_dict()

    def reduce_noalloc(self, lnL, ln_ratio=None):
        """The reduction of ``reduce`` through the entry point that allocates
        no device memory (its scratch is a static device array)."""
        lnL = torch.as_tensor(lnL, device=self.device, dtype=self.dtype).contiguous()
        lr = None if ln_ratio is None else torch.as_tensor(ln_ratio, device=self.device, dtype=self.dtype).contiguous()
        r = Result()
        self._check(lib().rift_ile_reduce_noalloc(self.h, lnL.numel(), _ptr(lnL), _ptr(lr), C.byref(r)))
        return r.as_dict()

    def adapt(self, point, bins, lnw, mask=0x3F, floor_eps=0.1):
        bins = torch.as_tensor(bins, device=self.device, dtype=torch.uint8).contiguous()
        lnw = torch.as_tensor(lnw, device=self.device, dtype=self.dtype).contiguous()
        self._check(lib().rift_ile_adapt(self.h, point, lnw.numel(), _ptr(bins), _ptr(lnw), mask, floor_eps))

    def get_proposal(self, point):
        cdf = np.zeros((NPAR, NBINS + 1))
        mask = C.c_uint()
        self._check(lib().rift_ile_get_proposal(self.h, point, _dptr(cdf), C.byref(mask)))
        return cdf, mask.value

    def set_proposal(self, point, cdf, mask):
        cdf = np.ascontiguousarray(cdf, dtype=np.float64)
        self._check(lib().rift_ile_set_proposal(self.h, point, _dptr(cdf), mask))

    def get_gmm(self, point):
        """Mixture proposal of a point: dict K, mask, floor_eps, n_trained and
        w, mu, sd [7, 4] (K = 0: the point holds a histogram proposal)."""
        K, mask, eps, ntr = C.c_int(), C.c_uint(), C.c_double(), C.c_double()
        w, mu, sd = (np.zeros((NPAR, GMM_MAX)) for _ in range(3))
        self._check(lib().rift_ile_get_gmm(self.h, point, C.byref(K), C.byref(mask), C.byref(eps), C.byref(ntr),
                                           _dptr(w), _dptr(mu), _dptr(sd)))
        return dict(K=K.value, mask=mask.value, floor_eps=eps.value, n_trained=ntr.value, w=w, mu=mu, sd=sd)

    def set_gmm(self, point, K, mask, floor_eps, n_trained, w, mu, sd):
        arrs = []
        for a in (w, mu, sd):
            x = np.zeros((NPAR, GMM_MAX))
            a = np.asarray(a, dtype=np.float64)
            x[:, :a.shape[1]] = a
            arrs.append(np.ascontiguousarray(x))
        self._check(lib().rift_ile_set_gmm(self.h, point, K, mask, floor_eps, n_trained, *(_dptr(a) for a in arrs)))

    def adapt_gmm(self, point, u, lnw, mask, floor_eps, K, n_iter, pairs=()):
        u = torch.as_tensor(u, device=self.device, dtype=torch.float32).contiguous()
        lnw = torch.as_tensor(lnw, device=self.device, dtype=self.dtype).contiguous()
        self._check(lib().rift_ile_adapt_gmm(self.h, point, lnw.numel(), _ptr(u), _ptr(lnw), mask,
                                             encode_pairs(pairs), floor_eps, K, n_iter))

    def set_gmm_pairs(self, point, pairs, w, mu, cov):
        """pairs: list of (a, b); w [P, K], mu [P, K, 2], cov [P, K, 3]."""
        W, MU, CV = np.zeros((3, GMM_MAX)), np.zeros((3, GMM_MAX, 2)), np.zeros((3, GMM_MAX, 3))
        for i in range(len(pairs)):
            k = np.asarray(w[i]).shape[0]
            W[i, :k], MU[i, :k], CV[i, :k] = w[i], mu[i], cov[i]
        self._check(lib().rift_ile_set_gmm_pairs(self.h, point, encode_pairs(pairs), _dptr(W), _dptr(MU),
                                                 _dptr(CV)))

    def get_gmm_pairs(self, point):
        code = C.c_uint()
        W, MU, CV, Z = np.zeros((3, GMM_MAX)), np.zeros((3, GMM_MAX, 2)), np.zeros((3, GMM_MAX, 3)), np.zeros(3)
        self._check(lib().rift_ile_get_gmm_pairs(self.h, point, C.byref(code), _dptr(W), _dptr(MU), _dptr(CV),
                                                 _dptr(Z)))
        return dict(pairs=decode_pairs(code.value), w=W, mu=MU, cov=CV, box_mass=Z)

    def marginalize(self, seed, n_per_point, n_rounds=1, adapt_mask=0, floor_eps=0.1, reset=True,
                    return_samples=False, gradient=False, n_ascent=0, ascent_steps=0, ascent_mix=0.0,
                    gmm_components=0, gmm_iters=0, gmm_pairs=(), first_round=0):
        npp = np.ascontiguousarray(np.broadcast_to(np.asarray(n_per_point, dtype=np.int64), (self.n_points,)))
        mc = MC(seed, 0, npp.ctypes.data_as(C.POINTER(C.c_int64)), n_rounds, adapt_mask, floor_eps, int(reset),
                RIFT_MC_GRADIENT if gradient else 0, n_ascent, ascent_steps, ascent_mix, gmm_components, gmm_iters,
                encode_pairs(gmm_pairs), first_round)
        res = (Result * self.n_points)()
        th = lw = None
        if return_samples:
            total = int(npp.sum()) * n_rounds
            th = torch.empty((NPAR, total), device=self.device, dtype=self.dtype)
            lw = torch.empty(total, device=self.device, dtype=self.dtype)
        self._check(lib().rift_ile_marginalize(self.h, C.byref(mc), res, _ptr(th), _ptr(lw)))
        out = [r.as_dict() for r in res]
        if return_samples:
            return out, th, lw
        return out

    def save_checkpoint(self):
        """Proposals and pooled estimates of every point, as bytes."""
        n = lib().rift_ile_checkpoint_bytes(self.h)
        buf = C.create_string_buffer(n)
        self._check(lib().rift_ile_save_checkpoint(self.h, buf, n))
        return buf.raw

    def load_checkpoint(self, data):
        buf = C.create_string_buffer(bytes(data), len(data))
        self._check(lib().rift_ile_load_checkpoint(self.h, buf, len(data)))

    def backward(self, theta, grad_lnL=None, items=None, want_lnL=False):
        th = self._as_theta(theta)
        n = th.shape[1]
        g = None if grad_lnL is None else torch.as_tensor(grad_lnL, device=self.device, dtype=self.dtype).contiguous()
        out = torch.empty((NPAR, n), device=self.device, dtype=self.dtype)
        lt = torch.empty(n, device=self.device, dtype=self.dtype) if want_lnL else None
        its = items if items is not None else [(0, 0, n)]
        arr = (Item * len(its))(*[Item(int(p), int(o), int(c)) for p, o, c in its])
        self._check(lib().rift_ile_backward(self.h, len(its), arr, n, _ptr(th), _ptr(g), _ptr(out), _ptr(lt)))
        return (out, lt) if want_lnL else out


def precompute(data, psd, modes, df, f_low, row0, n_rows):
    """Q [K, n_rows, M], U, V [K, M, M] (complex128, host) of Eq. (QUV) from
    frequency-domain data [K, N], PSD values S_k(|f_i|) [K, N] and modes
    [M, N] on the two-sided grid in FFT order (rift_ile_precompute)."""
    data = np.ascontiguousarray(np.asarray(data, dtype=np.complex128))
    psd = np.ascontiguousarray(np.asarray(psd, dtype=np.float64))
    modes = np.ascontiguousarray(np.asarray(modes, dtype=np.complex128))
    K, N = data.shape
    M = modes.shape[0]
    if psd.shape != (K, N) or modes.shape[1] != N:
        raise ValueError("data [K, N], psd [K, N], modes [M, N]")
    fd = FdPoint(K, M, N, float(df), float(f_low), data.ctypes.data, psd.ctypes.data, modes.ctypes.data)
    Q = np.zeros((K, n_rows, M), dtype=np.complex128)
    U = np.zeros((K, M, M), dtype=np.complex128)
    V = np.zeros((K, M, M), dtype=np.complex128)
    st = lib().rift_ile_precompute(C.byref(fd), int(row0), int(n_rows), Q.ctypes.data, U.ctypes.data, V.ctypes.data)
    if st != 0:
        raise RiftError(st, lib().rift_ile_last_error(None).decode())
    return Q, U, V


class LnLFunction(torch.autograd.Function):
    """ln L_t(theta) with the hand-written adjoint as its backward."""

    @staticmethod
    def forward(ctx, theta, handle, items=None):
        ctx.handle, ctx.items = handle, items
        ctx.save_for_backward(theta)
        return handle.lnL(theta, items)

    @staticmethod
    def backward(ctx, grad_out):
        (theta,) = ctx.saved_tensors
        g = ctx.handle.backward(theta, grad_out.contiguous(), ctx.items)
        return g, None, None


def lnL_autograd(handle, theta, items=None):
    return LnLFunction.apply(theta, handle, items)
