"""Python handle on the FP64 CPU oracle (``liboracle.so``, built from
``rift_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product package never does.
It is argument marshalling: every number comes out of the C oracle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ALPHA, DELTA, PSI, IOTA, PHI, DIST, TAU = range(7)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable flags: the library travels to
    other hosts)."""
    if force or not os.path.exists(LIB_PATH):
        src = os.path.join(HERE, "rift_oracle.c")
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", src, "-o", tmp, "-lm"]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Point(C.Structure):
    _fields_ = [
        ("K", C.c_int), ("M", C.c_int), ("n_t", C.c_int), ("pad", C.c_int),
        ("ell", C.POINTER(C.c_int)), ("em", C.POINTER(C.c_int)),
        ("f_s", C.c_double), ("d_ref", C.c_double), ("gmst", C.c_double),
        ("det_pos", C.POINTER(C.c_double)), ("det_resp", C.POINTER(C.c_double)),
        ("Q", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)), ("V", C.POINTER(C.c_double)),
    ]


class _Result(C.Structure):
    _fields_ = [
        ("lnL_marg", C.c_double), ("sigma_lnL", C.c_double), ("n_eff", C.c_double),
        ("n_ess", C.c_double), ("n_var", C.c_double), ("max_lnw", C.c_double),
        ("n", C.c_int64), ("n_nonfinite", C.c_int64),
    ]


_lib = None
_dp = C.POINTER(C.c_double)


def _load(path):
    L = C.CDLL(path)
    L.or_delay.restype = C.c_double
    L.or_lnL_t.restype = C.c_double
    L.or_lnL_tD.restype = C.c_double
    L.or_u01.restype = C.c_double
    L.or_rows.restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _load(LIB_PATH)
    return _lib


def use_native_build(out_dir):
    """Compile the oracle for the host it runs on (-O3 -march=native, OpenMP)
    into out_dir and make this module use that build.  For timing the oracle
    as a CPU baseline; the portable build stays the one the tests load."""
    global _lib
    src = os.path.join(HERE, "rift_oracle.c")
    path = os.path.join(out_dir, "liboracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11", src, "-o", path,
                           "-lm"])
    _lib = _load(path)
    return path


def threads():
    return lib().or_threads()


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


class Point:
    """One intrinsic point, held as contiguous FP64 arrays.

    Q: complex [K, L, M]; U, V: complex [K, M, M]; det_pos [K, 3];
    det_resp [K, 3, 3].  Complex inputs may be complex64 (the FP32-rounded
    values a GPU run consumed); they are upcast exactly.
    """

    def __init__(self, *, Q, U, det_pos, det_resp, ell, em, n_t, pad, f_s, d_ref, gmst, V=None):
        self.Q = np.ascontiguousarray(np.asarray(Q).astype(np.complex128)).view(np.float64)
        self.U = np.ascontiguousarray(np.asarray(U).astype(np.complex128)).view(np.float64)
        self.V = None if V is None else np.ascontiguousarray(np.asarray(V).astype(np.complex128)).view(np.float64)
        self.det_pos = np.ascontiguousarray(det_pos, dtype=np.float64)
        self.det_resp = np.ascontiguousarray(det_resp, dtype=np.float64)
        self.ell = np.ascontiguousarray(ell, dtype=np.int32)
        self.em = np.ascontiguousarray(em, dtype=np.int32)
        K, M = self.det_pos.shape[0], self.ell.shape[0]
        L = n_t + 2 * pad + 3
        assert np.asarray(Q).shape == (K, L, M), (np.asarray(Q).shape, (K, L, M))
        assert np.asarray(U).shape == (K, M, M)
        self.K, self.M, self.n_t, self.pad, self.L = K, M, n_t, pad, L
        self.s = _Point(
            K, M, n_t, pad,
            self.ell.ctypes.data_as(C.POINTER(C.c_int)), self.em.ctypes.data_as(C.POINTER(C.c_int)),
            float(f_s), float(d_ref), float(gmst),
            _ptr(self.det_pos), _ptr(self.det_resp), _ptr(self.Q), _ptr(self.U), _ptr(self.V),
        )

    @classmethod
    def from_dict(cls, d, complex64=False):
        cast = (lambda z: np.asarray(z).astype(np.complex64)) if complex64 else (lambda z: z)
        return cls(Q=cast(d["Q"]), U=cast(d["U"]), V=None if d.get("V") is None else cast(d["V"]),
                   det_pos=d["det_pos"], det_resp=d["det_resp"], ell=d["ell"], em=d["em"],
                   n_t=d["n_t"], pad=d["pad"], f_s=d["f_s"], d_ref=d["d_ref"], gmst=d["gmst"])


def _theta7(theta):
    t = np.zeros(7)
    t[: len(theta)] = theta
    return t


# --- geometry --------------------------------------------------------------

def antenna(D, alpha, delta, psi, gmst):
    fp, fc = C.c_double(), C.c_double()
    lib().or_antenna(_ptr(np.ascontiguousarray(D, dtype=np.float64).reshape(9)), C.c_double(alpha),
                     C.c_double(delta), C.c_double(psi), C.c_double(gmst), C.byref(fp), C.byref(fc))
    return fp.value, fc.value


def delay(r, alpha, delta, gmst):
    return lib().or_delay(_ptr(np.ascontiguousarray(r, dtype=np.float64)), C.c_double(alpha),
                          C.c_double(delta), C.c_double(gmst))


def direction(alpha, delta, gmst):
    n = np.zeros(3)
    lib().or_direction(C.c_double(alpha), C.c_double(delta), C.c_double(gmst), _ptr(n))
    return n


def sylm(l, m, iota, phi):
    re, im = C.c_double(), C.c_double()
    lib().or_sylm(l, m, C.c_double(iota), C.c_double(phi), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def catmull_rom(mu):
    w, dw = np.zeros(4), np.zeros(4)
    lib().or_catmull_rom(C.c_double(mu), _ptr(w), _ptr(dw))
    return w, dw


# --- likelihood ------------------------------------------------------------

def coeffs(p: Point, theta):
    a = np.zeros(2 * p.K * p.M)
    B = C.c_double()
    lib().or_coeffs(C.byref(p.s), _ptr(_theta7(theta)), _ptr(a), C.byref(B))
    return a.view(np.complex128).reshape(p.K, p.M), B.value


def ell(p: Point, theta):
    out = np.zeros(p.n_t)
    lib().or_ell(C.byref(p.s), _ptr(_theta7(theta)), _ptr(out))
    return out


def lnL_t(p: Point, theta):
    """theta: [7] -> float, or [7, N] -> [N] (OpenMP over samples)."""
    th = np.asarray(theta, dtype=np.float64)
    if th.ndim == 1:
        return lib().or_lnL_t(C.byref(p.s), _ptr(_theta7(th)))
    th = np.ascontiguousarray(th)
    n = th.shape[1]
    out = np.zeros(n)
    lib().or_lnL_t_batch(C.byref(p.s), C.c_int64(n), C.c_int64(n), _ptr(th), _ptr(out))
    return out


def lnL_tD(p: Point, theta, d_min=10.0, d_max=1000.0, panels=0):
    """Distance-marginalized ln L_tD: theta [7] (theta[5] not read) -> float,
    or [7, N] -> [N] (OpenMP over samples)."""
    th = np.asarray(theta, dtype=np.float64)
    if th.ndim == 1:
        return lib().or_lnL_tD(C.byref(p.s), _ptr(_theta7(th)), C.c_double(d_min), C.c_double(d_max), int(panels))
    th = np.ascontiguousarray(th)
    n = th.shape[1]
    out = np.zeros(n)
    lib().or_lnL_tD_batch(C.byref(p.s), C.c_int64(n), C.c_int64(n), _ptr(th), C.c_double(d_min), C.c_double(d_max),
                          int(panels), _ptr(out))
    return out


def gauss_legendre(n):
    x, w = np.zeros(n), np.zeros(n)
    lib().or_gauss_legendre(int(n), _ptr(x), _ptr(w))
    return x, w


def grad(p: Point, theta):
    """theta [7, N] -> (lnL_t [N], grad [7, N])."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    if th.ndim == 1:
        th = th.reshape(7, 1)
    n = th.shape[1]
    l, g = np.zeros(n), np.zeros((7, n))
    lib().or_grad_batch(C.byref(p.s), C.c_int64(n), C.c_int64(n), _ptr(th), _ptr(l), _ptr(g))
    return l, g


def reduce(lnw):
    lnw = np.ascontiguousarray(lnw, dtype=np.float64)
    r = _Result()
    lib().or_reduce(C.c_int64(lnw.size), _ptr(lnw), C.byref(r))
    return {f: getattr(r, f) for f, _ in _Result._fields_}


# --- sampler ---------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return list(o)


def u01(x):
    return lib().or_u01(C.c_uint32(x))


def draw(seed, point, rnd, n, *, d_min=10.0, d_max=1000.0, tau_width=0.0, cdf=None, nb=100,
         adapt_mask=0, start=0, frame=None, phase=False):
    """Samples start..start+n-1 of (point, round): theta [7, n], ln_ratio [n],
    bins [7, n] (uint8), raw Philox words [8, n].  frame = (det_pos [>=2, 3],
    gmst): the sky is drawn in the network frame of detectors 0 and 1.
    phase: polarization and phase drawn in phase-rotated coordinates."""
    th = np.zeros((7, n))
    lr = np.zeros(n)
    bins = np.zeros((7, n), dtype=np.uint8)
    raw = np.zeros((8, n), dtype=np.uint32)
    cd = None if cdf is None else np.ascontiguousarray(cdf, dtype=np.float64)
    t7 = np.zeros(7)
    l1 = C.c_double()
    b7 = (C.c_uint8 * 7)()
    r8 = (C.c_uint32 * 8)()
    L = lib()
    fp = None if frame is None else np.ascontiguousarray(np.asarray(frame[0], dtype=np.float64)[:2].reshape(6))
    gm = 0.0 if frame is None else float(frame[1])
    for i in range(n):
        L.or_draw_coords(C.c_uint64(seed), C.c_uint32(point), C.c_uint32(rnd), C.c_uint64(start + i),
                         C.c_double(d_min), C.c_double(d_max), C.c_double(tau_width), _ptr(cd), nb,
                         C.c_uint(adapt_mask), _ptr(fp), C.c_double(gm), int(bool(phase)), _ptr(t7), C.byref(l1),
                         b7, r8)
        th[:, i] = t7
        lr[i] = l1.value
        bins[:, i] = list(b7)
        raw[:, i] = list(r8)
    return th, lr, bins, raw


def phase_rot(us, ud):
    """Phase-rotated coordinates (u_s, u_d) -> (psi, phi)."""
    psi, phi = C.c_double(), C.c_double()
    lib().or_phase_rot(C.c_double(us), C.c_double(ud), C.byref(psi), C.byref(phi))
    return psi.value, phi.value


def network_frame(det_pos):
    """[3, 3] rows x', y', z' of the network sky frame of detectors 0 and 1."""
    fp = np.ascontiguousarray(np.asarray(det_pos, dtype=np.float64)[:2].reshape(6))
    ax = np.zeros(9)
    lib().or_network_frame(_ptr(fp), _ptr(ax))
    return ax.reshape(3, 3)


def frame_u(det_pos, gmst, alpha, delta):
    """(alpha, delta) -> (u_phi', u_cos theta') in the network frame."""
    fp = np.ascontiguousarray(np.asarray(det_pos, dtype=np.float64)[:2].reshape(6))
    u0, u1 = C.c_double(), C.c_double()
    lib().or_frame_u(_ptr(fp), C.c_double(gmst), C.c_double(alpha), C.c_double(delta), C.byref(u0), C.byref(u1))
    return u0.value, u1.value


def adapt(bins, lnw, *, nb=100, floor_eps=0.1, adapt_mask=0x3F):
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    lnw = np.ascontiguousarray(lnw, dtype=np.float64)
    n = lnw.size
    cdf = np.zeros((7, nb + 1))
    lib().or_adapt(C.c_int64(n), bins.ctypes.data_as(C.POINTER(C.c_uint8)), C.c_int64(bins.shape[1]),
                   _ptr(lnw), nb, C.c_double(floor_eps), C.c_uint(adapt_mask), _ptr(cdf))
    return cdf


def quv(data, psd, modes, df, f_low, row0, n_rows):
    """Q [K, n_rows, M], U, V [K, M, M] (complex) of Eq. (QUV) from
    frequency-domain data [K, N] (complex), one-sided PSD values S_k(|f_i|)
    [K, N] and modes [M, N] (complex), on the two-sided grid in FFT order."""
    data = np.ascontiguousarray(np.asarray(data, dtype=np.complex128))
    psd = np.ascontiguousarray(np.asarray(psd, dtype=np.float64))
    modes = np.ascontiguousarray(np.asarray(modes, dtype=np.complex128))
    K, N = data.shape
    M = modes.shape[0]
    Q = np.zeros((K, n_rows, M), dtype=np.complex128)
    U = np.zeros((K, M, M), dtype=np.complex128)
    V = np.zeros((K, M, M), dtype=np.complex128)
    lib().or_quv(K, M, C.c_int64(N), C.c_double(df), C.c_double(f_low), _ptr(data.view(np.float64)), _ptr(psd),
                 _ptr(modes.view(np.float64)), C.c_int64(row0), C.c_int64(n_rows), _ptr(Q.view(np.float64)),
                 _ptr(U.view(np.float64)), _ptr(V.view(np.float64)))
    return Q, U, V
