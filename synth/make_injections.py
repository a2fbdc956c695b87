"""Write ``synth/injections.npz``: for every synthetic point, the injected
signal's per-detector coefficients a_k = (D_ref/D) F_k Y_lm, its arrival
delays dt_k and the network SNR^2 of the unscaled U, all computed by the FP64
oracle (and nothing else).

    python synth/make_injections.py
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synth  # noqa: E402
from oracle import oracle  # noqa: E402


def injection_for(spec):
    th, gmst = synth.draw_injection(spec)
    U0, V = synth.make_U(spec)
    pos, resp, P = synth.geometry(spec)
    M = spec.n_modes
    ell = [lm[0] for lm in synth.MODE_SETS[M]]
    em = [lm[1] for lm in synth.MODE_SETS[M]]
    K = len(spec.dets)
    L = spec.n_t + 2 * P + 3
    p = oracle.Point(Q=np.zeros((K, L, M), np.complex128), U=U0, V=V, det_pos=pos, det_resp=resp,
                     ell=ell, em=em, n_t=spec.n_t, pad=P, f_s=spec.f_s, d_ref=spec.d_ref, gmst=gmst)
    a, B = oracle.coeffs(p, th)
    dt = np.array([oracle.delay(pos[k], th[0], th[1], gmst) for k in range(K)])
    # with V = 0, B = sum_k a^dag U a / 4 = rho^2 / 2; with V != 0 the same
    # quadratic term defines the SNR of the real signal
    rho2 = 2.0 * B
    return a, dt, rho2, synth._fingerprint(th, U0)


def main():
    specs = synth.all_specs()
    seen = {}
    for s in specs:
        if s.kernel == "none":
            continue
        seen.setdefault(s.key(), s)
    arrays = {"keys": np.array(list(seen.keys()))}
    rho2s, fps = [], []
    for i, (k, s) in enumerate(seen.items()):
        a, dt, rho2, fp = injection_for(s)
        arrays[f"a_{i}"] = a
        arrays[f"dt_{i}"] = dt
        rho2s.append(rho2)
        fps.append(fp)
    arrays["rho2"] = np.array(rho2s)
    arrays["fp"] = np.array(fps)
    np.savez_compressed(synth.INJECTION_FILE, **arrays)
    print(f"wrote {len(seen)} injections to {synth.INJECTION_FILE}")


if __name__ == "__main__":
    main()
